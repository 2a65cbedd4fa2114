"""Seeded synthetic inputs: equal-mass Plummer spheres in N-body units.

This module draws random numbers and shapes them into initial conditions; it holds none of the
integration or force arithmetic.  Both the HIP path's tests and the oracle's tests take their
inputs from here.

Recipe (Sec. 4: Plummer model sampled by the method of Aarseth, Henon & Wielen 1974, equal
masses, N-body units):
  * cumulative-mass fraction X ~ U(0, 1), kept if X <= 0.999 (a radial cut, standard for this
    sampler), radius r = (X^(-2/3) - 1)^(-1/2) in units of the Plummer scale length;
  * isotropic direction for the position;
  * speed fraction q in [0, 1] by von Neumann rejection on g(q) = q^2 (1 - q^2)^(7/2) (the
    bound 0.1 exceeds max g), speed q * sqrt(2) * (1 + r^2)^(-1/4) (a fraction of the local
    escape speed), isotropic direction;
  * masses 1/N; centre of mass moved to rest at the origin;
  * scaled to standard N-body units (G = M = 1, E = -1/4): positions by 3*pi/16, velocities by
    sqrt(16 / (3*pi)).  A Plummer model so scaled is in virial equilibrium (2T = -W) in
    expectation; an individual realisation deviates by O(N^-1/2).

The generator is numpy's PCG64 seeded with the integer ``seed``.
"""
from __future__ import annotations

import math

import numpy as np

RADIAL_CUT = 0.999
LENGTH_SCALE = 3.0 * math.pi / 16.0


def _isotropic(rng, n):
    """Unit vectors uniform on the sphere."""
    z = 1.0 - 2.0 * rng.random(n)
    phi = 2.0 * math.pi * rng.random(n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def _mass_fractions(rng, n):
    out = np.empty(n)
    filled = 0
    while filled < n:
        x = rng.random(2 * (n - filled) + 16)
        x = x[(x > 0.0) & (x <= RADIAL_CUT)]
        take = min(x.size, n - filled)
        out[filled:filled + take] = x[:take]
        filled += take
    return out


def _speed_fractions(rng, n):
    out = np.empty(n)
    filled = 0
    while filled < n:
        m = 12 * (n - filled) + 64
        q = rng.random(m)
        y = 0.1 * rng.random(m)
        q = q[y < q * q * (1.0 - q * q) ** 3.5]
        take = min(q.size, n - filled)
        out[filled:filled + take] = q[:take]
        filled += take
    return out


def plummer(n: int, seed: int):
    """Return (x (n,3), v (n,3), m (n,)) float64 for an equal-mass Plummer sphere."""
    n = int(n)
    if n <= 0:
        return np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0)
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    xm = _mass_fractions(rng, n)
    r = 1.0 / np.sqrt(xm ** (-2.0 / 3.0) - 1.0)
    x = r[:, None] * _isotropic(rng, n)
    q = _speed_fractions(rng, n)
    speed = q * math.sqrt(2.0) * (1.0 + r * r) ** -0.25
    v = speed[:, None] * _isotropic(rng, n)
    m = np.full(n, 1.0 / n)
    x -= (m[:, None] * x).sum(axis=0) / m.sum()
    v -= (m[:, None] * v).sum(axis=0) / m.sum()
    x *= LENGTH_SCALE
    v /= math.sqrt(LENGTH_SCALE)
    return x, v, m


def ensemble_sizes(n_clusters: int, seed: int, lo: int = 64, hi: int = 4096):
    """Cluster sizes drawn log-uniform in [lo, hi] (rounded to integers)."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    u = rng.random(int(n_clusters))
    return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def perturb(x, v, sigma: float, seed: int):
    """Copies of x and v with independent N(0, sigma^2) noise added to every coordinate."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    return (np.asarray(x) + sigma * rng.standard_normal(np.shape(x)),
            np.asarray(v) + sigma * rng.standard_normal(np.shape(v)))


def sample_indices(n: int, count: int, seed: int):
    """``count`` distinct indices in [0, n), sorted (all of them when count >= n)."""
    if count >= n:
        return np.arange(n, dtype=np.int64)
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)
