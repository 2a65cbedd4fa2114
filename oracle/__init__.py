"""FP64 CPU oracle of the Hermite block-step direct N-body scheme (Portegies Zwart, Belleman &
Geldof 2007, Sec. 2 and App. A).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the HIP library; its compiled part is
plain C built by gcc (``oracle/build.py``).

Array conventions: positions/velocities/accelerations/jerks are (n, 3) float64 arrays (AoS),
masses (n,), particle times are int64 ticks of 2**-lmax, levels are int32 with dt = 2**-level.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# NBODY_ORACLE_LIB lets the mutation test load a deliberately broken build of the same source.
_LIB_PATH = os.environ.get("NBODY_ORACLE_LIB") or os.path.join(_HERE, "_nbody_oracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "orc_force": (None, [_I64, _i64, _I64, _d, _d, _d, _D, _d, _d, _d]),
        "orc_force_scale": (None, [_I64, _i64, _I64, _d, _d, _d, _D, _d, _d]),
        "orc_energy": (None, [_I64, _d, _d, _d, _D, _d, _d]),
        "orc_predict": (None, [_I64, _d, _d, _d, _d, _i64, _I64, _D, _d, _d]),
        "orc_correct": (None, [_I64, _i64, _i32, _d, _d, _d, _d, _d, _d, _d, _d, _d, _d, _d]),
        "orc_aarseth_dt": (_D, [_D, _D, _D]),
        "orc_initial_dt": (_D, [_D, _d, _d]),
        "orc_level_from_dt": (_I32, [_D, _I32, _I32]),
        "orc_next_level": (_I32, [_D, _I32, _I64, _I32, _I32]),
        "orc_select_block": (_I64, [_I64, _i64, _i32, _I32, _i64, _i64]),
        "orc_init": (None, [_I64, _d, _d, _d, _D, _D, _I32, _I32, _d, _d, _d, _i64, _i32]),
        "orc_block_step": (_I64, [_I64, _d, _d, _d, _d, _d, _d, _i64, _i32, _D, _D, _I32, _I32,
                                  _i64, _i64, _d, _i64]),
        "orc_shared_step": (None, [_I64, _d, _d, _d, _d, _d, _d, _D, _D]),
        "orc_num_threads": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a, kind=_d):
    return a.ctypes.data_as(kind)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads():
    """Threads the oracle's parallel loops use (OpenMP)."""
    return int(_load().orc_num_threads())


def force(x, v, m, eps2, idx=None):
    """Acceleration, jerk and potential (Eq. Force, App. A) on the particles ``idx`` (all if
    None) from all others.  Returns (acc (n_i,3), jerk (n_i,3), pot (n_i,))."""
    lib = _load()
    x = _f64(x, (-1, 3)); v = _f64(v, (-1, 3)); m = _f64(m)
    n = x.shape[0]
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, np.int64)
    ni = idx.shape[0]
    acc = np.zeros((ni, 3)); jerk = np.zeros((ni, 3)); pot = np.zeros(ni)
    lib.orc_force(ni, _p(idx, _i64), n, _p(x), _p(v), _p(m), float(eps2), _p(acc), _p(jerk),
                  _p(pot))
    return acc, jerk, pot


def force_scale(x, v, m, eps2, idx=None):
    """Sum over j != i of the sizes of the terms of Eq. Force on the particles ``idx`` (all if
    None): (sa (n_i,), sk (n_i,)) with sa_i = sum_j m_j |d| s^-3/2 and
    sk_i = sum_j m_j (|u| s^-3/2 + 3 |d.u| |d| s^-5/2).  A sum of terms each rounded to a
    relative u is off by at most about u times this scale, however much the terms cancel."""
    lib = _load()
    x = _f64(x, (-1, 3)); v = _f64(v, (-1, 3)); m = _f64(m)
    n = x.shape[0]
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, np.int64)
    ni = idx.shape[0]
    sa = np.zeros(ni); sk = np.zeros(ni)
    lib.orc_force_scale(ni, _p(idx, _i64), n, _p(x), _p(v), _p(m), float(eps2), _p(sa), _p(sk))
    return sa, sk


def energy(x, v, m, eps2):
    """(kinetic, potential) energy, softened potential (Sec. 4.2 diagnostic)."""
    lib = _load()
    x = _f64(x, (-1, 3)); v = _f64(v, (-1, 3)); m = _f64(m)
    ek = ctypes.c_double(); ep = ctypes.c_double()
    lib.orc_energy(x.shape[0], _p(x), _p(v), _p(m), float(eps2), ctypes.byref(ek),
                   ctypes.byref(ep))
    return ek.value, ep.value


def predict(x, v, a, k, tick, t_target, lmax=26):
    """Sec. 2 predictor of every particle from its own time to ``t_target`` (ticks)."""
    lib = _load()
    x = _f64(x, (-1, 3)); v = _f64(v, (-1, 3)); a = _f64(a, (-1, 3)); k = _f64(k, (-1, 3))
    tick = np.ascontiguousarray(tick, np.int64)
    n = x.shape[0]
    xp = np.empty_like(x); vp = np.empty_like(v)
    lib.orc_predict(n, _p(x), _p(v), _p(a), _p(k), _p(tick, _i64), int(t_target),
                    float(np.ldexp(1.0, -lmax)), _p(xp), _p(vp))
    return xp, vp


def correct(idx, level, xp, vp, a1, k1, pot1, x, v, a, k, pot):
    """Sec. 2 corrector of the block ``idx`` in place on (x, v, a, k, pot).  Returns the
    time-step criterion inputs, (n_act, 2): |a1||a2p| + |k1|^2 and |k1||a3| + |a2p|^2."""
    lib = _load()
    idx = np.ascontiguousarray(idx, np.int64)
    level = np.ascontiguousarray(level, np.int32)
    na = idx.shape[0]
    crit = np.zeros((na, 2))
    for arr in (x, v, a, k, pot):
        assert arr.dtype == np.float64 and arr.flags.c_contiguous
    xp = _f64(xp, (-1, 3)); vp = _f64(vp, (-1, 3))
    a1 = _f64(a1, (-1, 3)); k1 = _f64(k1, (-1, 3)); pot1 = _f64(pot1)
    lib.orc_correct(na, _p(idx, _i64), _p(level, _i32), _p(xp), _p(vp), _p(a1), _p(k1),
                    _p(pot1), _p(x), _p(v), _p(a), _p(k), _p(pot), _p(crit))
    return crit


def aarseth_dt(nu, crit_num, crit_den):
    return _load().orc_aarseth_dt(float(nu), float(crit_num), float(crit_den))


def initial_dt(nu, a, k):
    a = _f64(a); k = _f64(k)
    return _load().orc_initial_dt(float(nu), _p(a), _p(k))


def level_from_dt(dt_raw, lmin, lmax=26):
    return int(_load().orc_level_from_dt(float(dt_raw), int(lmin), int(lmax)))


def next_level(dt_raw, l_old, t, lmin, lmax=26):
    return int(_load().orc_next_level(float(dt_raw), int(l_old), int(t), int(lmin), int(lmax)))


def select_block(tick, level, lmax=26):
    """Block selection of Sec. 2: returns (t_next, ascending index array of the block)."""
    lib = _load()
    tick = np.ascontiguousarray(tick, np.int64)
    level = np.ascontiguousarray(level, np.int32)
    idx = np.empty(tick.shape[0], np.int64)
    na = ctypes.c_int64()
    t_next = lib.orc_select_block(tick.shape[0], _p(tick, _i64), _p(level, _i32), int(lmax),
                                  _p(idx, _i64), ctypes.byref(na))
    return int(t_next), idx[: na.value].copy()


class BlockIntegrator:
    """Hermite block-step integration of Sec. 2 on FP64 state (oracle).

    ``lmin`` sets the largest step 2**-lmin, ``lmax`` the smallest 2**-lmax (also the tick).
    """

    def __init__(self, x, v, m, eps, nu, lmin=3, lmax=26):
        self.x = _f64(x, (-1, 3)).copy()
        self.v = _f64(v, (-1, 3)).copy()
        self.m = _f64(m).copy()
        self.n = self.x.shape[0]
        self.eps2 = float(eps) ** 2
        self.nu = float(nu)
        self.lmin, self.lmax = int(lmin), int(lmax)
        self.a = np.zeros((self.n, 3)); self.k = np.zeros((self.n, 3)); self.pot = np.zeros(self.n)
        self.tick = np.zeros(self.n, np.int64)
        self.level = np.zeros(self.n, np.int32)
        self.dt_raw = np.full(self.n, np.nan)
        self.t = 0
        self.n_steps = 0
        self.n_active_total = 0
        self.n_dtmin = 0
        self.last_block = np.zeros(0, np.int64)
        _load().orc_init(self.n, _p(self.x), _p(self.v), _p(self.m), self.eps2, self.nu,
                         self.lmin, self.lmax, _p(self.a), _p(self.k), _p(self.pot),
                         _p(self.tick, _i64), _p(self.level, _i32))

    @property
    def tick_len(self):
        return float(np.ldexp(1.0, -self.lmax))

    @property
    def time(self):
        return self.t * self.tick_len

    def step(self):
        """One block step; returns (t_next in ticks, the block's indices)."""
        idx = np.empty(self.n, np.int64)
        na = ctypes.c_int64()
        ndm = ctypes.c_int64(0)
        t_next = _load().orc_block_step(
            self.n, _p(self.x), _p(self.v), _p(self.a), _p(self.k), _p(self.m), _p(self.pot),
            _p(self.tick, _i64), _p(self.level, _i32), self.eps2, self.nu, self.lmin, self.lmax,
            _p(idx, _i64), ctypes.byref(na), _p(self.dt_raw), ctypes.byref(ndm))
        self.t = int(t_next)
        self.n_steps += 1
        self.n_active_total += na.value
        self.n_dtmin += ndm.value
        self.last_block = idx[: na.value].copy()
        return self.t, self.last_block

    def run_until(self, t_end, callback=None):
        """Step until the global time reaches ``t_end`` (time units, a multiple of the tick)."""
        t_end_ticks = int(round(t_end / self.tick_len))
        while self.t < t_end_ticks:
            self.step()
            if callback is not None:
                callback(self)
        return self

    def synchronised(self):
        return bool(np.all(self.tick == self.t))

    def energy(self):
        """Total energy; valid when every particle sits at the same time (synchronised)."""
        ek, ep = energy(self.x, self.v, self.m, self.eps2)
        return ek + ep


class SharedStepIntegrator:
    """Hermite integration with one fixed step for every particle (shared-step mode)."""

    def __init__(self, x, v, m, eps, dt):
        self.x = _f64(x, (-1, 3)).copy()
        self.v = _f64(v, (-1, 3)).copy()
        self.m = _f64(m).copy()
        self.n = self.x.shape[0]
        self.eps2 = float(eps) ** 2
        self.dt = float(dt)
        self.a, self.k, self.pot = force(self.x, self.v, self.m, self.eps2)
        self.time = 0.0

    def step(self, nsteps=1):
        lib = _load()
        for _ in range(int(nsteps)):
            lib.orc_shared_step(self.n, _p(self.x), _p(self.v), _p(self.a), _p(self.k),
                                _p(self.m), _p(self.pot), self.eps2, self.dt)
            self.time += self.dt
        return self

    def energy(self):
        ek, ep = energy(self.x, self.v, self.m, self.eps2)
        return ek + ep


# ------------------------------------------------------------------ derivatives of shared runs
def shared_run(x0, v0, m, eps, dt, nsteps):
    """Final (x, v) of `nsteps` shared Hermite steps of size dt (FP64)."""
    it = SharedStepIntegrator(x0, v0, m, eps, dt)
    it.step(nsteps)
    return it.x, it.v


def mean_sq_distance(x, target):
    """Trajectory loss: mean over particles of |x_i - target_i|^2."""
    return float(np.mean(np.sum((np.asarray(x) - np.asarray(target)) ** 2, axis=1)))


def fd_gradient(x0, v0, m, eps, dt, nsteps, target, coords, rel_h=1e-6, rel_h_mass=1e-3):
    """Central finite differences of mean_sq_distance(shared_run(...), target) with respect
    to the listed coordinates: ("x" | "v", particle, component) or ("m", particle, 0).
    Step h = rel_h * max(|value|, 1) for x and v; rel_h_mass * m_i for a mass (a mass changes
    the trajectory so little that a smaller step leaves the quotient at the rounding noise of
    the run)."""
    x0 = _f64(x0, (-1, 3)); v0 = _f64(v0, (-1, 3)); m = _f64(m)
    out = []
    for kind, i, c in coords:
        arrs = {"x": x0, "v": v0, "m": m}
        base = arrs[kind]
        val = base[i, c] if kind != "m" else base[i]
        h = rel_h * max(abs(val), 1.0) if kind != "m" else rel_h_mass * abs(val)
        vals = []
        for sgn in (1, -1):
            xx, vv, mm = x0.copy(), v0.copy(), m.copy()
            tgt = {"x": xx, "v": vv, "m": mm}[kind]
            if kind == "m":
                tgt[i] = val + sgn * h
            else:
                tgt[i, c] = val + sgn * h
            xf, _ = shared_run(xx, vv, mm, eps, dt, nsteps)
            vals.append(mean_sq_distance(xf, target))
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)
