"""Write tests/golden/adjoint_fd.json: central finite differences of the FP64 oracle for the
differentiable shared-step workload at its full size, at 32 sampled coordinates.

Workload: Plummer N = 16384 (seed 5), eps = 1/128, 64 shared Hermite steps of dt = 1/1024.
Target: the final positions of the oracle's run from the same initial conditions with every
coordinate of x and v perturbed by N(0, 1e-3^2) (seed 6).  Loss: mean over particles of
|x_i(T) - target_i|^2.  Derivatives with respect to 12 initial position coordinates, 12 initial
velocity coordinates and 8 masses (seeded samples), steps as in oracle.fd_gradient.  With
--refine-masses the mass derivatives are evaluated again at half the step and the Richardson
value (4 D(h/2) - D(h)) / 3 is stored beside them: a mass is varied by a relative step of 1e-3,
so the central difference's own truncation error can matter for the smallest mass derivatives.
With --wide-masses they are evaluated at relative steps 1e-2 and 5e-3 with their Richardson
value (see wide_masses).
Calls only the oracle and the seeded input generator.

    python tests/golden/make_adjoint_reference.py [--refine-masses | --wide-masses]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_astro_ph_0702058_amd.plummer import perturb, plummer, sample_indices  # noqa: E402

N, SEED, EPS, DT, NSTEPS = 16384, 5, 1.0 / 128, 2.0 ** -10, 64


def coords():
    out = []
    for kind, count, seed in (("x", 12, 50), ("v", 12, 51), ("m", 8, 52)):
        for k, i in enumerate(sample_indices(N, count, seed)):
            out.append((kind, int(i), 0 if kind == "m" else k % 3))
    return out


def refine_masses(path):
    g = json.load(open(path))
    t0 = time.time()
    x0, v0, m = plummer(N, SEED)
    xp, vp = perturb(x0, v0, 1e-3, 6)
    target, _ = oracle.shared_run(xp, vp, m, EPS, DT, NSTEPS)
    cs = [tuple(c) for c in g["coords"]]
    sel = [k for k, c in enumerate(cs) if c[0] == "m"]
    half = oracle.fd_gradient(x0, v0, m, EPS, DT, NSTEPS, target, [cs[k] for k in sel],
                              rel_h_mass=0.5e-3)
    g["fd_half"] = [None] * len(cs)
    g["fd_richardson"] = [None] * len(cs)
    for k, d in zip(sel, half):
        g["fd_half"][k] = float(d)
        g["fd_richardson"][k] = (4.0 * float(d) - g["fd"][k]) / 3.0
    g["seconds_refine"] = time.time() - t0
    with open(path, "w") as f:
        json.dump(g, f, indent=1)
    print("refined", len(sel), "mass derivatives", g["seconds_refine"], flush=True)


def wide_masses(path):
    """Mass derivatives again at relative steps 1e-2 and 5e-3 and their Richardson value.  At
    the steps of 1e-3 and 5e-4 the two quotients of every sampled mass differ by 2-4e-13
    whatever the derivative's size (7e-8 .. 6e-7), the signature of the run's rounding noise
    divided by the step rather than of truncation error, which would scale with the derivative;
    ten times the step leaves a tenth of that noise, and the Richardson value removes the
    h^2 truncation term the larger step brings."""
    g = json.load(open(path))
    t0 = time.time()
    x0, v0, m = plummer(N, SEED)
    xp, vp = perturb(x0, v0, 1e-3, 6)
    target, _ = oracle.shared_run(xp, vp, m, EPS, DT, NSTEPS)
    cs = [tuple(c) for c in g["coords"]]
    sel = [k for k, c in enumerate(cs) if c[0] == "m"]
    d1 = oracle.fd_gradient(x0, v0, m, EPS, DT, NSTEPS, target, [cs[k] for k in sel],
                            rel_h_mass=1e-2)
    d2 = oracle.fd_gradient(x0, v0, m, EPS, DT, NSTEPS, target, [cs[k] for k in sel],
                            rel_h_mass=5e-3)
    g["fd_mass_wide"] = {"rel_steps": [1e-2, 5e-3], "coords": [list(cs[k]) for k in sel],
                         "d_h": [float(t) for t in d1], "d_h2": [float(t) for t in d2],
                         "richardson": [(4.0 * float(b) - float(a)) / 3.0 for a, b in zip(d1, d2)],
                         "seconds": time.time() - t0}
    with open(path, "w") as f:
        json.dump(g, f, indent=1)
    print("wide mass steps", len(sel), "derivatives", g["fd_mass_wide"]["seconds"], flush=True)


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_fd.json")
    if "--refine-masses" in sys.argv[1:]:
        return refine_masses(path)
    if "--wide-masses" in sys.argv[1:]:
        return wide_masses(path)
    t0 = time.time()
    x0, v0, m = plummer(N, SEED)
    xp, vp = perturb(x0, v0, 1e-3, 6)
    target, _ = oracle.shared_run(xp, vp, m, EPS, DT, NSTEPS)
    xf, _ = oracle.shared_run(x0, v0, m, EPS, DT, NSTEPS)
    loss = oracle.mean_sq_distance(xf, target)
    cs = coords()
    fd = oracle.fd_gradient(x0, v0, m, EPS, DT, NSTEPS, target, cs)
    out = dict(params=dict(n=N, seed=SEED, eps=EPS, dt=DT, nsteps=NSTEPS, target_seed=6,
                           target_sigma=1e-3),
               loss=loss, target_sum=float(np.sum(target)), coords=cs, fd=fd.tolist(),
               seconds=time.time() - t0, threads=oracle.num_threads())
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("loss", loss, "seconds", out["seconds"], flush=True)


if __name__ == "__main__":
    main()
