"""Write tests/golden/accuracy_sweep.json: the energy-conservation experiment of Sec. Results
(accuracy measurements) run with the FP64 oracle.  For Plummer spheres of N = 1024 and 16384
(eps = 1/256, dt <= 1/8) and the accuracy parameter nu = 0.1 / 2^k, k = 0 .. 8, the block-step
integrator runs from t = 0 to t = 1/4, then on to t = 1/2; recorded are
|E(1/2) - E(1/4)| / |E(1/4)|, the block steps and the mean block size of the measured interval,
and how many step requests fell below 2^-26 and were clamped (whole run).
Calls only the oracle and the seeded input generator.

    python tests/golden/make_accuracy_reference.py [--only N]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_astro_ph_0702058_amd.plummer import plummer  # noqa: E402

SIZES = {1024: 1, 16384: 7}          # N -> seed of the initial conditions
NUS = [0.1 / 2 ** k for k in range(9)]
EPS, LMIN, T0, T1 = 1 / 256, 3, 0.25, 0.5


def sweep_one(n, seed, nu):
    x, v, m = plummer(n, seed)
    it = oracle.BlockIntegrator(x, v, m, eps=EPS, nu=nu, lmin=LMIN)
    t_a = time.time()
    it.run_until(T0)
    e0, s0, a0 = it.energy(), it.n_steps, it.n_active_total
    it.run_until(T1)
    e1 = it.energy()
    return dict(nu=nu, e_t0=e0, e_t1=e1, de_rel=abs((e1 - e0) / e0), n_steps=it.n_steps - s0,
                mean_block=(it.n_active_total - a0) / max(it.n_steps - s0, 1),
                n_dtmin=it.n_dtmin,
                seconds=time.time() - t_a)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", type=int)
    a = ap.parse_args()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "accuracy_sweep.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    out["params"] = dict(eps=EPS, lmin=LMIN, t0=T0, t1=T1, seeds={str(k): s for k, s in SIZES.items()})
    for n, seed in SIZES.items():
        if a.only and n != a.only:
            continue
        rows = []
        for nu in NUS:
            r = sweep_one(n, seed, nu)
            rows.append(r)
            print(n, f"nu={nu:.5g} dE/E={r['de_rel']:.3e} steps={r['n_steps']} "
                     f"{r['seconds']:.1f}s", flush=True)
        out[str(n)] = dict(seed=seed, threads=oracle.num_threads(), rows=rows)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
