"""Write tests/golden/plummer_runs.json: block-step runs of the FP64 oracle on the Plummer
workloads used by the GPU run tests (energy error, block-step count, mean block size, and the
positions of a few sampled particles at the end).  Calls only the oracle and the seeded input
generator.

    python tests/golden/make_plummer_reference.py [--only NAME]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_astro_ph_0702058_amd.plummer import plummer, sample_indices  # noqa: E402

RUNS = {
    # Plummer N = 1024, eps = 1/256, nu = 0.01, dt <= 1/64, to t = 1/8
    "n1024_t0.125": dict(n=1024, seed=1, eps=1 / 256, nu=0.01, lmin=6, t_end=0.125),
    # Plummer N = 65536, eps = 1e-3, nu = 0.01, dt <= 1/8, to t = 1
    "n65536_t1": dict(n=65536, seed=2, eps=1e-3, nu=0.01, lmin=3, t_end=1.0),
}


def run(name, p):
    x, v, m = plummer(p["n"], p["seed"])
    it = oracle.BlockIntegrator(x, v, m, eps=p["eps"], nu=p["nu"], lmin=p["lmin"])
    e0 = it.energy()
    t0 = time.time()
    it.run_until(p["t_end"])
    e1 = it.energy()
    idx = sample_indices(p["n"], 16, 99)
    return dict(params=p, energy0=e0, energy1=e1, de_rel=(e1 - e0) / e0, n_steps=it.n_steps,
                n_active_sum=it.n_active_total, mean_block=it.n_active_total / it.n_steps,
                n_dtmin=it.n_dtmin, sample_idx=idx.tolist(), x_sample=it.x[idx].tolist(),
                seconds=time.time() - t0, threads=oracle.num_threads())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only")
    a = ap.parse_args()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plummer_runs.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name, p in RUNS.items():
        if a.only and name != a.only:
            continue
        out[name] = run(name, p)
        print(name, {k: out[name][k] for k in ("de_rel", "n_steps", "mean_block", "seconds")},
              flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
