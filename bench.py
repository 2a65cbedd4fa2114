"""Benchmark: direct N-body force + Hermite block steps on one MI355X.

Workload (default): an equal-mass Plummer sphere of N = 2^20 particles in N-body units,
softening 1/256, eta = 0.01, largest step 1/8.  One bench step is the whole hot path once:
nb_init (full force of all N i-particles against all N j-particles, initial time steps, first
block selection) followed by 8 block steps (schedule, predict, block force, correct).  The
initial positions and velocities are restored (a device copy) at the start of every step so that
every step does the same work.

Output: one JSON line.  `value` is force interactions per second over the timed steps
(N^2 for the full force plus N times each block's size, the self slot counted as the paper's
operation count does); `roofline` reports the single-precision force kernel against the
MI355X FP32 vector peak at 60 flop per interaction; `cpu_baseline` is the FP64 CPU oracle
timed on a sample of i-particles of the same workload on this host.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X dense FP32 vector peak (published)
PEAK_FP64_TFLOPS = 78.6
FLOP_PER_INTERACTION = 60     # acc + jerk + potential, the paper's operation count
METRIC = "interactions/s (acc+jerk) & %FP32 VALU peak at N=2^20; FP32 vs double-single"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "ds_arith.hpp"):
        with open(os.path.join(ROOT, "paper_astro_ph_0702058_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel_sym, n, args, variant=None):
    """HBM bytes per launch of the full-force kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by its reading for a plain copy of known
    size), or None when the summary is for another workload or launch configuration, or the
    kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "force_full_fp32_plummer_n1048576_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel") != kernel_sym or t.get("n") != n or t.get("eps") != args.eps
            or t.get("kernel_source_sha256_16") != kernel_source_hash()
            or (variant is not None and t.get("variant") != variant)):
        return None
    return t.get("hbm_bytes_per_launch")


def rms_rel(got, ref):
    import numpy as np
    got, ref = np.asarray(got), np.asarray(ref)
    if got.ndim == 1:
        return float(np.sqrt(np.mean(((got - ref) / ref) ** 2)))
    return float(np.sqrt(np.mean(np.sum((got - ref) ** 2, 1) / np.sum(ref ** 2, 1))))


def bench_ensemble(args, emit=True):
    """Ensemble workload: every cluster integrated by its own block steps to t_end; one step of
    the bench = the whole run from the initial conditions (nb_ens_init + nb_ens_run)."""
    if args.gpus != 1:
        print("bench.py measures one GPU only (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_astro_ph_0702058_amd import nbody
    from paper_astro_ph_0702058_amd.plummer import ensemble_sizes, plummer
    sizes = ensemble_sizes(args.clusters, 4)
    eps = 1.0 / sizes
    parts = [plummer(int(nc), 1000 + c) for c, nc in enumerate(sizes)]
    x = np.concatenate([p[0] for p in parts]); v = np.concatenate([p[1] for p in parts])
    m = np.concatenate([p[2] for p in parts])
    st = nbody.DeviceState(x, v, m)
    x0, v0 = st.x.clone(), st.v.clone()
    ens = nbody.Ensemble(sizes, eps, lmin=3, precision=args.precision)
    ens.nb_ens_bind(st)
    if args.ens_local:
        lim, nst, wrk = (int(float(t)) for t in args.ens_local.split(","))
        ens.nb_ens_set_local(lim, nst, wrk)
    eta = 0.02
    layout = None
    if args.tune:
        from paper_astro_ph_0702058_amd.tuning import ensemble_autotune
        layout = ensemble_autotune(ens, st, x0, v0, eta)
        log(f"[bench] ensemble layout {layout}")
    lanes = None
    if args.ens_lanes == "probe":
        # untimed, like the tuner: a run to t = 1/4 picks the 4 clusters with the most block
        # steps for a lane of their own
        from paper_astro_ph_0702058_amd.tuning import ensemble_lanes
        t_p = time.perf_counter()
        lane = ensemble_lanes(ens, st, x0, v0, eta)
        lanes = {"lanes": int(lane.max()) + 1, "lane0_clusters": np.flatnonzero(lane == 0).tolist(),
                 "assignment": "the 4 clusters with the most block steps in a probe run to "
                               "t = 1/4 (untimed) in lane 0, the rest in lane 1",
                 "probe_s": time.perf_counter() - t_p}
        log(f"[bench] ensemble lanes: {lanes}")

    def step():
        st.x.copy_(x0); st.v.copy_(v0)
        ens.nb_ens_init(eta)
        ens.nb_ens_run(eta, args.t_end, steps_per_launch=args.ens_spl)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctl = ens.nb_ens_control()
    ek, ep = ens.nb_ens_energy()
    st.x.copy_(x0); st.v.copy_(v0)
    ens.nb_ens_init(eta)
    ek0, ep0 = ens.nb_ens_energy()
    ens.close()
    inter = sum(int(nc) * int(nc) + int(nc) * c.n_active_sum for nc, c in zip(sizes, ctl))
    elapsed = (t1 - t0) / args.steps
    de = np.abs((ek + ep) - (ek0 + ep0)) / np.abs(ek0 + ep0)
    result = {
        "metric": "interactions/s, batched ensemble", "value": inter / elapsed,
        "unit": "interactions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "ds": "f32x2", "fp64": "f64", "fp32all": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.clusters} Plummer clusters, N_c log-uniform [64, 4096] "
                               f"(total {int(sizes.sum())}), eps=1/N_c, eta=0.02, t -> {args.t_end}",
                   "clusters": args.clusters, "particles": int(sizes.sum()),
                   "local_blocks": args.ens_local or "default",
                   "interactions_per_run": inter, "layout": layout, "lanes": lanes,
                   "max_block_steps": max(c.n_steps for c in ctl),
                   "mean_block_steps": float(np.mean([c.n_steps for c in ctl])),
                   "dE_over_E_max": float(de.max()), "dE_over_E_median": float(np.median(de))},
        "roofline": {"bound": "alu", "achieved": round(60 * inter / elapsed / 1e12, 3),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(60 * inter / elapsed / 1e12 / PEAK_FP32_TFLOPS, 4),
                     "traffic": None,
                     "basis": "60 flop per interaction over the whole run's wall clock (all "
                              "kernels; the run is bound by the latency of its global steps)"},
    }
    if not args.no_cpu_baseline:
        # the oracle on the same clusters in index order, each for at most 2 s of its own block
        # steps (or to t_end), until the time budget is spent
        import oracle
        spent, inter_c, done_c, desc = 0.0, 0, 0, []
        for c, nc in enumerate(sizes):
            nc = int(nc)
            it = oracle.BlockIntegrator(parts[c][0], parts[c][1], parts[c][2], eps=1.0 / nc,
                                        nu=eta, lmin=3)
            t_a = time.perf_counter()
            while time.perf_counter() - t_a < 2.0 and it.time < args.t_end:
                it.step()
            spent += time.perf_counter() - t_a
            inter_c += nc * nc + nc * it.n_active_total
            done_c += 1
            desc.append(f"{nc}:{it.time:.3g}")
            if spent > args.cpu_seconds:
                break
        result["cpu_baseline"] = {
            "value": inter_c / spent, "unit": "interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"oracle on the first {done_c} clusters (N_c:time reached) "
                      f"{' '.join(desc)}, {spent:.1f} s"}
    if emit:
        print(json.dumps(result), flush=True)
    return result


RUNS = {
    # Plummer N = 1024, eps = 1/256, nu = 0.01, dt <= 1/64, to t = 1/8
    "n1024_t0.125": dict(n=1024, seed=1, eps=1 / 256, nu=0.01, lmin=6, t_end=0.125),
    # Plummer N = 65536, eps = 1e-3, nu = 0.01, dt <= 1/8, to t = 1
    "n65536_t1": dict(n=65536, seed=2, eps=1e-3, nu=0.01, lmin=3, t_end=1.0),
}


def bench_run(args, emit=True):
    """Block-step run workload: a Plummer sphere integrated from t = 0 to t_end by the
    device-resident loop (nb_init + nb_run, graph replay).  `value` = force interactions per
    second over the whole run (sum over block steps of N times the block size, plus the N^2 of
    the initial force), wall clock around nb_init + nb_run.  The block-step force kernel's
    launch time comes from an eager replay of the same run with timing events on (graph replay
    records no events); both replays must take the same number of block steps."""
    if args.gpus != 1:
        print("bench.py measures one GPU only (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_astro_ph_0702058_amd import nbody
    from paper_astro_ph_0702058_amd.plummer import plummer
    p = RUNS[args.run]
    n, eps, nu, lmin, t_end = p["n"], p["eps"], p["nu"], p["lmin"], p["t_end"]
    x0, v0, m = plummer(n, p["seed"])

    def one(prec, graph, profile=False, max_steps=0):
        st = nbody.DeviceState(x0, v0, m)
        ctx = nbody.Context(n, eps, lmin=lmin, lmax=26, precision=prec)
        ctx.nb_bind(st)
        if args.resident >= 0:
            ctx.nb_set_resident(args.resident)
        if profile:
            ctx.nb_profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.nb_init(nu)
        failed = None
        try:
            ctx.nb_run(nu, t_end, max_steps=max_steps, chunk=256, use_graph=graph)
            ctx.nb_sync()
            wall = time.perf_counter() - t0
            if ctx.nb_read_control().t_cur < int(round(t_end * 2 ** 26)):
                failed = f"stopped at the limit of {max_steps} block steps"
        except nbody.NBodyError as err:
            # e.g. an arithmetic whose rounding noise drives the step criterion to the 2^-26
            # floor (NB_EDTMIN)
            failed = str(err)
        if failed:  # reported with how far the run got
            wall = time.perf_counter() - t0
            info = {}
            try:
                c = ctx.nb_read_control(check=False)
                info = dict(t_reached=c.t_cur * 2.0 ** -26, n_steps=c.n_steps,
                            mean_block=c.n_active_sum / max(c.n_steps, 1))
            except nbody.NBodyError:
                pass
            ctx.close()
            return dict(failed=failed, wall=wall, **info)
        c = ctx.nb_read_control()
        ek1, ep1 = ctx.nb_energy()
        prof = ctx.nb_profile_read(1) if profile else None
        ctx.close()
        return dict(wall=wall, n_steps=c.n_steps, n_active_sum=c.n_active_sum,
                    e1=ek1 + ep1, prof=prof)

    # E0 from the same energy routine, before the run
    st = nbody.DeviceState(x0, v0, m)
    with nbody.Context(n, eps, lmin=lmin, lmax=26, precision="fp64") as ctx:
        ctx.nb_bind(st)
        ctx.nb_init(nu)
        ek0, ep0 = ctx.nb_energy()
    e0 = ek0 + ep0
    for _ in range(args.warmup):
        one(args.precision, True)
    runs = [one(args.precision, True) for _ in range(max(1, args.steps))]
    if "failed" in runs[0]:
        raise RuntimeError(f"{args.run} {args.precision}: {runs[0]}")
    wall = min(r["wall"] for r in runs)
    r = runs[0]
    inter = n * n + n * r["n_active_sum"]
    log(f"[bench] {args.run} {args.precision}: {r['n_steps']} block steps, mean block "
        f"{r['n_active_sum'] / r['n_steps']:.1f}, {wall:.3f} s")
    eager = one(args.precision, False, profile=True)
    # the timing replay takes the launch chain; a small context's run takes the resident
    # workgroup (nb_set_resident), whose summation order differs: the same steps in FP64 and
    # double-single, within rounding-decided levels in FP32
    assert abs(eager["n_steps"] - r["n_steps"]) <= 0.02 * r["n_steps"], (eager["n_steps"], r["n_steps"])
    ms, launches = eager["prof"]
    per_launch = n * r["n_active_sum"] / launches
    peak = PEAK_FP64_TFLOPS if args.precision == "fp64" else PEAK_FP32_TFLOPS
    tflops = FLOP_PER_INTERACTION * per_launch / (ms / launches * 1e-3) / 1e12
    result = {
        "metric": "interactions/s over a block-step run (force interactions incl. the initial "
                  "full force / wall clock)",
        "value": inter / wall, "unit": "interactions/s", "n_gpus": 1, "steps": len(runs),
        "warmup": args.warmup, "ms_per_step": 1e3 * wall, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "ds": "f32x2", "fp64": "f64", "fp32all": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"Plummer N={n} (eps={eps:g}, eta={nu}, dt_max=2^-{lmin}) "
                               f"block-step run t=0 -> {t_end}", "n": n, "eps": eps, "eta": nu,
                   "lmin": lmin, "t_end": t_end, "precision": args.precision,
                   "n_steps": r["n_steps"], "mean_block": r["n_active_sum"] / r["n_steps"],
                   "de_rel": (r["e1"] - e0) / e0, "wall_s": wall},
        "roofline": {"bound": "alu", "kernel": "force_kernel (block-step launch class)",
                     "achieved": round(tflops, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(tflops / peak, 4), "traffic": None, "launches": launches,
                     "avg_launch_ms": round(ms / launches, 4),
                     "interactions_per_launch": per_launch,
                     "flop_per_interaction": FLOP_PER_INTERACTION,
                     "source": "eager replay of the same run with timing events (launch chain)"},
    }
    gold = os.path.join(ROOT, "tests", "golden", "plummer_runs.json")
    g_run = json.load(open(gold)).get(args.run) if os.path.exists(gold) else None
    variants = {}
    for prec in [q for q in args.variants.split(",") if q and q != "none" and q != args.precision]:
        # a run whose blocks fragment is stopped at 4 times the oracle run's block steps
        vr = one(prec, True, max_steps=4 * g_run["n_steps"] if g_run else 0)
        if "failed" in vr:
            variants[prec] = {k: vr[k] for k in ("failed", "t_reached", "n_steps", "mean_block")
                              if k in vr}
            variants[prec]["wall_s"] = vr["wall"]
            log(f"[bench] {prec}: stopped, {variants[prec]}")
            continue
        variants[prec] = {"wall_s": vr["wall"], "n_steps": vr["n_steps"],
                          "mean_block": vr["n_active_sum"] / vr["n_steps"],
                          "de_rel": (vr["e1"] - e0) / e0}
        log(f"[bench] {prec}: {vr['n_steps']} steps, {vr['wall']:.3f} s, dE/E {variants[prec]['de_rel']:.3e}")
    result["variants"] = variants
    if g_run:
        result["oracle_reference_run"] = {
            "de_rel": g_run["de_rel"], "n_steps": g_run["n_steps"],
            "mean_block": g_run["mean_block"], "seconds": g_run["seconds"],
            "threads": g_run["threads"],
            "note": "committed FP64 oracle run of the same initial conditions"}
    if not args.no_cpu_baseline:
        import oracle
        t_a = time.perf_counter()  # the oracle's init (the N^2 force) is part of the sample
        it = oracle.BlockIntegrator(x0, v0, m, eps=eps, nu=nu, lmin=lmin)
        while time.perf_counter() - t_a < args.cpu_seconds and it.time < t_end:
            it.step()
        el = time.perf_counter() - t_a
        result["cpu_baseline"] = {
            "value": (n * n + n * it.n_active_total) / el, "unit": "interactions/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"oracle init + its first {it.n_steps} block steps of the same run "
                      f"(t = 0 -> {it.time:.4g}), {el:.1f} s"}
    if emit:
        print(json.dumps(result), flush=True)
    return result


def bench_accuracy(args):
    """Energy conservation against the accuracy parameter (Sec. Results, accuracy
    measurements): Plummer N = 1024 (seed 1) and 16384 (seed 7), eps = 1/256, dt <= 1/8,
    nu = 0.1 / 2^k for k = 0 .. 8; each run goes from t = 0 to 1/4 and on to 1/2 and reports
    |E(1/2) - E(1/4)| / |E(1/4)| for the four interaction arithmetics (all-single as in the
    paper's kernel, FP32 with double separations, double-single, FP64).  E comes from the FP64
    energy diagnostic; E' = kinetic + (1/2) sum_i m_i phi_i uses the force kernel's own
    potentials instead (at t = 1/4 and 1/2 every particle has just been evaluated), which is
    how an energy check reads when the potential comes from the force pass (taken at the
    predicted positions, and in the paper's kernel from single-precision sums).  A run whose
    block steps exceed 4 times the oracle's count at that nu (over t = 0 .. 1/2) is stopped and
    marked collapsed: rounding noise in a and k, divided by dt^2 and dt^3 in the corrector's
    derivative estimates, drives the step criterion down towards the 2^-26 floor.  `value` = force interactions per
    second over all the runs; the committed oracle curves are attached."""
    if args.gpus != 1:
        print("bench.py measures one GPU only (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_astro_ph_0702058_amd import nbody
    from paper_astro_ph_0702058_amd.plummer import plummer
    sizes = {1024: 1, 16384: 7}
    nus = [0.1 / 2 ** k for k in range(9)]
    precs = ["fp32all", "fp32", "ds", "fp64"]
    gold = os.path.join(ROOT, "tests", "golden", "accuracy_sweep.json")
    g = json.load(open(gold)) if os.path.exists(gold) else {}
    curves, inter, wall = {}, 0.0, 0.0
    for n, seed in sizes.items():
        x, v, m = plummer(n, seed)
        ref_steps = {round(r["nu"], 12): r["n_steps"] for r in g.get(str(n), {}).get("rows", [])}
        for prec in precs:
            rows = []
            for nu in nus:
                budget = 4 * 2 * ref_steps.get(round(nu, 12), 20000)   # both halves
                st = nbody.DeviceState(x, v, m)
                with nbody.Context(n, 1 / 256, lmin=3, lmax=26, precision=prec,
                                   allow_dtmin=True) as ctx:
                    ctx.nb_bind(st)
                    torch.cuda.synchronize()
                    t_a = time.perf_counter()
                    ctx.nb_init(nu)
                    ctx.nb_run(nu, 0.25, max_steps=budget, chunk=256)
                    ek, ep = ctx.nb_energy()
                    c0 = ctx.nb_read_control()
                    mp0 = float((st.m * st.pot).sum()) / 2
                    ok = c0.t_cur == 1 << 24
                    if ok:
                        ctx.nb_run(nu, 0.5, max_steps=budget - c0.n_steps, chunk=256)
                    ek1, ep1 = ctx.nb_energy()
                    c1 = ctx.nb_read_control()
                    mp1 = float((st.m * st.pot).sum()) / 2
                    ok = ok and c1.t_cur == 1 << 25
                    el = time.perf_counter() - t_a
                e0, e1 = ek + ep, ek1 + ep1
                steps = c1.n_steps - c0.n_steps
                row = {"nu": nu, "collapsed": not ok, "dtmin_clamped": ctx.dtmin_clamped,
                       "t_reached": c1.t_cur / 2.0 ** 26, "seconds": el}
                if ok:
                    row.update({"steps_vs_oracle": steps / ref_steps.get(round(nu, 12), steps),
                                "de_rel": abs((e1 - e0) / e0),
                                "de_rel_kernel_pot": abs((ek1 + mp1 - ek - mp0) / (ek + mp0)),
                                "n_steps": steps,
                                "mean_block": (c1.n_active_sum - c0.n_active_sum) / max(steps, 1)})
                rows.append(row)
                inter += n * n + n * c1.n_active_sum
                wall += el
                log(f"[bench] N={n} {prec} nu={nu:.5g}: " + (
                    f"dE/E {row['de_rel']:.2e} (kernel phi {row['de_rel_kernel_pot']:.2e}), "
                    f"{steps} steps, {el:.2f} s" if ok else
                    f"collapsed at t={row['t_reached']:.6f} after {c1.n_steps} steps, {el:.2f} s"))
            curves[f"{n}/{prec}"] = rows
    result = {
        "metric": "|dE/E| over t = 1/4 .. 1/2 against nu (energy conservation experiment); value = "
                  "force interactions/s over all runs",
        "value": inter / wall, "unit": "interactions/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * wall, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32,f32,f32x2,f64", "data": "synthetic",
        "config": {"workload": "Plummer N=1024 (seed 1) and N=16384 (seed 7), eps=1/256, "
                               "dt_max=1/8, nu=0.1/2^k (k=0..8), t=0 -> 1/4 -> 1/2",
                   "precisions": precs},
        "curves": curves,
    }
    if g:
        result["oracle_curves"] = {k: [{"nu": r["nu"], "de_rel": r["de_rel"],
                                        "n_steps": r["n_steps"]} for r in g[k]["rows"]]
                                   for k in g if k != "params"}
    print(json.dumps(result), flush=True)


# Wall-clock seconds over t = 1/4 .. 1/2 printed in the paper's results table (Sec. Results):
# GRAPE-6Af, GeForce 8800GTX, Quadro FX1400, Xeon host; None where not measured.
PAPER_TIMED_RUNS = {
    256: (0.07098, 2.708, 3.423, 0.1325), 512: (0.1410, 8.777, 10.59, 0.5941),
    1024: (0.3327, 17.46, 20.20, 2.584), 2048: (0.7652, 45.27, 54.16, 10.59),
    4096: (1.991, 128.3, 157.8, 50.40), 8192: (5.552, 342.7, 617.3, 224.7),
    16384: (16.32, 924.4, 3398, 994.0), 32768: (51.68, 1907, 13180, 4328),
    65536: (178.2, 3973, 40560, 19290), 131072: (None, 8844, None, None),
    262144: (None, 22330, None, None), 524288: (None, 63960, None, None),
}


def bench_timed(args):
    """The timed runs of the paper's results table: Plummer spheres of N = 256 .. 2^19 (seed
    100 + log2 N), eps = 1/256, nu = 0.01, dt in [2^-26, 1/8], integrated from t = 0 to 1/2 by
    the device-resident loop and timed over t = 1/4 .. 1/2.  Reported per N: wall seconds,
    block steps and mean block size over the window, with the paper's fits n_block = a N^b and
    n_steps = c N^d refitted, and the block-step time fitted to
    t_step = tau_0 + tau_pred N + tau_corr n_block + tau_fe N n_block (non-negative least
    squares over all N; the paper's model with the host and bus terms replaced by device work).
    `value` = force interactions per second over the window at the largest N."""
    if args.gpus != 1:
        print("bench.py measures one GPU only (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from scipy.optimize import nnls
    from paper_astro_ph_0702058_amd import nbody
    from paper_astro_ph_0702058_amd.plummer import plummer
    ns = [n for n in sorted(PAPER_TIMED_RUNS) if n <= args.max_n]
    n = 2 * ns[-1]
    while n <= args.max_n:      # beyond the paper's largest N
        ns.append(n)
        n *= 2
    eps, nu, lmin = 1 / 256, 0.01, 3
    rows = []
    for n in ns:
        x, v, m = plummer(n, 100 + int(math.log2(n)))
        st = nbody.DeviceState(x, v, m)
        with nbody.Context(n, eps, lmin=lmin, lmax=26, precision=args.precision) as ctx:
            ctx.nb_bind(st)
            if args.resident >= 0:
                ctx.nb_set_resident(args.resident)
            ctx.nb_init(nu)
            ctx.nb_run(nu, 0.25, chunk=256)
            c0 = ctx.nb_read_control()
            torch.cuda.synchronize()
            t_a = time.perf_counter()
            ctx.nb_run(nu, 0.5, chunk=256)
            ctx.nb_sync()
            wall = time.perf_counter() - t_a
            c1 = ctx.nb_read_control()
        steps = c1.n_steps - c0.n_steps
        act = c1.n_active_sum - c0.n_active_sum
        paper = PAPER_TIMED_RUNS.get(n, (None,) * 4)
        rows.append({"n": n, "seconds": wall, "n_steps": steps, "mean_block": act / steps,
                     "interactions_per_s": n * act / wall, "us_per_step": 1e6 * wall / steps,
                     "paper_s": {"grape6af": paper[0], "gf8800gtx": paper[1], "fx1400": paper[2],
                                 "xeon": paper[3]}})
        log(f"[bench] N={n}: {wall:.3f} s over the window, {steps} steps, mean block "
            f"{act / steps:.1f}, {n * act / wall:.3e} interactions/s")
    big = [r for r in rows if r["n"] >= 1024]
    lb = np.polyfit(np.log([r["n"] for r in big]), np.log([r["mean_block"] for r in big]), 1)
    ls = np.polyfit(np.log([r["n"] for r in big]), np.log([4 * r["n_steps"] for r in big]), 1)
    A = np.array([[r["n_steps"], r["n_steps"] * r["n"], r["n_steps"] * r["mean_block"],
                   r["n_steps"] * r["mean_block"] * r["n"]] for r in rows])
    tau, _ = nnls(A / np.array([r["seconds"] for r in rows])[:, None], np.ones(len(rows)))
    last = rows[-1]
    result = {
        "metric": "wall seconds over t = 1/4 .. 1/2 per N (the paper's timed runs); value = force "
                  "interactions/s over the window at the largest N",
        "value": last["interactions_per_s"], "unit": "interactions/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": 1e3 * last["seconds"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "ds": "f32x2", "fp64": "f64", "fp32all": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"Plummer N=256..{ns[-1]} (seed 100+log2 N), eps=1/256, eta=0.01, "
                               "dt_max=1/8, run t=0 -> 1/2, timed t=1/4 -> 1/2",
                   "precision": args.precision},
        "rows": rows,
        "fits": {"n_block": {"a": float(np.exp(lb[1])), "b": float(lb[0]),
                             "paper": {"a": 0.20, "b": 0.81}},
                 "n_steps_per_time_unit": {"c": float(np.exp(ls[1])), "d": float(ls[0]),
                                           "paper": {"c": 247, "d": 0.35}},
                 "t_step_s": {"tau_0": tau[0], "tau_pred_per_particle": tau[1],
                              "tau_corr_per_block_member": tau[2],
                              "tau_fe_per_interaction": tau[3],
                              "paper_gf8800gtx": {"t_host_per_particle": 3.82e-7,
                                                  "tau_fe_per_interaction": 8.15e-10,
                                                  "send_per_particle": 1.76e-5,
                                                  "receive_per_particle": 5.97e-6}}},
    }
    if not args.no_cpu_baseline:
        import oracle
        spent, best = 0.0, None
        for n in ns:
            x, v, m = plummer(n, 100 + int(math.log2(n)))
            it = oracle.BlockIntegrator(x, v, m, eps=eps, nu=nu, lmin=lmin)
            t_a = time.perf_counter()
            it.run_until(0.25)
            s0, a0 = it.n_steps, it.n_active_total
            t_b = time.perf_counter()
            it.run_until(0.5)
            t_c = time.perf_counter()
            spent += t_c - t_a
            best = (n, t_c - t_b, it.n_active_total - a0)
            if spent * 4 > args.cpu_seconds:   # the next N costs about 4x more
                break
        n, el, act = best
        result["cpu_baseline"] = {
            "value": n * act / el, "unit": "interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"oracle timed over t = 1/4 .. 1/2 at N = {n}: {el:.2f} s (GPU: "
                      f"{next(r['seconds'] for r in rows if r['n'] == n):.3f} s)"}
    print(json.dumps(result), flush=True)


def bench_adjoint(args, emit=True):
    """Differentiable run: Plummer N = 16384, eps = 1/128, 64 shared steps of 1/1024, FP32
    force; loss = mean squared distance of the final positions to a target (the end of a run
    from initial conditions perturbed by N(0, 1e-3^2)); gradient with respect to x0, v0, m
    through the hand-written adjoint with checkpoints every 8 steps.  One bench step = forward
    + backward."""
    if args.gpus != 1:
        print("bench.py measures one GPU only (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_astro_ph_0702058_amd.adjoint import HermiteRun, SharedRunner
    from paper_astro_ph_0702058_amd.plummer import perturb, plummer
    n, eps, dt, nsteps, ce = 16384, 1.0 / 128, 2.0 ** -10, 64, 8
    prec = args.precision if args.precision != "ds" else "fp32"
    x0, v0, m = plummer(n, 5)
    xp_, vp_ = perturb(x0, v0, 1e-3, 6)
    soa = lambda a: torch.tensor(np.ascontiguousarray(np.asarray(a).T), dtype=torch.float64,
                                 device="cuda")
    runner = SharedRunner(n, eps, dt, nsteps, checkpoint_every=ce, precision=prec,
                          overlap=args.adj_overlap == "on")
    with torch.no_grad():  # target: the perturbed run, on the same engine
        tx, _ = HermiteRun.apply(soa(xp_), soa(vp_), torch.tensor(m, device="cuda"), runner)
        target = tx.clone()

    def step():
        X0 = soa(x0).requires_grad_(True); V0 = soa(v0).requires_grad_(True)
        M = torch.tensor(m, dtype=torch.float64, device="cuda").requires_grad_(True)
        x, _ = HermiteRun.apply(X0, V0, M, runner)
        loss = ((x - target) ** 2).sum(0).mean()
        loss.backward()
        return loss.detach(), X0.grad, V0.grad, M.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss, gx, gv, gm = step()
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / args.steps
    nseg = nsteps // ce
    forces = (nsteps + 1) + nseg * (ce - 1)    # forward + recomputation
    vjps = nsteps + 1
    result = {
        "metric": "gradient of a 64-step trajectory loss: interactions/s (forces + force VJPs)",
        "value": (forces + vjps) * n * n / elapsed, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64"}[prec], "data": "synthetic",
        "config": {"workload": "Plummer N=16384, eps=1/128, 64 shared steps dt=1/1024, "
                               "checkpoints every 8, loss = mean |x - x_target|^2",
                   "n": n, "force_evaluations": forces, "force_vjps": vjps,
                   "loss": float(loss), "grad_norms": {"x0": float(gx.norm()),
                                                       "v0": float(gv.norm()),
                                                       "m": float(gm.norm())}},
    }
    if not args.no_cpu_baseline:
        # the oracle's forward shared steps of the same run (the FP64 reference has no
        # hand-written adjoint; its gradient checks use finite differences of this forward)
        import oracle
        t_a = time.perf_counter()
        it = oracle.SharedStepIntegrator(x0, v0, m, eps, dt)
        steps = 0
        while time.perf_counter() - t_a < args.cpu_seconds and steps < nsteps:
            it.step(1)
            steps += 1
        el = time.perf_counter() - t_a
        result["cpu_baseline"] = {
            "value": (steps + 1) * n * n / el, "unit": "interactions/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"oracle forward of the same run: initial force + {steps} shared steps, "
                      f"{el:.1f} s (forward only)"}
    if emit:
        print(json.dumps(result), flush=True)
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--block-steps", type=int, default=8)
    ap.add_argument("--eta", type=float, default=0.01)
    ap.add_argument("--eps", type=float, default=1.0 / 256)
    ap.add_argument("--lmin", type=int, default=3)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "ds", "fp64", "fp32all"])
    ap.add_argument("--variants", default="ds,fp64,fp32fixed,fp32all",
                    help="other interaction arithmetics to time once (comma list, or 'none')")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--error-rows", type=int, default=65536,
                    help="rows of the N^2 force checked against the oracle (stratified)")
    ap.add_argument("--oracle-cache", default="~/.cache/libnbody",
                    help="directory of cached oracle reference rows, keyed by a hash of the "
                         "input and rows ('' to disable); the timed quarter is always "
                         "recomputed and must equal the stored rows")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the one-run summaries of the other workloads in the default line")
    ap.add_argument("--workload", default="full", choices=["full", "ensemble", "adjoint", "run", "accuracy", "timed"],
                    help="full: N-body force + block steps at N (default); ensemble: 512 "
                         "Plummer clusters, N_c log-uniform in [64, 4096], eps = 1/N_c, "
                         "eta = 0.02, to t = 1; adjoint: gradient of a trajectory loss over "
                         "64 shared steps at N = 16384; run: a block-step run (--run); "
                         "accuracy: energy error against nu for every arithmetic; timed: the "
                         "paper's timed runs over N")
    ap.add_argument("--max-n", type=int, default=1 << 19)
    ap.add_argument("--run", default="n65536_t1", choices=sorted(RUNS))
    ap.add_argument("--resident", type=int, default=-1,
                    help="nb_set_resident for the run and timed workloads (default: the "
                         "library's; 0: always the launch chain)")
    ap.add_argument("--clusters", type=int, default=512)
    ap.add_argument("--adj-overlap", default="on", choices=["on", "off"],
                    help="adjoint: recompute the next checkpoint segment on a second stream "
                         "while the current segment's step VJPs run (default on)")
    ap.add_argument("--ens-lanes", default="probe", choices=["probe", "one"],
                    help="ensemble: two independent lanes chosen by an untimed probe run "
                         "(default), or one lane")
    ap.add_argument("--ens-spl", type=int, default=128,
                    help="ensemble: global steps per graph replay (one host check per replay)")
    ap.add_argument("--ens-local", default="",
                    help="ensemble local blocks: LIMIT,STEPS,WORK (nb_ens_set_local; default: "
                         "the library's)")
    ap.add_argument("--t-end", type=float, default=1.0)
    ap.add_argument("--tune", action="store_true",
                    help="autotune the force-kernel variants first (untimed); default: the "
                         "library's defaults, which are the tuned choices for MI355X")
    args = ap.parse_args()

    if args.workload == "ensemble":
        return bench_ensemble(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "run":
        return bench_run(args)
    if args.workload == "accuracy":
        return bench_accuracy(args)
    if args.workload == "timed":
        return bench_timed(args)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_astro_ph_0702058_amd import nbody
    from paper_astro_ph_0702058_amd.plummer import plummer, sample_indices

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = args.n
    log(f"[bench] generating Plummer N={n} seed={args.seed}")
    x, v, m = plummer(n, args.seed)
    st = nbody.DeviceState(x, v, m)
    x0, v0 = st.x.clone(), st.v.clone()
    stream = torch.cuda.current_stream()

    ctx = nbody.Context(n, args.eps, lmin=args.lmin, lmax=26, precision=args.precision)
    ctx.nb_bind(st)

    if args.tune:
        import torch as _t
        ctx.nb_predict(_t.zeros(1, dtype=_t.int64, device="cuda"))
        from paper_astro_ph_0702058_amd.tuning import autotune
        t_tune = time.perf_counter()
        chosen = autotune(ctx, cache_path=None, reps=1)
        log(f"[bench] tuned in {time.perf_counter() - t_tune:.1f} s: {chosen}")
    variant_full, variant_block = ctx.nb_get_variant(0), ctx.nb_get_variant(1)

    def step():
        st.x.copy_(x0)
        st.v.copy_(v0)
        ctx.nb_init(args.eta)
        ctx.nb_step(args.eta, args.block_steps, use_graph=False)

    log(f"[bench] warmup {args.warmup} step(s)")
    for _ in range(args.warmup):
        step()
    ctx.nb_sync()
    # the device's FP32 FMA rate from the library's calibration kernel (warm clocks, untimed)
    fma_tflops = ctx.nb_fma_rate()
    log(f"[bench] measured FP32 FMA rate {fma_tflops:.1f} TFLOP/s")

    interactions = 0
    ctx.nb_profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c = ctx.nb_read_control()
    force_ms, launches = ctx.nb_profile_read(-1)
    # interactions: per step N^2 (initial full force) + N * (block sizes); the block sizes of
    # every timed step are identical (same initial state), read from the last one
    per_step = n * n + n * c.n_active_sum
    interactions = per_step * args.steps
    elapsed = t1 - t0
    value = interactions / elapsed
    log(f"[bench] {args.steps} steps in {elapsed:.3f} s; block steps sum n_act={c.n_active_sum}"
        f" ({c.n_active_sum / max(c.n_steps, 1):.0f} per block)")

    # roofline of the dominant kernel: the full-force launches (one per step, N^2 interactions)
    full_ms, full_n = ctx.nb_profile_read(0)
    blk_ms, blk_n = ctx.nb_profile_read(1)
    avg_full_ms = full_ms / max(full_n, 1)
    achieved = FLOP_PER_INTERACTION * n * n / (avg_full_ms * 1e-3) / 1e12
    kernel_sym = "force_kernel<ModeF32, %d, %d, true, 0>" % (variant_full["ipl"], variant_full["unroll"])
    traffic = committed_traffic(kernel_sym, n, args, variant_full)
    roofline = {"bound": "alu", "kernel": kernel_sym, "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "measured_fma_peak": round(fma_tflops, 2),
                "frac_of_measured_fma_peak": round(achieved / fma_tflops, 4),
                "launches": full_n, "avg_launch_ms": round(avg_full_ms, 3),
                "flop_per_interaction": FLOP_PER_INTERACTION,
                "interactions_per_launch": n * n,
                "block_step_launches": {"launches": blk_n,
                                        "avg_launch_ms": round(blk_ms / max(blk_n, 1), 4),
                                        "interactions": n * c.n_active_sum * args.steps,
                                        "tflops": round(FLOP_PER_INTERACTION * n * c.n_active_sum
                                                        * args.steps / max(blk_ms * 1e-3, 1e-12)
                                                        / 1e12, 3)}}
    if args.precision != "fp32":
        roofline["peak"] = PEAK_FP64_TFLOPS if args.precision == "fp64" else PEAK_FP32_TFLOPS
        roofline["frac"] = round(achieved / roofline["peak"], 4)
        roofline["kernel"] = kernel_sym.replace("ModeF32", {"ds": "ModeDS", "fp64": "ModeF64"}[args.precision])

    ctx.nb_profile(False)
    # accuracy of the timed arithmetic on a sample of i, against the oracle (untimed)
    st.x.copy_(x0); st.v.copy_(v0)
    ctx.nb_init(args.eta)
    ctx.nb_sync()
    g = st.numpy()
    ctx.close()

    result = {
        "metric": METRIC, "value": value, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"fp32": "f32", "ds": "f32x2",
                                                           "fp64": "f64", "fp32all": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"Plummer N={n} (eps={args.eps:g}, eta={args.eta:g}, "
                               f"dt_max=2^-{args.lmin}): full force + {args.block_steps} "
                               "block steps",
                   "n": n, "eps": args.eps, "eta": args.eta, "block_steps": args.block_steps,
                   "precision": args.precision, "interactions_per_step": per_step,
                   "variant_full_force": variant_full, "variant_block_steps": variant_block},
        "roofline": roofline,
        "context": {"paper_8800gtx_interactions_per_s": 1.23e9,
                    "paper_grape6af_interactions_per_s": 2.16e9},
    }

    # other interaction arithmetics: one full force each, timed with the same events
    variants = {}
    for prec in [p for p in args.variants.split(",") if p and p != "none"]:
        if prec == args.precision:
            continue
        st.x.copy_(x0); st.v.copy_(v0)
        cv = nbody.Context(n, args.eps, lmin=args.lmin, precision=prec)
        cv.nb_bind(st)
        cv.nb_profile(True)
        cv.nb_init(args.eta)
        ms, nl = cv.nb_profile_read(0)
        cv.nb_sync()
        gv = st.numpy()
        cv.close()
        rate = n * n / (ms * 1e-3)
        variants[prec] = {"interactions_per_s": rate, "full_force_ms": ms, "gv": gv}
        log(f"[bench] {prec}: full force {ms:.1f} ms, {rate:.3e} interactions/s")

    # CPU oracle on a stratified sample of i (all j): the accuracy reference, and its first
    # quarter timed as the CPU baseline
    if not args.no_cpu_baseline:
        import oracle
        idx = stratified_rows(n, args.error_rows, 7)
        count = idx.size
        q = max(1, count // 4)
        log(f"[bench] oracle on {count} i (one per {n // count} rows) x {n} j")
        t_a = time.perf_counter()
        parts = [oracle.force(x, v, m, args.eps ** 2, idx=idx[:q])]
        t_b = time.perf_counter()
        cached = load_oracle_reference(args.oracle_cache, x, v, m, args.eps, idx)
        if cached is not None and all(np.array_equal(c_[:q], p_) for c_, p_ in zip(cached, parts[0])):
            ra, rk, rp = cached  # the timed quarter, recomputed, equals the stored rows bitwise
            log(f"[bench] oracle rows {q}..{count} from the reference cache")
        else:
            cached = None
            if count > q:
                parts.append(oracle.force(x, v, m, args.eps ** 2, idx=idx[q:]))
            ra, rk, rp = (np.concatenate([p_[k] for p_ in parts]) for k in range(3))
            save_oracle_reference(args.oracle_cache, x, v, m, args.eps, idx, (ra, rk, rp))
        result["cpu_baseline"] = {
            "value": q * n / (t_b - t_a), "unit": "interactions/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{q} seeded i-particles (one per {4 * n // count} rows) x all {n} "
                      f"j-particles (FP64, long-double sums), {t_b - t_a:.1f} s"}

        def errs(gg):
            return {"e_acc": rms_rel(gg["a"][idx], ra), "e_jerk": rms_rel(gg["k"][idx], rk),
                    "e_pot": rms_rel(gg["pot"][idx], rp),
                    "max_row_rel_acc": float(np.max(np.linalg.norm(gg["a"][idx] - ra, axis=1)
                                                    / np.linalg.norm(ra, axis=1))),
                    "sample": count}
        errors = {args.precision: errs(g)}
        for prec, d in variants.items():
            errors[prec] = errs(d.pop("gv"))
        result["errors_vs_oracle"] = errors
        result["oracle_reference"] = {"rows": int(count), "rows_from_cache": cached is not None}
    else:
        for d in variants.values():
            d.pop("gv")
    # slowdown of each variant: its full-force time over the timed arithmetic's full force
    ns_per_int = avg_full_ms * 1e6 / (n * n)
    for prec, d in variants.items():
        d["slowdown_vs_" + args.precision] = (d["full_force_ms"] * 1e6 / (n * n)) / ns_per_int
    result["variants"] = variants
    if not args.no_configs:
        result["configs"] = other_configs(args)
    print(json.dumps(result), flush=True)


def _reference_path(cache_dir, x, v, m, eps, idx):
    """Cache file of the oracle's forces on rows idx of this exact input: keyed by a hash of
    the positions, velocities, masses, softening and rows."""
    import hashlib
    import numpy as np
    h = hashlib.sha256()
    for a in (x, v, m, np.array([eps], np.float64), idx):
        h.update(np.ascontiguousarray(a).tobytes())
    return os.path.join(os.path.expanduser(cache_dir), f"oracle_force_n{len(m)}_{h.hexdigest()[:24]}.npz")


def load_oracle_reference(cache_dir, x, v, m, eps, idx):
    """(acc, jerk, pot) of the oracle on rows idx from the cache, or None."""
    import numpy as np
    if not cache_dir:
        return None
    path = _reference_path(cache_dir, x, v, m, eps, idx)
    if not os.path.exists(path):
        return None
    try:
        with np.load(path, allow_pickle=False) as f:
            return f["acc"], f["jerk"], f["pot"]
    except (OSError, ValueError, KeyError):
        return None


def save_oracle_reference(cache_dir, x, v, m, eps, idx, ref):
    import numpy as np
    if not cache_dir:
        return
    path = _reference_path(cache_dir, x, v, m, eps, idx)
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp.npz"
        np.savez(tmp, acc=ref[0], jerk=ref[1], pot=ref[2])
        os.replace(tmp, path)
    except OSError:
        pass


def stratified_rows(n, count, seed):
    """`count` rows of n, one seeded row from each of `count` equal runs of rows."""
    import numpy as np
    block = max(1, n // count)
    r = np.random.default_rng(seed).integers(0, block, (n + block - 1) // block)
    return np.minimum(np.arange(r.size) * block + r, n - 1).astype(np.int64)


def other_configs(args):
    """One run of each of the other workloads (steps = 1 after one warmup, no CPU baseline),
    summarised: the N = 1024 block-step run to t = 1/8 (dt <= 1/64), the N = 65536 run to t = 1
    in FP32 (FP64-formed separations), double-single and the paper's all-single arithmetic
    against the committed oracle run, the 512-cluster ensemble to t = 1, and the gradient of
    the 64-step trajectory loss at N = 16384."""
    sub = argparse.Namespace(**vars(args))
    sub.steps, sub.warmup, sub.no_cpu_baseline = 1, 1, True
    out = {}

    def run_summary(r):
        c = r["config"]
        s = {"wall_s": c["wall_s"], "interactions_per_s": r["value"], "n_steps": c["n_steps"],
             "mean_block": c["mean_block"], "de_rel": c["de_rel"],
             "us_per_block_step": 1e6 * c["wall_s"] / c["n_steps"],
             "block_force_frac_fp32_peak": r["roofline"]["frac"]}
        ref = r.get("oracle_reference_run")
        if ref:
            s["oracle"] = {"n_steps": ref["n_steps"], "de_rel": ref["de_rel"]}
        for prec, v in r.get("variants", {}).items():
            s[prec] = v if "failed" in v else {"wall_s": v["wall_s"], "n_steps": v["n_steps"],
                                               "de_rel": v["de_rel"]}
        return s

    sub.precision, sub.variants = "fp32", "none"
    sub.run = "n1024_t0.125"
    sub.no_cpu_baseline = False  # the oracle runs this whole workload in well under a second
    r = bench_run(sub, emit=False)
    out["n1024_t0.125"] = run_summary(r)
    if "cpu_baseline" in r:
        out["n1024_t0.125"]["cpu_oracle_end_to_end"] = r["cpu_baseline"]
    sub.no_cpu_baseline = True
    sub.run, sub.variants = "n65536_t1", "ds,fp32all"
    out["n65536_t1"] = run_summary(bench_run(sub, emit=False))
    sub.variants, sub.clusters, sub.t_end, sub.tune = "none", 512, 1.0, False
    r = bench_ensemble(sub, emit=False)
    out["ensemble_512"] = {"wall_s": r["ms_per_step"] / 1e3, "interactions_per_s": r["value"],
                           "frac_fp32_peak": r["roofline"]["frac"],
                           "max_block_steps": r["config"]["max_block_steps"],
                           "dE_over_E_median": r["config"]["dE_over_E_median"],
                           "lanes": (r["config"]["lanes"] or {}).get("lanes", 1)}
    r = bench_adjoint(sub, emit=False)
    out["adjoint_n16384"] = {"ms_per_gradient": r["ms_per_step"], "interactions_per_s": r["value"]}
    return out


if __name__ == "__main__":
    main()
