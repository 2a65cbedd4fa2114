"""Turn rocprofv3 CSV output into the short text summaries kept under profiles/.

    python -m paper_astro_ph_0702058_amd.profiling stats  <kernel_stats.csv> --cmd "..." > out.txt
    python -m paper_astro_ph_0702058_amd.profiling traffic <fetch.csv> <write.csv> \
        --kernel SUBSTR --copy-bytes B --json out.json --cmd-fetch "..." --cmd-write "..."
    python -m paper_astro_ph_0702058_amd.profiling counters <counter_collection.csv> --kernel SUBSTR

Traffic: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the kernel are each scaled by
(known bytes of a plain device copy) / (what the same counter reads for that copy), using the
largest copyBuffer dispatch in the same run.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hpp", "ds_arith.hpp"):
        with open(os.path.join(ROOT, "paper_astro_ph_0702058_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats(path, cmd, top=12):
    rows = list(csv.DictReader(open(path)))
    out = [f"# rocprofv3 --kernel-trace --stats summary", f"# command: {cmd}", "",
           f"{'calls':>6} {'total ms':>11} {'avg ms':>11} {'min ms':>10} {'max ms':>10} {'%':>7}  kernel"]
    for r in rows[:top]:
        out.append(f"{int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:11.3f} "
                   f"{float(r['AverageNs']) / 1e6:11.4f} {float(r['MinNs']) / 1e6:10.4f} "
                   f"{float(r['MaxNs']) / 1e6:10.4f} {float(r['Percentage']):7.3f}  {r['Name'][:110]}")
    return "\n".join(out)


def _per_dispatch(path, counter):
    rows = list(csv.DictReader(open(path)))
    return [(r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"]))
            for r in rows if r["Counter_Name"] == counter]


def traffic(fetch_csv, write_csv, kernel, copy_bytes):
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        d = _per_dispatch(path, counter)
        copies = [v for name, grid, v in d if "copyBuffer" in name]
        ref = max(copies)  # KiB read for the largest plain copy of the run
        scale = (copy_bytes / 1024.0) / ref
        vals = [v for name, grid, v in d if kernel in name]
        res[counter] = {"kib_per_dispatch": vals, "copy_kib": ref, "scale": scale,
                        "bytes_per_dispatch": statistics.median(vals) * 1024.0 * scale}
    return res


def counters(path, kernel):
    rows = list(csv.DictReader(open(path)))
    agg = {}
    for r in rows:
        if kernel in r["Kernel_Name"]:
            agg.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: statistics.median(v) for k, v in agg.items()}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats"); a.add_argument("csv"); a.add_argument("--cmd", required=True)
    a.add_argument("--top", type=int, default=12, help="kernels listed, by total time")
    b = sub.add_parser("traffic"); b.add_argument("fetch"); b.add_argument("write")
    b.add_argument("--kernel", required=True); b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--json"); b.add_argument("--n", type=int, required=True)
    b.add_argument("--eps", type=float, required=True); b.add_argument("--symbol", required=True)
    b.add_argument("--algorithmic-bytes", type=float, required=True)
    b.add_argument("--cmd-fetch", required=True); b.add_argument("--cmd-write", required=True)
    b.add_argument("--variant", help="launch configuration of the profiled launches (JSON)")
    c = sub.add_parser("counters"); c.add_argument("csv"); c.add_argument("--kernel", required=True)
    c.add_argument("--interactions", type=float,
                   help="interactions per dispatch: also print per-interaction figures")
    c.add_argument("--ms", type=float, help="dispatch duration (ms) for the rates")
    args = ap.parse_args(argv)
    if args.what == "stats":
        print(stats(args.csv, args.cmd, args.top))
    elif args.what == "traffic":
        t = traffic(args.fetch, args.write, args.kernel, args.copy_bytes)
        fb, wb = t["FETCH_SIZE"]["bytes_per_dispatch"], t["WRITE_SIZE"]["bytes_per_dispatch"]
        doc = {"kernel": args.symbol, "n": args.n, "eps": args.eps,
               "hbm_bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
               "fetch_scale": t["FETCH_SIZE"]["scale"], "write_scale": t["WRITE_SIZE"]["scale"],
               "copy_bytes": args.copy_bytes, "algorithmic_bytes_per_launch": args.algorithmic_bytes,
               "kernel_source_sha256_16": kernel_source_hash(),
               "variant": json.loads(args.variant) if args.variant else None,
               "commands": {"FETCH_SIZE": args.cmd_fetch, "WRITE_SIZE": args.cmd_write},
               "raw_kib": {"FETCH_SIZE": t["FETCH_SIZE"]["kib_per_dispatch"],
                           "WRITE_SIZE": t["WRITE_SIZE"]["kib_per_dispatch"],
                           "copy_FETCH_SIZE": t["FETCH_SIZE"]["copy_kib"],
                           "copy_WRITE_SIZE": t["WRITE_SIZE"]["copy_kib"]}}
        if args.json:
            with open(args.json, "w") as f:
                json.dump(doc, f, indent=1)
        print(json.dumps(doc, indent=1))
    else:
        m = counters(args.csv, args.kernel)
        for k, v in sorted(m.items()):
            print(f"{k:32s} {v:.6g}")
        if args.interactions:
            n2 = args.interactions
            per = lambda k: m.get(k, 0.0) * 64 / n2   # wave-level counts x 64 lanes
            print("\n# derived (wave-level counts x 64 lanes / interactions):")
            print(f"VALU instructions per interaction      {per('SQ_INSTS_VALU'):.2f}")
            print(f"v_rsq_f32 per interaction              {per('SQ_INSTS_VALU_TRANS_F32'):.3f}")
            print(f"hardware-counted FP32 flop/interaction {per('SQ_INSTS_VALU_FLOPS_FP32'):.2f}"
                  "   (FMA = 2; the paper's convention counts 60)")
            print(f"LDS instructions per interaction       {per('SQ_INSTS_LDS'):.3f}")
            if args.ms:
                t = args.ms * 1e-3
                print(f"hardware-counted FP32 rate             "
                      f"{per('SQ_INSTS_VALU_FLOPS_FP32') * n2 / t / 1e12:.1f} TFLOP/s at {args.ms:.2f} ms")
                print(f"60-flop-convention rate                {60 * n2 / t / 1e12:.1f} TFLOP/s = "
                      f"{100 * 60 * n2 / t / 157.3e12:.1f}% of 157.3")
                print(f"VALU lane-instructions per second      {per('SQ_INSTS_VALU') * n2 / t:.3e}")


if __name__ == "__main__":
    sys.exit(main())
