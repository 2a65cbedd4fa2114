"""Autotuning of force-kernel launch variants with an on-disk cache.

The library's nb_tune() times every compiled variant (i-particles per work-item, j-loop unroll,
work items per launch, which fixes the j-split) on the live device.  This module runs it for the
two call classes of a context -- full-force calls and block-step calls, the latter at the block
size the paper's fit predicts (0.20 N^0.81) -- and remembers the winners per device name,
precision and N in a JSON file, so that later contexts of the same shape reuse them.
"""
from __future__ import annotations

import json
import os

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "libnbody_tune.json")


def expected_block_size(n: int) -> int:
    """Mean block size of the block time-step scheme, 0.20 N^0.81 (the paper's fit, Sec. 5)."""
    return max(1, min(n, int(round(0.20 * n ** 0.81))))


def _key(ctx, which, n_i):
    import torch
    name = torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{name}|{ctx.precision}|eps>0={ctx.eps > 0}|n={ctx.n}|which={which}|n_i={n_i}"


def autotune(ctx, cache_path: str | None = DEFAULT_CACHE, reps: int = 2, retune: bool = False):
    """Tune (or load) both variants of a bound, predicted context.  Returns {which: variant}."""
    cache = {}
    if cache_path and os.path.exists(cache_path) and not retune:
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    chosen = {}
    for which, n_i in ((0, ctx.n), (1, expected_block_size(ctx.n))):
        key = _key(ctx, which, n_i)
        if key in cache and "scalar_tiles" in cache[key]["variant"]:
            ctx.nb_set_variant(which, cache[key]["variant"])
            chosen[which] = ctx.nb_get_variant(which)
            continue
        v, ms = ctx.nb_tune(which, n_i, reps)
        cache[key] = {"variant": v, "ms": ms}
        chosen[which] = v
    if cache_path:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return chosen


def ensemble_autotune(ens, state, x0, v0, eta, t_probe=0.25, steps_per_launch=128):
    """Choose the ensemble's force work layout by timing runs from the initial state to
    t_probe (default 1/4: the phase in which nearly every cluster is active and which takes
    most of a run's time): first the fewest lanes per block particle of a force item (smin,
    which bounds an item's size), then the j-loop unroll, then, for each size class of clusters
    (N < 512, 512 <= N < 2048, N >= 2048), the whole j-tiles per work item halved or doubled
    from the default's.  The winner is timed again against the library's default layout (at
    most 4 j-ranges per cluster, smin 8, unroll 2) on the same probe and kept only if it is
    faster; the state is
    restored from (x0, v0) before every trial and after tuning.  Returns the layout in effect
    with both probe times and whether the search beat the default."""
    import time
    import numpy as np
    import torch

    sizes = np.diff(ens.offsets)
    classes = [sizes < 512, (sizes >= 512) & (sizes < 2048), sizes >= 2048]

    def trial(tpi, smin, ipl, unroll):
        ens.nb_ens_set_layout(tpi, ipl, unroll)
        ens.nb_ens_set_split(smin)
        state.x.copy_(x0); state.v.copy_(v0)
        ens.nb_ens_init(eta)
        torch.cuda.synchronize()
        t = time.perf_counter()
        ens.nb_ens_run(eta, t_probe, steps_per_launch=steps_per_launch)
        return time.perf_counter() - t

    # the library's default: at most 4 j-ranges per cluster, 8 lanes per block particle
    ntiles = (sizes + 255) // 256
    default = (np.maximum(1, (ntiles + 3) // 4).astype(np.int32), 8, 1, 2)
    trial(*default)  # warm: graphs and caches of the default layout
    tpi = default[0].copy()
    timed = {sm: trial(tpi, sm, 1, 2) for sm in (2, 4, 8, 16)}
    smin = min(timed, key=timed.get)
    best = timed[smin]
    t1 = trial(tpi, smin, 1, 1)
    unroll = 1 if t1 < best else 2
    best = min(best, t1)
    for mask in classes:  # per size class: the default's tiles per item halved or doubled
        if not mask.any():
            continue
        for scale in (0.5, 2.0):
            t2 = tpi.copy()
            t2[mask] = np.maximum(1, np.rint(tpi[mask] * scale)).astype(np.int32)
            if np.array_equal(t2, tpi):
                continue
            t = trial(t2, smin, 1, unroll)
            if t < best:
                best, tpi = t, t2
    # the search's winner against the default, each timed once more, in that order
    t_best = trial(tpi, smin, 1, unroll)
    t_default = trial(*default)
    beats = t_best < t_default
    if not beats:
        tpi, smin, _, unroll = default
    ens.nb_ens_set_layout(tpi, 1, unroll)
    ens.nb_ens_set_split(smin)
    state.x.copy_(x0); state.v.copy_(v0)
    return {"smin": int(smin), "ipl": 1, "unroll": int(unroll),
            "tiles_per_item_by_class": [sorted(set(int(t) for t in tpi[m])) if m.any() else None
                                        for m in classes],
            "probe_t_end": t_probe, "probe_seconds_chosen": t_best,
            "probe_seconds_default": t_default, "beats_default": bool(beats)}


def ensemble_lanes(ens, state, x0, v0, eta, t_probe=0.25, top=4, steps_per_launch=128):
    """Two independent lanes for an ensemble (nb_ens_set_lanes): a probe run to t_probe from the
    initial state (x0, v0) counts every cluster's block steps, and the `top` clusters with the
    most steps get a lane of their own, so the global step count of the rest no longer follows
    the cluster with the tightest encounters.  On MI355X, 512 Plummer clusters of 64-4096
    particles to t = 1 (alternated on one machine): 0.657-0.658 s against 0.757-0.758 s in one
    lane; 2 / 8 / 16 / 32 / 64 clusters apart 0.661 / 0.683 / 0.709 / 0.710 / 0.710 s; three
    lanes (8 / 56 / the rest) 0.85-0.88 s; 8 apart by size 1.01 s.
    The probe leaves the ensemble re-initialised at (x0, v0).  Returns the lane of each cluster
    (numpy int32) after setting it."""
    import numpy as np
    ens.nb_ens_set_lanes(None)
    state.x.copy_(x0); state.v.copy_(v0)
    ens.nb_ens_init(eta)
    ens.nb_ens_run(eta, t_probe, steps_per_launch=steps_per_launch)
    steps = np.array([c.n_steps for c in ens.nb_ens_control()])
    lane = np.ones(len(steps), np.int32)
    if len(steps) > top:
        lane[np.argsort(-steps, kind="stable")[:top]] = 0
        ens.nb_ens_set_lanes(lane)
    else:
        lane[:] = 0
    state.x.copy_(x0); state.v.copy_(v0)
    ens.nb_ens_init(eta)
    return lane
