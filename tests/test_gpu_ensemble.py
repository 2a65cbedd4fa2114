"""GPU parity of the ensemble path (nb_ens_*): every cluster of an ensemble integrated together
must match an independent oracle run of that cluster."""
import numpy as np
import pytest

import oracle
from paper_astro_ph_0702058_amd import nbody
from paper_astro_ph_0702058_amd.plummer import ensemble_sizes, plummer

pytestmark = pytest.mark.gpu

LMAX = 26


def build(sizes, seed0=100):
    xs, vs, ms = [], [], []
    for c, n in enumerate(sizes):
        x, v, m = plummer(int(n), seed0 + c)
        xs.append(x); vs.append(v); ms.append(m)
    return xs, vs, ms


def run_ensemble(sizes, eps, eta, t_end, prec, lmin=3, layout=None, graph=True, spl=8,
                 local=None, split=None, lanes=None):
    xs, vs, ms = build(sizes)
    st = nbody.DeviceState(np.concatenate(xs), np.concatenate(vs), np.concatenate(ms))
    ens = nbody.Ensemble(sizes, eps, lmin=lmin, lmax=LMAX, precision=prec)
    ens.nb_ens_bind(st)
    if layout:
        ens.nb_ens_set_layout(**layout)
    if local:
        ens.nb_ens_set_local(**local)
    if split:
        ens.nb_ens_set_split(split)
    if lanes is not None:
        ens.nb_ens_set_lanes(lanes)
    ens.nb_ens_init(eta)
    e0 = ens.nb_ens_energy()
    ens.nb_ens_run(eta, t_end, steps_per_launch=spl, max_steps=200000, use_graph=graph)
    ctl = ens.nb_ens_control()
    e1 = ens.nb_ens_energy()
    g = st.numpy()
    ens.close()
    return xs, vs, ms, g, ctl, e0, e1


def check_against_oracle_runs(sizes, t_end, prec="fp64"):
    """eps = 1/N_c, eta = 0.02: every cluster follows its own oracle run step for step
    (levels, ticks, positions, energies)."""
    assert float(t_end * 8).is_integer(), "the oracle's energy needs synchronised particles"
    eps = [1.0 / n for n in sizes]
    xs, vs, ms, g, ctl, e0, e1 = run_ensemble(sizes, eps, 0.02, t_end, prec)
    off = np.concatenate([[0], np.cumsum(sizes)])
    for c, n in enumerate(sizes):
        ref = oracle.BlockIntegrator(xs[c], vs[c], ms[c], eps=eps[c], nu=0.02, lmin=3)
        E0 = ref.energy()
        ref.run_until(t_end)
        sl = slice(off[c], off[c + 1])
        assert ctl[c].n_steps == ref.n_steps, (c, ctl[c].n_steps, ref.n_steps)
        assert ctl[c].n_active_sum == ref.n_active_total
        assert ctl[c].t_cur == ref.t and ctl[c].flags == 1
        assert np.array_equal(g["level"][sl], ref.level) and np.array_equal(g["tick"][sl], ref.tick)
        assert np.max(np.abs(g["x"][sl] - ref.x)) < 1e-10, c
        assert abs((e0[0][c] + e0[1][c]) - E0) <= 1e-13 * abs(E0)
        assert abs((e1[0][c] + e1[1][c]) - ref.energy()) <= 1e-11 * abs(E0)


def test_ensemble_fp64_matches_independent_oracle_runs():
    """Six clusters of uneven size (tiles plus ragged tails, last tiles of one particle), to
    t = 1/8."""
    check_against_oracle_runs([64, 100, 257, 300, 513, 1000], 0.125)


def test_ensemble_double_single_matches_independent_oracle_runs():
    """The double-single interaction (forces to about 1e-14 of the FP64 oracle's) keeps every
    cluster on its oracle run step for step as well, to t = 1/8."""
    check_against_oracle_runs([64, 257, 700, 1000], 0.125, "ds")


def test_ensemble_cluster_beyond_the_selection_cache():
    """A cluster larger than the 4096 particles whose t_i + dt_i the cluster-local selection
    keeps in LDS (it then reads them again for the compaction), beside a small one, to t = 1/8
    (every particle synchronised, where the oracle's energy applies): both follow their oracle
    runs step for step."""
    check_against_oracle_runs([5000, 64], 1 / 8)


def test_ensemble_whole_tiles_and_tiny_clusters():
    """Clusters that fill whole j-tiles exactly (256, 512), one short of a tile, and the
    degenerate one- and two-particle clusters (a lone particle feels no force and takes the
    longest step), to t = 1/8."""
    check_against_oracle_runs([1, 256, 2, 512, 255], 0.125)


def test_ensemble_layouts_agree():
    """Different work layouts (tiles per item, unroll, lanes per block particle) only reorder
    sums: FP64 runs take the same block steps with positions to 1e-12."""
    sizes = [70, 600, 1300]
    eps = [1.0 / n for n in sizes]
    outs = []
    for layout, split in ((dict(tiles_per_item=1, ipl=1, unroll=2), None),
                          (dict(tiles_per_item=4, ipl=1, unroll=1), None),
                          (dict(tiles_per_item=[1, 2, 3], ipl=1, unroll=2), None),
                          (dict(tiles_per_item=1, ipl=1, unroll=2), 1),
                          (dict(tiles_per_item=2, ipl=1, unroll=2), 16),
                          (dict(tiles_per_item=1, ipl=1, unroll=1), 64)):
        *_, g, ctl, e0, e1 = run_ensemble(sizes, eps, 0.02, 1 / 32, "fp64", layout=layout,
                                          split=split)
        outs.append((g, [c.n_steps for c in ctl]))
    for g, steps in outs[1:]:
        assert steps == outs[0][1]
        assert np.max(np.abs(g["x"] - outs[0][0]["x"])) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("graph", [True, False])
def test_ensemble_lanes_give_the_same_runs(prec, graph):
    """Clusters split into independent lanes (each its own global steps, graph and stream) give
    bitwise the same states, block steps and energies as one lane: the clusters are
    independent.  Lanes of one, two and three groups of uneven size, replays of 8 global steps
    (several per lane, the lanes finishing at different replays)."""
    sizes = [70, 600, 1300, 90, 2100, 300, 64]
    eps = [1.0 / n for n in sizes]
    ref = run_ensemble(sizes, eps, 0.02, 1 / 16, prec, graph=graph)
    for lane_of in ([1, 0, 0, 1, 0, 1, 1], [2, 0, 1, 2, 0, 2, 1]):
        out = run_ensemble(sizes, eps, 0.02, 1 / 16, prec, graph=graph, lanes=lane_of)
        g, ctl, e1 = out[3], out[4], out[6]
        for key in ("x", "v", "a", "k", "tick", "level"):
            assert np.array_equal(g[key], ref[3][key]), (lane_of, key)
        assert [(c.n_steps, c.n_active_sum, c.t_cur) for c in ctl] == \
               [(c.n_steps, c.n_active_sum, c.t_cur) for c in ref[4]]
        assert np.array_equal(e1[0], ref[6][0]) and np.array_equal(e1[1], ref[6][1])


def test_ensemble_lanes_stop_at_max_steps():
    """A global step advances every unfinished cluster by one block step, in one lane or in
    several, so a run stopped after the same number of global steps (max_steps 16 at 8 per
    replay) leaves bitwise the same state in one lane and in two."""
    sizes = [600, 90, 1300, 64]
    eps = [1.0 / n for n in sizes]
    outs = []
    for lanes in (None, [0, 1, 1, 0]):
        xs, vs, ms = build(sizes)
        st = nbody.DeviceState(np.concatenate(xs), np.concatenate(vs), np.concatenate(ms))
        ens = nbody.Ensemble(sizes, eps, lmin=3, lmax=LMAX, precision="fp64")
        ens.nb_ens_bind(st)
        if lanes is not None:
            ens.nb_ens_set_lanes(lanes)
        ens.nb_ens_init(0.02)
        ens.nb_ens_run(0.02, 1.0, steps_per_launch=8, max_steps=16)
        ctl = ens.nb_ens_control()
        outs.append((st.numpy(), [(c.n_steps, c.t_cur) for c in ctl]))
        ens.close()
    assert all(n == 16 for n, _ in outs[0][1]), outs[0][1]
    assert outs[1][1] == outs[0][1]
    for key in ("x", "v", "a", "k", "tick", "level"):
        assert np.array_equal(outs[1][0][key], outs[0][0][key]), key


def test_ensemble_lanes_are_checked():
    """nb_ens_set_lanes refuses a lane outside [0, lanes), an empty lane and more than three."""
    sizes = [70, 300, 90]
    xs, vs, ms = build(sizes)
    st = nbody.DeviceState(np.concatenate(xs), np.concatenate(vs), np.concatenate(ms))
    ens = nbody.Ensemble(sizes, [1 / 70, 1 / 300, 1 / 90], lmin=3, lmax=LMAX, precision="fp32")
    ens.nb_ens_bind(st)
    ens.nb_ens_set_lanes([0, 1, 2])
    ens.nb_ens_set_lanes(None)
    for bad in ([0, 2, 2], [0, -1, 1], [0, 1, 3]):
        with pytest.raises(RuntimeError, match="lane"):
            ens.nb_ens_set_lanes(bad)
    ens.close()
    sizes = [64] * 5
    xs, vs, ms = build(sizes)
    st = nbody.DeviceState(np.concatenate(xs), np.concatenate(vs), np.concatenate(ms))
    ens = nbody.Ensemble(sizes, 1 / 64, lmin=3, lmax=LMAX, precision="fp32")
    ens.nb_ens_bind(st)
    with pytest.raises(RuntimeError, match="lanes"):
        ens.nb_ens_set_lanes([0, 1, 2, 3, 0])
    ens.close()


def test_ensemble_split_is_a_power_of_two():
    """nb_ens_set_split takes powers of two from 1 to 64 and refuses anything else."""
    sizes = [70, 300]
    xs, vs, ms = build(sizes)
    st = nbody.DeviceState(np.concatenate(xs), np.concatenate(vs), np.concatenate(ms))
    ens = nbody.Ensemble(sizes, [1 / 70, 1 / 300], lmin=3, lmax=LMAX, precision="fp32")
    ens.nb_ens_bind(st)
    for ok in (1, 2, 8, 64):
        ens.nb_ens_set_split(ok)
    for bad in (0, 3, 12, 128, -4):
        with pytest.raises(RuntimeError, match="smin"):
            ens.nb_ens_set_split(bad)
    ens.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ensemble_local_steps_agree(prec):
    """Which blocks a cluster's own workgroup advances only changes summation orders: no local
    blocks (every block through the GPU-wide force), the defaults, every block of up to 1024
    particles local one step per global step, and every block local with unlimited steps per
    launch all take the same block steps (FP64: to 1e-12 in position; FP32: step counts within
    2 %, the decisions near a power of two being taken from forces that differ by rounding)."""
    sizes = [64, 300, 1000, 2100]
    eps = [1.0 / n for n in sizes]
    outs = []
    for local in (dict(local_limit=0, local_steps=0, local_work=0), None,
                  dict(local_limit=1 << 40, local_steps=1, local_work=1 << 40),
                  dict(local_limit=1 << 40, local_steps=1 << 30, local_work=1 << 40)):
        *_, g, ctl, e0, e1 = run_ensemble(sizes, eps, 0.02, 1 / 8, prec, local=local)
        assert all(c.flags == 1 and c.t_cur == 1 << (LMAX - 3) for c in ctl)
        outs.append((g, np.array([c.n_steps for c in ctl]),
                     np.array([c.n_active_sum for c in ctl])))
    for g, steps, act in outs[1:]:
        print(f"{prec}: steps {steps} vs {outs[0][1]}", flush=True)
        if prec == "fp64":
            assert np.array_equal(steps, outs[0][1]) and np.array_equal(act, outs[0][2])
            assert np.max(np.abs(g["x"] - outs[0][0]["x"])) < 1e-12
        else:
            assert np.all(np.abs(steps - outs[0][1]) <= 0.02 * outs[0][1])


def test_ensemble_graph_equals_eager():
    sizes = [90, 400, 700]
    eps = [1.0 / n for n in sizes]
    a = run_ensemble(sizes, eps, 0.02, 1 / 16, "fp32", graph=False, spl=4)
    b = run_ensemble(sizes, eps, 0.02, 1 / 16, "fp32", graph=True, spl=4)
    for key in ("x", "v", "tick", "level"):
        assert np.array_equal(a[3][key], b[3][key]), key


def test_ensemble_fp32_log_uniform_sizes():
    """48 clusters, sizes log-uniform in [64, 4096], eps = 1/N_c, eta = 0.02, to t = 1/4, in FP32
    and in FP64 (the FP64 ensemble follows the oracle step for step, see above): every cluster
    finishes; at eta = 0.02 the energy error is the integrator's (Sec. 4.2), so the FP32 run's
    error stays within 10x of the FP64 run's (plus 1e-6), and step counts agree within 10 %."""
    sizes = ensemble_sizes(48, 4)
    eps = 1.0 / sizes
    res = {}
    for prec in ("fp32", "fp64"):
        xs, vs, ms, g, ctl, e0, e1 = run_ensemble(sizes, eps, 0.02, 0.25, prec, spl=16)
        de = np.abs((e1[0] + e1[1]) - (e0[0] + e0[1])) / np.abs(e0[0] + e0[1])
        assert all(c.flags == 1 and c.t_cur == 1 << (LMAX - 2) for c in ctl)
        res[prec] = (de, np.array([c.n_steps for c in ctl]))
    de32, st32 = res["fp32"]
    de64, st64 = res["fp64"]
    print("dE/E fp32 median %.2e max %.2e; fp64 median %.2e max %.2e" %
          (np.median(de32), de32.max(), np.median(de64), de64.max()), flush=True)
    assert np.all(de32 <= 10 * de64 + 1e-6), np.max(de32 / (10 * de64 + 1e-6))
    assert np.all(np.abs(st32 - st64) <= 0.1 * st64)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_ensemble_against_committed_oracle_runs(prec):
    """The batched workload at full size: 512 Plummer clusters, N_c log-uniform in [64, 4096]
    (551629 particles), eps = 1/N_c, eta = 0.02, every cluster to t = 1, against the FP64 oracle
    run of each cluster committed in tests/golden/ensemble_runs.json (make_ensemble_reference.py).
    FP64 interaction: every cluster takes exactly the oracle's block steps (count and particle
    steps) and its energy error agrees to 1e-12.  FP32: each cluster's block steps within 1 %,
    the particle steps of the whole run within 0.1 %, and the energy error, set by the
    integrator at this eta (median 1.2e-7), within a factor 4 of the oracle's plus 1e-8 for
    every cluster, with the median ratio within 10 % of 1."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ensemble_runs.json")
    if not os.path.exists(path):
        pytest.skip("the oracle ensemble runs have not been written")
    g = json.load(open(path))
    p = g["params"]
    sizes = ensemble_sizes(p["clusters"], p["size_seed"])
    parts = [plummer(int(nc), p["seed0"] + c) for c, nc in enumerate(sizes)]
    st = nbody.DeviceState(np.concatenate([q[0] for q in parts]), np.concatenate([q[1] for q in parts]),
                           np.concatenate([q[2] for q in parts]))
    ens = nbody.Ensemble(sizes, 1.0 / sizes, lmin=p["lmin"], lmax=LMAX, precision=prec)
    ens.nb_ens_bind(st)
    ens.nb_ens_init(p["eta"])
    ek0, ep0 = ens.nb_ens_energy()
    ens.nb_ens_run(p["eta"], p["t_end"], steps_per_launch=32, max_steps=60000)
    ctl = ens.nb_ens_control()
    ek1, ep1 = ens.nb_ens_energy()
    ens.close()
    ref = g["clusters"]
    steps = np.array([c.n_steps for c in ctl]); rsteps = np.array([r["n_steps"] for r in ref])
    act = np.array([c.n_active_sum for c in ctl]); ract = np.array([r["n_active_sum"] for r in ref])
    de = (ek1 + ep1 - ek0 - ep0) / (ek0 + ep0)
    rde = np.array([(r["energy1"] - r["energy0"]) / r["energy0"] for r in ref])
    assert np.all([c.t_cur == 1 << LMAX for c in ctl]) and np.all([c.flags == 1 for c in ctl])
    print(f"{prec}: {np.sum(steps == rsteps)} of {len(ref)} clusters with the oracle's step count; "
          f"max |ddE/E| {np.max(np.abs(de - rde)):.2e}", flush=True)
    if prec == "fp64":
        assert np.array_equal(steps, rsteps) and np.array_equal(act, ract)
        assert np.max(np.abs(de - rde)) <= 1e-12
    else:
        assert np.max(np.abs(steps - rsteps) / rsteps) <= 0.01
        assert abs(act.sum() / ract.sum() - 1.0) <= 1e-3
        assert np.all(np.abs(de) <= 4 * np.abs(rde) + 1e-8)
        ratio = np.abs(de) / np.maximum(np.abs(rde), 1e-300)
        assert abs(np.median(ratio) - 1.0) <= 0.1
