"""GPU parity of the force path (nb_predict + nb_force through the C ABI) against the FP64 oracle.

Two error measures, both asserted on every check:
* rms relative, over the listed i: e_a = sqrt(mean_i |a_i - a_i^ref|^2 / |a_i^ref|^2), likewise
  for the jerk and the potential;
* per row, against the size of the row's terms: |a_i - a_i^ref| / sa_i with
  sa_i = sum_{j != i} m_j |d| s^-3/2, and |k_i - k_i^ref| / sk_i with
  sk_i = sum_{j != i} m_j (|u| s^-3/2 + 3 |d.u| |d| s^-5/2) (oracle.force_scale); the potential
  terms share one sign, so its per-row relative error is that measure already.  A sum of terms
  rounded to relative u is off by at most about u times that scale however much the pulls
  cancel, so no row, including one near the centre whose pulls cancel to a tiny |a|, may exceed
  the target on it.
Tolerances (the same number bounds the rms and every row):
  fp32: acc 2e-6 (the target for single-precision arithmetic), jerk 1e-5, pot 2e-6;
  ds:   acc 1e-11 (the target for double-single arithmetic), jerk 1e-10, pot 1e-11;
  fp64: 1e-13 for all three (a few ulp per term; tile sums keep growth well below that).
The all-single arithmetic (fp32all) is compared with the oracle fed the same float-rounded
inputs; its sums stay in float (256-term tile sums added in float), so first-order rounding
grows like u sqrt(256 + N/256) times the ratio of the sum of |terms| to |sum| (about 10 for
a Plummer sphere): with u = 6e-8 and N <= 20000 that is 1e-5 for acc and pot, and 1e-4 for
the jerk (whose sum cancels more).
"""
import numpy as np
import pytest

import oracle
from paper_astro_ph_0702058_amd import nbody
from paper_astro_ph_0702058_amd.plummer import plummer, sample_indices
from _parity import TOL, check, reference, rms_rel, stratified_rows

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "ds", "fp64"])
def test_force_all_i_ragged(prec):
    """N = 1000 (three full tiles plus a ragged tail), all i against all j."""
    x, v, m = plummer(1000, 11)
    eps = 1 / 256
    got = nbody.force_on_state(x, v, m, eps, prec)
    ref, scale = reference(x, v, m, eps * eps)
    check(prec, got, ref, scale, "N=1000")


@pytest.mark.parametrize("prec", ["fp32", "ds", "fp64"])
def test_force_subset_uses_j_split(prec):
    """Few i against many j: the work is split over j-ranges and summed in a second pass."""
    n = 20000
    x, v, m = plummer(n, 12)
    eps = 1e-3
    idx = sample_indices(n, 300, 5)
    got = nbody.force_on_state(x, v, m, eps, prec, idx=idx)
    ref, scale = reference(x, v, m, eps * eps, idx=idx)
    check(prec, got, ref, scale, "N=20000 j-split")


@pytest.mark.parametrize("prec", ["fp32", "ds", "fp64"])
def test_force_unsoftened(prec):
    """eps = 0: the self pair is masked out instead of subtracted."""
    x, v, m = plummer(700, 13)
    got = nbody.force_on_state(x, v, m, 0.0, prec)
    ref, scale = reference(x, v, m, 0.0)
    check(prec, got, ref, scale, "eps=0")


@pytest.mark.parametrize("prec", ["fp32", "ds", "fp64"])
def test_force_degenerate_sizes(prec):
    # a single particle feels nothing
    a, k, p = nbody.force_on_state(np.array([[0.3, -0.2, 0.1]]), np.array([[1.0, 0, 0]]),
                                   np.array([1.0]), 0.01, prec)
    assert np.all(a == 0) and np.all(k == 0) and np.all(p == 0)
    # the two-body closed form: d = (1,2,2), eps^2 = 16, m_j = 1, u = (0,0,1)
    x = np.array([[0.0, 0, 0], [1.0, 2, 2]]); v = np.array([[0.0, 0, 0], [0.0, 0, 1]])
    m = np.array([1.0, 1.0])
    a, k, p = nbody.force_on_state(x, v, m, 4.0, prec)
    tol = 1e-6 if prec == "fp32" else 1e-14
    np.testing.assert_allclose(a[0], [0.008, 0.016, 0.016], rtol=tol, atol=0)
    np.testing.assert_allclose(k[0], [-0.00192, -0.00384, 0.00416], rtol=tol, atol=1e-20)
    np.testing.assert_allclose(p, [-0.2, -0.2], rtol=tol)
    np.testing.assert_allclose(a[1], -a[0], rtol=tol)
    # an empty i-list is a no-op
    a, k, p = nbody.force_on_state(x, v, m, 4.0, prec, idx=np.zeros(0, np.int32))
    assert a.shape == (0, 3)


def test_force_is_deterministic():
    x, v, m = plummer(5000, 14)
    r1 = nbody.force_on_state(x, v, m, 1 / 256, "fp32")
    r2 = nbody.force_on_state(x, v, m, 1 / 256, "fp32")
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)


def _full_force(x, v, m, eps, prec):
    """All-i force of the state at its own time through nb_predict + nb_force without a device
    count: the full-force launch class the benchmark times (j-split partials and the
    scalar-load j-loop at this size).  Returns the device tensors (acc, jerk, pot)."""
    import torch
    n = x.shape[0]
    st = nbody.DeviceState(x, v, m)
    with nbody.Context(n, eps, precision=prec) as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        acc = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        jerk = torch.zeros_like(acc)
        pot = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.nb_force(acc, jerk, pot)
        ctx.nb_sync()
    return acc, jerk, pot


def _rows_of(t, rows):
    import torch
    acc, jerk, pot = t
    ii = torch.as_tensor(rows, device="cuda")
    return acc[:, ii].cpu().numpy().T, jerk[:, ii].cpu().numpy().T, pot[ii].cpu().numpy()


def test_force_full_size_sampled():
    """N = 2^20 Plummer sphere, eps = 1/256: the full all-i force (the launch the benchmark
    times: 4096 i-blocks of 256 against K = 16 j-ranges, XCD-ordered work items, fixed-order
    reduction).  Single precision is checked on one seeded row of every 256-row i-block plus
    the first and last row (4098 rows); double-single, through the same all-i call, on one
    row of every 2048 (every eighth of those rows: 514 rows spread over all i-blocks)."""
    n = 1 << 20
    x, v, m = plummer(n, 3)
    eps = 1 / 256
    rows = stratified_rows(n, 256, 21)
    assert rows.size == 4098
    ref, scale = reference(x, v, m, eps * eps, idx=rows)
    got = _rows_of(_full_force(x, v, m, eps, "fp32"), rows)
    check("fp32", got, ref, scale, "N=2^20 all-i launch, one row per i-block")
    sub = np.unique(np.concatenate([np.arange(0, rows.size, 8), [rows.size - 1]]))
    assert sub.size >= 512
    got = _rows_of(_full_force(x, v, m, eps, "ds"), rows[sub])
    check("ds", got, tuple(r[sub] for r in ref), (scale[0][sub], scale[1][sub]),
          "N=2^20 all-i launch, one row per 2048")


def test_nonfinite_input_is_reported():
    """A NaN position makes forces non-finite: the device latches the flag and the next
    synchronising call reports NB_ENONFINITE (the kernels themselves finish normally)."""
    import torch
    x, v, m = plummer(300, 15)
    x[7, 0] = np.nan
    st = nbody.DeviceState(x, v, m)
    with nbody.Context(300, 0.01, precision="fp32") as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        acc = torch.zeros((3, 300), dtype=torch.float64, device="cuda")
        jerk = torch.zeros_like(acc); pot = torch.zeros(300, dtype=torch.float64, device="cuda")
        ctx.nb_force(acc, jerk, pot)
        with pytest.raises(nbody.NBodyError) as e:
            ctx.nb_sync()
        assert e.value.status == nbody.NB_ENONFINITE


def test_argument_errors_on_device():
    import torch
    x, v, m = plummer(64, 16)
    st = nbody.DeviceState(x, v, m)
    with nbody.Context(64, 0.01) as ctx:
        acc = torch.zeros((3, 64), dtype=torch.float64, device="cuda")
        with pytest.raises(nbody.NBodyError) as e:
            ctx.nb_force(acc, acc, acc[0])          # nothing bound yet
        assert e.value.status == nbody.NB_ESTATE
        ctx.nb_bind(st)
        with pytest.raises(nbody.NBodyError) as e:
            ctx.nb_force(acc, acc, acc[0])          # not predicted yet
        assert e.value.status == nbody.NB_ESTATE


@pytest.mark.parametrize("prec", ["fp32", "ds", "fp64"])
@pytest.mark.parametrize("n_i", [1, 3, 37, 130, 255])
def test_force_small_lists_lane_split(prec, n_i):
    """Fewer i-particles than a workgroup: several lanes share each i, take interleaved j of
    every tile and are combined by wave shuffles; eps > 0 and eps = 0."""
    n = 5000
    x, v, m = plummer(n, 17)
    idx = sample_indices(n, n_i, 9 + n_i)
    for eps in (1 / 256, 0.0):
        got = nbody.force_on_state(x, v, m, eps, prec, idx=idx)
        ref, scale = reference(x, v, m, eps * eps, idx=idx)
        check(prec, got, ref, scale, f"n_i={n_i} eps={eps}")


@pytest.mark.parametrize("eps", [1 / 256, 0.0])
def test_force_all_single_matches_rounded_inputs(eps):
    """The all-single arithmetic (the paper's kernel) rounds the predicted positions,
    velocities and masses to float before forming separations; against the oracle evaluated on
    those same rounded inputs it meets the tolerances derived above.  All i at N = 1000
    (ragged tail), a j-split subset at N = 20000, and a short lane-split list."""
    for n, count, seed in ((1000, None, 31), (20000, 300, 32), (5000, 37, 33)):
        x, v, m = plummer(n, seed)
        idx = None if count is None else sample_indices(n, count, seed)
        got = nbody.force_on_state(x, v, m, eps, "fp32all", idx=idx)
        xr, vr, mr = (np.asarray(a, np.float32).astype(np.float64) for a in (x, v, m))
        ref, scale = reference(xr, vr, mr, eps * eps, idx=idx)
        check("fp32all", got, ref, scale, f"N={n} eps={eps}")
        exact = oracle.force(x, v, m, eps * eps, idx=idx)
        print(f"  against unrounded inputs: e_acc={rms_rel(got[0], exact[0]):.3e}", flush=True)


@pytest.mark.parametrize("prec", ["fp32", "ds", "fp64", "fp32fixed", "fp32all"])
def test_force_scalar_load_and_lds_paths(prec):
    """All i at N = 4999 (19 full j-tiles and a ragged tail of 135), once with 8 work items
    (one j-range of 20 tiles per item: the float modes read the j-records with scalar loads)
    and once with 400 (20 i-blocks of 256 against 20 j-ranges of one tile: LDS tiles with the
    scalar-load threshold at 16 tiles, scalar loads with it at 1, the ragged last tile read
    that way too; one lane per i throughout).  All meet the tolerances against
    the oracle (fp32all: against the oracle on float-rounded inputs); the first two differ only
    in how the per-tile sums are grouped, so they agree to 1e-11 relative (fp32all, whose sums
    stay in float: 1e-6; fp32fixed: bitwise); the last two group them alike and agree
    bitwise."""
    import torch
    n, eps = 4999, 1 / 256
    x, v, m = plummer(n, 34)
    st = nbody.DeviceState(x, v, m)
    res = []
    with nbody.Context(n, eps, precision=prec) as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        for target, st_min in ((8, 16), (400, 16), (400, 1)):
            ctx.nb_set_variant(0, dict(ipl=1, unroll=2, target=target, kmax=64,
                                       scalar_tiles=st_min))
            acc = torch.zeros((3, n), dtype=torch.float64, device="cuda")
            jerk = torch.zeros_like(acc)
            pot = torch.zeros(n, dtype=torch.float64, device="cuda")
            ctx.nb_force(acc, jerk, pot)
            ctx.nb_sync()
            res.append((acc.cpu().numpy().T.copy(), jerk.cpu().numpy().T.copy(), pot.cpu().numpy()))
    if prec == "fp32all":
        xr, vr, mr = (np.asarray(a, np.float32).astype(np.float64) for a in (x, v, m))
        ref, scale = reference(xr, vr, mr, eps * eps)
    else:
        ref, scale = reference(x, v, m, eps * eps)
    tol_key = "fp32" if prec == "fp32fixed" else prec
    for r, label in zip(res, ("scalar-load path", "LDS path", "one-tile scalar-load path")):
        check(tol_key, r, ref, scale, f"N={n} {label}")
    for c in range(3):
        if prec == "fp32fixed":
            assert np.array_equal(res[0][c], res[1][c]), c
        else:
            lim = 1e-6 if prec == "fp32all" else 1e-11
            assert rms_rel(res[0][c], res[1][c]) <= lim, (c, rms_rel(res[0][c], res[1][c]))
        assert np.array_equal(res[1][c], res[2][c]), c
