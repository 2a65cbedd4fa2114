"""Order-independent single precision (fp32fixed): float sums over aligned 64-j sub-blocks added
into int64 fixed point.  Its forces must be bitwise identical for every launch variant (i per
lane 1 or 2, unroll 1 or 2), every work-item target (which changes the j-split K, for short
lists the lane split), whether an item reads its j-records with scalar loads or stages them in
LDS (scalar_tiles 1 or 16 against items of 1 to 20 tiles), and between the full-force and
block-step launch classes; they must
meet the single-precision tolerances against the oracle, also on a sample that reaches the
halo, where accelerations and jerks are small (the fixed-point steps, 2^-44 for acc and pot and
2^-42 for the jerk, add rounding of about one step times sqrt(N/64): near 1e-11 absolute at
N = 2^20); and sums outside the fixed-point range must be reported, not wrapped.
"""
import numpy as np
import pytest
import torch

from paper_astro_ph_0702058_amd import nbody
from paper_astro_ph_0702058_amd.plummer import plummer, sample_indices
from _parity import check, reference

pytestmark = pytest.mark.gpu

VARIANTS = [dict(ipl=i, unroll=u, target=t, kmax=65536, scalar_tiles=s)
            for i in (1, 2) for u in (1, 2) for t in (8, 256, 4096) for s in (1, 16)]


def forces(ctx, n, idx, which):
    """Force on the listed i through the block-step class (device count) or the full class."""
    acc = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    jerk = torch.zeros_like(acc)
    pot = torch.zeros(n, dtype=torch.float64, device="cuda")
    if which == 1:
        ii = torch.as_tensor(idx.astype(np.int32), device="cuda")
        cnt = torch.tensor([idx.size], dtype=torch.int32, device="cuda")
        ctx.nb_force(acc, jerk, pot, i_idx=ii, n_i=cnt)
    else:
        ii = torch.as_tensor(idx.astype(np.int32), device="cuda")
        a2 = torch.zeros((3, idx.size), dtype=torch.float64, device="cuda")
        k2 = torch.zeros_like(a2)
        p2 = torch.zeros(idx.size, dtype=torch.float64, device="cuda")
        ctx.nb_force(a2, k2, p2, i_idx=ii)
        acc[:, :idx.size] = a2; jerk[:, :idx.size] = k2; pot[:idx.size] = p2
    ctx.nb_sync()
    return (acc[:, :idx.size].cpu().numpy().T.copy(), jerk[:, :idx.size].cpu().numpy().T.copy(),
            pot[:idx.size].cpu().numpy().copy())


@pytest.mark.parametrize("eps", [1 / 256, 0.0])
@pytest.mark.parametrize("count", [3, 37, 200, 700, 5001])
def test_bitwise_identical_across_variants(eps, count):
    n = 5001
    x, v, m = plummer(n, 41)
    idx = np.arange(n) if count == n else sample_indices(n, count, 7 + count)
    st = nbody.DeviceState(x, v, m)
    results = []
    with nbody.Context(n, eps, precision="fp32fixed") as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        for var in VARIANTS:
            for which in (0, 1):
                ctx.nb_set_variant(which, var)
                results.append((var, which, forces(ctx, n, idx, which)))
    ref, scale = reference(x, v, m, eps * eps, idx=idx)
    first = results[0][2]
    check("fp32", first, ref, scale, f"fp32fixed count={count} eps={eps}")
    for var, which, got in results[1:]:
        for c in range(3):
            assert np.array_equal(got[c], first[c]), (var, which, c)


def test_full_size_sampled_and_same_as_block_class():
    """N = 2^20, eps = 1/256: the all-i launch (j-split K = 2 at the default 16 items per CU)
    and a 2048-particle list through the block class give bitwise the same rows; both meet
    the tolerances against the oracle on that uniform sample (halo particles included)."""
    n = 1 << 20
    x, v, m = plummer(n, 3)
    idx = np.sort(sample_indices(n, 2048, 21))
    st = nbody.DeviceState(x, v, m)
    with nbody.Context(n, 1 / 256, precision="fp32fixed") as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        acc = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        jerk = torch.zeros_like(acc); pot = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.nb_force(acc, jerk, pot)
        ctx.nb_sync()
        ii = torch.as_tensor(idx, device="cuda")
        full = (acc[:, ii].cpu().numpy().T, jerk[:, ii].cpu().numpy().T, pot[ii].cpu().numpy())
        blk = forces(ctx, n, idx, 1)
    ref, scale = reference(x, v, m, (1 / 256) ** 2, idx=idx)
    check("fp32", full, ref, scale, "fp32fixed N=2^20")
    for c in range(3):
        assert np.array_equal(full[c], blk[c]), c


def test_range_overflow_is_reported():
    """Unsoftened pair at separation 1e-4 with unit masses: |acc| = 1e8 > 2^19, outside the
    fixed-point range; the result is poisoned and the next synchronising call reports it."""
    x = np.array([[0.0, 0.0, 0.0], [1e-4, 0.0, 0.0], [1.0, 1.0, 1.0]])
    v = np.zeros((3, 3)); m = np.ones(3)
    st = nbody.DeviceState(x, v, m)
    with nbody.Context(3, 0.0, precision="fp32fixed") as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        acc = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
        jerk = torch.zeros_like(acc); pot = torch.zeros(3, dtype=torch.float64, device="cuda")
        ctx.nb_force(acc, jerk, pot)
        with pytest.raises(nbody.NBodyError) as e:
            ctx.nb_sync()
        assert e.value.status == nbody.NB_ENONFINITE
        a = acc.cpu().numpy()
    assert np.all(np.isnan(a[:, :2])) and np.all(np.isfinite(a[:, 2]))
