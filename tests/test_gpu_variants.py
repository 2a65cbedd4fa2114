"""Every compiled force-kernel launch variant computes the same sums (to the precision's
tolerance against the oracle), with and without a j-split; the autotuner picks a valid one."""
import numpy as np
import pytest
import torch

from paper_astro_ph_0702058_amd import nbody
from paper_astro_ph_0702058_amd.plummer import plummer, sample_indices
from _parity import check, reference

pytestmark = pytest.mark.gpu

F32 = [(i, u) for i in (1, 2) for u in (1, 2, 4)] + [(4, 1), (4, 2)]
OTHER = [(1, u) for u in (1, 2)]
CASES = [("fp32",) + c for c in F32] + [("ds",) + c for c in OTHER] + [("fp64",) + c for c in OTHER]


@pytest.mark.parametrize("prec,ipl,unr", CASES)
@pytest.mark.parametrize("target", [8, 1024])
@pytest.mark.parametrize("count", [37, 700])
@pytest.mark.parametrize("scalar_tiles", [1, 16])
def test_variant_parity(prec, ipl, unr, target, count, scalar_tiles):
    """700 listed i: whole i-blocks of the variant; 37: the lane split, which every variant
    takes for lists shorter than a workgroup.  N = 3001 is 12 j-tiles: with scalar_tiles 1 the
    float modes read every item's j-records with scalar loads (a one-tile item at target 1024,
    the ragged last tile included), with 16 every item stages LDS tiles."""
    n = 3001
    x, v, m = plummer(n, 31)
    eps = 1 / 256
    idx = sample_indices(n, count, 3).astype(np.int32)
    st = nbody.DeviceState(x, v, m)
    with nbody.Context(n, eps, precision=prec) as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        var = dict(ipl=ipl, unroll=unr, target=target, kmax=65536, scalar_tiles=scalar_tiles)
        ctx.nb_set_variant(1, var)
        assert ctx.nb_get_variant(1) == var
        ii = torch.as_tensor(idx, device="cuda")
        cnt = torch.tensor([idx.size], dtype=torch.int32, device="cuda")
        acc = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        jerk = torch.zeros_like(acc); pot = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.nb_force(acc, jerk, pot, i_idx=ii, n_i=cnt)   # device count -> block variant
        ctx.nb_sync()
    ref, scale = reference(x, v, m, eps * eps, idx=idx)
    got = (acc[:, :idx.size].cpu().numpy().T, jerk[:, :idx.size].cpu().numpy().T,
           pot[:idx.size].cpu().numpy())
    check(prec, got, ref, scale,
          f"ipl={ipl} unroll={unr} target={target} count={count} scalar_tiles={scalar_tiles}")
    assert np.all(acc[:, idx.size:].cpu().numpy() == 0)   # rows beyond the count untouched


def test_set_variant_rejects_unavailable():
    x, v, m = plummer(512, 32)
    with nbody.Context(512, 0.01, precision="ds") as ctx:
        with pytest.raises(nbody.NBodyError):
            ctx.nb_set_variant(0, dict(ipl=2, unroll=2, target=64, kmax=256))   # ds: ipl 1 only
        with pytest.raises(nbody.NBodyError):
            ctx.nb_set_variant(0, dict(ipl=1, unroll=3, target=64, kmax=256))
        with pytest.raises(nbody.NBodyError):
            ctx.nb_set_variant(0, dict(ipl=1, unroll=2, target=10 ** 7, kmax=256))
        with pytest.raises(nbody.NBodyError):
            ctx.nb_set_variant(0, dict(ipl=1, unroll=2, target=64, kmax=10 ** 6))
        with pytest.raises(nbody.NBodyError):
            ctx.nb_set_variant(0, dict(ipl=1, unroll=2, target=64, kmax=256, scalar_tiles=-1))
        # absent (or 0): the context keeps its current scalar-load threshold
        before = ctx.nb_get_variant(0)["scalar_tiles"]
        ctx.nb_set_variant(0, dict(ipl=1, unroll=2, target=64, kmax=256))
        assert ctx.nb_get_variant(0) == dict(ipl=1, unroll=2, target=64, kmax=256,
                                             scalar_tiles=before)


def test_tuner_picks_a_working_variant():
    n = 20000
    x, v, m = plummer(n, 33)
    st = nbody.DeviceState(x, v, m)
    with nbody.Context(n, 1 / 256, precision="fp32") as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        from paper_astro_ph_0702058_amd.tuning import autotune, expected_block_size
        chosen = autotune(ctx, cache_path=None, reps=1)
        assert set(chosen) == {0, 1}
        assert ctx.nb_get_variant(0) == chosen[0] and ctx.nb_get_variant(1) == chosen[1]
        assert all(chosen[w]["scalar_tiles"] in (1, 4, 16) for w in (0, 1))
        assert expected_block_size(n) == round(0.2 * n ** 0.81)
        idx = sample_indices(n, 200, 4)
        acc = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        jerk = torch.zeros_like(acc); pot = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.nb_force(acc, jerk, pot)
        ctx.nb_sync()
        got = (acc.cpu().numpy().T[idx], jerk.cpu().numpy().T[idx], pot.cpu().numpy()[idx])
    ref, scale = reference(x, v, m, (1 / 256) ** 2, idx=idx)
    check("fp32", got, ref, scale, f"tuned {chosen}")
