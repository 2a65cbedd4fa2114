"""The no-allocation force entry point (nb_force_noalloc) against nb_force through the C ABI:
the same kernels and plan with the j-split partial sums in the library's static device array
instead of the context's workspace, so the results must be bitwise equal; two calls in a row,
the second on a smaller list, for host- and device-held counts; a call whose j-split would not
fit the array is refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_astro_ph_0702058_amd import nbody
from paper_astro_ph_0702058_amd.plummer import plummer, sample_indices

pytestmark = pytest.mark.gpu


def _outs(k):
    a = torch.zeros((3, k), dtype=torch.float64, device="cuda")
    return a, torch.zeros_like(a), torch.zeros(k, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("prec", ["fp32", "ds", "fp64", "fp32fixed"])
def test_noalloc_force_equals_nb_force(prec):
    n = 20000
    x, v, m = plummer(n, 51)
    st = nbody.DeviceState(x, v, m)
    with nbody.Context(n, 1 / 256, precision=prec) as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        for count in (3000, 700, 37):   # host count: j-split lists, then the lane split
            ii = torch.as_tensor(sample_indices(n, count, count).astype(np.int32), device="cuda")
            ref, got = _outs(count), _outs(count)
            ctx.nb_force(*ref, i_idx=ii)
            ctx.nb_force_noalloc(*got, i_idx=ii)
            ctx.nb_sync()
            for r, g in zip(ref, got):
                assert torch.equal(r, g), (prec, count)
            assert torch.all(ref[0] != 0)
        for count in (900, 200):         # device count, the block-step launch class
            ii = torch.as_tensor(sample_indices(n, count, 7 + count).astype(np.int32), device="cuda")
            cnt = torch.tensor([count], dtype=torch.int32, device="cuda")
            ref, got = _outs(n), _outs(n)
            ctx.nb_force(*ref, i_idx=ii, n_i=cnt)
            ctx.nb_force_noalloc(*got, i_idx=ii, n_i=cnt)
            ctx.nb_sync()
            for r, g in zip(ref, got):
                assert torch.equal(r, g), (prec, count)
            assert torch.all(got[0][:, :count] != 0) and torch.all(got[0][:, count:] == 0)


def test_noalloc_refuses_a_split_beyond_the_array():
    """A full force on 200000 particles splits j into 64 ranges: 64 * 200192 partial rows of 7
    doubles (717 MB) exceed the 64 MiB array; the call is refused with NB_EINVAL and the context
    keeps working (nb_force on the same arguments, and a small noalloc list after it)."""
    n = 200000
    x, v, m = plummer(n, 52)
    st = nbody.DeviceState(x, v, m)
    with nbody.Context(n, 1 / 256, precision="fp32") as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        outs = _outs(n)
        with pytest.raises(nbody.NBodyError) as e:
            ctx.nb_force_noalloc(*outs)
        assert e.value.status == nbody.NB_EINVAL and "static array" in str(e.value)
        ctx.nb_force(*outs)
        ii = torch.as_tensor(np.arange(0, n, 997, dtype=np.int32), device="cuda")
        ref, got = _outs(ii.numel()), _outs(ii.numel())
        ctx.nb_force(*ref, i_idx=ii)
        ctx.nb_force_noalloc(*got, i_idx=ii)
        ctx.nb_sync()
        for r, g in zip(ref, got):
            assert torch.equal(r, g)
