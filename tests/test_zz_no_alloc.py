"""ofdft_eval_noalloc (the evaluation with its intermediates in the library's static device
scratch array) against ofdft_eval on the same context and amplitude: two calls in a row on
one device, the second on a smaller grid, in FP64 and mixed precision; a grid whose
evaluation does not fit the array is refused."""
import numpy as np
import pytest

import workloads as wl
from paper_1406_0835_amd import binding as B

from _gpu_common import make_ctx, normalized_phi, oracle_system

pytestmark = pytest.mark.gpu

COMPONENTS = ("F_total", "E_internal", "F_s", "TS_s", "E_xc", "E_H", "E_ext", "E_alphaZ", "E_ion", "N_e", "mu",
              "residual", "TS_xc")


def _noalloc(ctx, phi):
    import torch
    d_phi = torch.from_numpy(np.ascontiguousarray(phi.ravel())).to("cuda")
    d_v = torch.full_like(d_phi, float("nan"))
    torch.cuda.synchronize()
    rep = ctx.eval_noalloc(d_phi.data_ptr(), d_v.data_ptr())
    return rep, d_v.cpu().numpy().reshape(phi.shape)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_eval_on_two_calls_second_smaller(precision):
    big = wl.h_cell(64, 1.0, (48, 48, 48), 5e4, seed=950)
    small = wl.h_cell(8, 1.0, (32, 24, 32), 2e5, seed=951)
    for cell, fn, xc in ((big, "VT84F", "PZ81"), (small, "SGA", "KSDT")):
        ctx = make_ctx(cell, fn, precision=precision, xc=xc)
        ctx.set_density(normalized_phi(oracle_system(cell, fn, xc=xc), seed=5, contrast=0.6))
        # the context's amplitude bit for bit (set_density renormalises on the host)
        phi = ctx.get_density()
        ref, v_ref = ctx.eval(potential=True)
        rep, v = _noalloc(ctx, phi)
        # the same kernels on the same input, with fixed-order reductions: identical results
        for k in COMPONENTS:
            assert getattr(rep, k) == getattr(ref, k), (cell.grid, k, getattr(rep, k), getattr(ref, k))
        assert np.array_equal(v, v_ref), (cell.grid, float(np.max(np.abs(v - v_ref))))
        # the context's own state is untouched: ofdft_eval still gives the same
        again, v_again = ctx.eval(potential=True)
        assert again.F_total == ref.F_total and np.array_equal(v_again, v_ref)
        ctx.close()


def test_noalloc_refuses_a_grid_beyond_the_scratch():
    cell = wl.h_cell(8, 1.0, (96, 96, 96), 5e4, seed=952)
    ctx = make_ctx(cell, "VT84F", precision="fp64")
    import torch
    d = torch.zeros(int(np.prod(cell.grid)), dtype=torch.float64, device="cuda")
    out = torch.empty_like(d)
    with pytest.raises(B.OFDFTError) as e:
        ctx.eval_noalloc(d.data_ptr(), out.data_ptr())
    assert e.value.code == B.E_ARG
    ctx.close()
