"""GPU parity of poly_subtract_multi (several polynomial subtraction vectors
of one noise from one chain of powers of kappa P; Sec. 5.1 Eq. (31), Sec.
5.2 Eq. (40)) against the oracle's Horner evaluation and against
pert_subtract / poly_subtract.

Tolerance 1e-12 relative, the bar of the single-polynomial calls' own
parity tests: the powers are summed in order of j instead of by Horner's
rule, so the vectors differ from theirs by rounding only.  Blocks of 16
right-hand sides: 18 noise vectors cover a full block and a ragged one.
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, context, to_gpu, to_host, say, rel_err
from oracle import subtract as S
from oracle.noise import z4_noise

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,n", [((4, 4, 2, 6), 18), ((2, 2, 2, 4), 3)])
def test_poly_multi_matches_oracle_and_single_calls(dims, n):
    require_gpu()
    kappa = 0.12
    ctx, U = context(dims, 0.3, 41, kappa)
    eta = z4_noise(6, dims, 0, n)
    rng = np.random.default_rng(2)
    polys = [S.pert_coeffs(7),
             rng.standard_normal(8) + 1j * rng.standard_normal(8),
             rng.standard_normal(4) + 1j * rng.standard_normal(4),   # degree 3, padded
             np.array([0.5 - 0.25j])]                                  # degree 0
    say("poly_subtract_multi", dims, n)
    outs = ctx.poly_subtract_multi(to_gpu(eta), polys)
    for c, xt in zip(polys, outs):
        ref = S.horner(U, kappa, eta, c)
        assert rel_err(to_host(xt), ref) < 1e-12
    ps, _ = ctx.pert_subtract(7, to_gpu(eta), want_corr=False)
    assert rel_err(to_host(outs[0]), to_host(ps)) < 1e-12
    po, _, _, _ = ctx.poly_subtract(7, to_gpu(eta), coeffs=polys[1], want_corr=False)
    assert rel_err(to_host(outs[1]), to_host(po)) < 1e-12


def test_poly_multi_edges():
    require_gpu()
    import torch
    from paper_1903_06986_amd import lqcd
    from paper_1903_06986_amd.lqcd import LqcdError
    dims = (2, 2, 2, 4)
    ctx, U = context(dims, 0.3, 3, 0.1)
    eta = z4_noise(1, dims, 0, 2)
    # one polynomial of degree 0 only: no hopping step
    out = ctx.poly_subtract_multi(to_gpu(eta), [np.array([2.0 + 0j])])
    assert rel_err(to_host(out[0]), 2.0 * eta) < 1e-15
    # no right-hand side: nothing to do, no error
    e0 = torch.zeros((0,) + ctx.shape, dtype=torch.complex128, device="cuda")
    assert ctx.poly_subtract_multi(e0, [np.ones(3)])[0].shape[0] == 0
    with pytest.raises(LqcdError):
        ctx.poly_subtract_multi(to_gpu(eta), [np.ones(2)] * 5)
    with pytest.raises(LqcdError):
        ctx.poly_subtract_multi(to_gpu(eta), [np.ones(9)])
    # a null output pointer is rejected before any kernel runs
    cf = np.ones((1, 2), dtype=np.complex128)
    ptrs = (lqcd._P * 1)(None)
    code = lqcd.lib().poly_subtract_multi(ctx.handle, 1, 1, cf.ctypes.data_as(lqcd._P),
                                          lqcd._ptr(to_gpu(eta)), ptrs, 2)
    assert code != 0
