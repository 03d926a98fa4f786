"""loop_estimate_noalloc (the estimator with its partial sums in the
library's fixed device scratch, for callers that cannot allocate) against
loop_estimate on the same inputs, called through the C ABI: two calls in a
row, the second with a smaller input (fewer right-hand sides, another
lattice), so that stale partial sums of the first call would show; and the
size limit reported as EINVAL before any device work."""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import require_gpu, context, to_gpu, say
from oracle.noise import z4_noise

pytestmark = pytest.mark.gpu

THETAS = (0, 1, 2, 3, 4, 5, 6, 7, 8)


def _call(fn, ctx, eta, x, xt, corr):
    from paper_1903_06986_amd import lqcd
    th = np.ascontiguousarray(np.asarray(THETAS, dtype=np.int32))
    n, Lt = eta.shape[0], ctx.dims[3]
    est = np.zeros((len(THETAS), Lt + 1), dtype=np.complex128)
    err = np.zeros((len(THETAS), Lt + 1, 2))
    smp = np.zeros((n, len(THETAS), Lt + 1), dtype=np.complex128)
    c = np.ascontiguousarray(corr)
    code = fn(ctx.handle, th.ctypes.data_as(ctypes.c_void_p), len(THETAS), lqcd._ptr(eta), lqcd._ptr(x),
              lqcd._ptr(xt), n, c.ctypes.data_as(ctypes.c_void_p), est.ctypes.data_as(ctypes.c_void_p),
              err.ctypes.data_as(ctypes.c_void_p), smp.ctypes.data_as(ctypes.c_void_p))
    return code, est, err, smp


@pytest.mark.parametrize("first,second", [(((8, 8, 4, 8), 12), ((4, 4, 4, 4), 3)),
                                          (((6, 4, 2, 8), 7), ((6, 4, 2, 8), 2))])
def test_noalloc_matches_loop_estimate(first, second):
    require_gpu()
    from paper_1903_06986_amd import lqcd
    L = lqcd.lib()
    rng = np.random.default_rng(23)
    for dims, n in (first, second):
        ctx, U = context(dims, 0.3, 5, 0.12)
        eta = z4_noise(17, dims, 0, n)
        x = rng.standard_normal(eta.shape) + 1j * rng.standard_normal(eta.shape)
        xt = rng.standard_normal(eta.shape) + 1j * rng.standard_normal(eta.shape)
        corr = rng.standard_normal((len(THETAS), dims[3])) + 1j * rng.standard_normal((len(THETAS), dims[3]))
        eg, xg, tg = to_gpu(eta), to_gpu(x), to_gpu(xt)
        say("loop_estimate_noalloc", dims, n)
        code0, e0, s0, m0 = _call(L.loop_estimate, ctx, eg, xg, tg, corr)
        code1, e1, s1, m1 = _call(L.loop_estimate_noalloc, ctx, eg, xg, tg, corr)
        assert code0 == 0 and code1 == 0
        # same kernels and chunking at these sizes: the same sums in the same order
        assert np.array_equal(m0, m1) and np.array_equal(e0, e1) and np.array_equal(s0, s1)
        ctx.close()


def test_noalloc_rejects_more_partial_sums_than_its_scratch():
    require_gpu()
    from paper_1903_06986_amd import lqcd
    dims = (2, 2, 2, 64)      # Lt = 64, 10 partial-sum slots: at most 409 right-hand sides fit
    ctx, U = context(dims, 0.3, 5, 0.12)
    n = 410
    eta = to_gpu(z4_noise(3, dims, 0, n))
    say("loop_estimate_noalloc oversize", dims, n)
    code, _, _, _ = _call(lqcd.lib().loop_estimate_noalloc, ctx, eta, eta, None, np.zeros((9, 64), complex))
    assert code == 1 and b"scratch" in lqcd.lib().lqcd_last_error()
    code, _, _, _ = _call(lqcd.lib().loop_estimate_noalloc, ctx, eta[:409], eta[:409], None,
                          np.zeros((9, 64), complex))
    assert code == 0
