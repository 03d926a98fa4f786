"""Two contexts of one lattice, each on its own stream, driven from two host
threads at once (as the benchmark's concurrent pipelines): the solves, the
subtraction vectors and the estimates equal, bit for bit, what the same
calls give one after the other.  The deflation spaces and the trace
corrections come from one context's setup and are shared; their caches are
filled either by a sequential pass first or by both threads at once."""
import threading

import numpy as np
import pytest

from tests.gpu_common import require_gpu, to_host, say

pytestmark = pytest.mark.gpu

THETAS = (0, 1, 2, 3, 4, 5, 6, 7, 8)


@pytest.mark.parametrize("cold", [False, True])
def test_two_pipelines_match_sequential(cold):
    """cold: the two threads start on deflation spaces whose caches (the
    FP32 copy, eigenpairs, trace bilinears, lexicographic copies) are still
    empty, so they fill them at the same time; the sequential reference runs
    afterwards."""
    require_gpu()
    import torch
    from paper_1903_06986_amd import Context, lqcd
    from synth import random_su3_links
    dims, kappa = (6, 4, 2, 8), 0.13
    U = random_su3_links(dims, 0.3, 1001)
    ctxs = [Context(dims, U, kappa, stream=torch.cuda.Stream()) for _ in range(2)]
    with torch.cuda.stream(ctxs[0].stream):
        eta0 = ctxs[0].noise_z4(7, 0, 1)
        _, defl, _ = ctxs[0].gmresdr_solve(eta0, op="schur", m=20, k=10, tol=1e-11, tol_super=1e-13)
        _, hdefl, _ = ctxs[0].gmresdr_solve(eta0, op="MG5", m=30, k=15, tol=1e-11, tol_super=1e-12,
                                            n_eig=8, max_cycles=400, method="minres-dr")
        _, corr = ctxs[0].pert_subtract(4, eta0, THETAS)
        ctxs[0].stream.synchronize()

    def pipeline(ctx, first):
        with torch.cuda.stream(ctx.stream):
            eta = ctx.noise_z4(7, first, 4)
            x, _, st = ctx.gmresdr_solve(eta, op="schur", m=20, k=10, tol=1e-11, inner="f16", inner_tol=1e-4,
                                         rhs_block=4, defl=defl)
            xt, _ = ctx.pert_subtract(4, eta, THETAS, want_corr=False)
            est, err = ctx.loop_estimate(eta, x, xt, corr, THETAS)[:2]
            xh, ch, _ = ctx.deflate_project(hdefl, 6, eta, xt=xt, corr=corr, mode=lqcd.DEFL_EIGPOLY,
                                            coeffs=np.ones(5, dtype=np.complex128), thetas=THETAS)
            esth = ctx.loop_estimate(eta, x, xh, ch, THETAS)[0]
            ctx.stream.synchronize()
            return (to_host(x), to_host(xt), np.asarray(est), np.asarray(err), np.asarray(esth),
                    [s["matvecs"] for s in st])

    ref = None
    if not cold:
        say("sequential pipelines")
        ref = [pipeline(ctxs[i], 1 + 100 * i) for i in range(2)]
    out = [[], []]
    errs = []

    def run(i):
        try:
            for _ in range(3):
                out[i].append(pipeline(ctxs[i], 1 + 100 * i))
        except BaseException as e:  # noqa: BLE001 - reported below
            errs.append(e)

    say("concurrent pipelines")
    threads = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errs, errs
    if cold:
        say("sequential pipelines")
        ref = [pipeline(ctxs[i], 1 + 100 * i) for i in range(2)]
    for i in range(2):
        assert len(out[i]) == 3
        for rep in out[i]:
            for a, b in zip(rep[:5], ref[i][:5]):
                np.testing.assert_array_equal(a, b)
            assert rep[5] == ref[i][5]
