"""GPU parity of the batched multi-lattice path (lattices of different
sizes and hopping parameters, uneven right-hand-side counts).

* batch_wilson_apply: one persistent launch per half hop over every
  lattice's fields (or one link-tiled launch per lattice) equals the
  oracle's even/odd operator (FP32 rounding);
* batch_solve (eager and hipGraph-captured cycles, right-hand-side blocks
  that mix lattices, both stencil forms; with link tiles the blocks' lattice
  runs change from block to block, so the captured cycle is recorded
  again): every solution equals dense LU to 1e-9 with an FP64 true residual
  below the tolerance, and the captured and eager runs give the same
  iteration counts and bitwise equal solutions;
* batch_autotune returns one of its candidates and a rate for each.
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, context, to_gpu, to_host, say, rel_err
from oracle import wilson as W
from oracle.noise import z4_noise

pytestmark = pytest.mark.gpu

LATS = [((4, 4, 4, 4), 0.12, 5, 1001), ((6, 4, 2, 8), 0.13, 3, 1002), ((4, 4, 2, 4), 0.125, 4, 1003)]


def _setup(lats):
    ctxs, Us, defls, etas = [], [], [], []
    for dims, kappa, nr, seed in lats:
        ctx, U = context(dims, 0.3, seed, kappa)
        say("batch setup deflation", dims, kappa)
        eta0 = z4_noise(seed + 5000, dims, 0, 1)
        _, defl, _ = ctx.gmresdr_solve(to_gpu(eta0), op="schur", m=20, k=10, tol=1e-12, tol_super=1e-13)
        ctxs.append(ctx)
        Us.append(U)
        defls.append(defl)
        etas.append(z4_noise(seed + 7000, dims, 0, nr))
    return ctxs, Us, defls, etas


@pytest.mark.parametrize("tile", [0, 32])
def test_batch_wilson_apply(tile):
    require_gpu()
    from paper_1903_06986_amd import Batch
    lats = LATS + [((2, 2, 2, 4), 0.1, 2, 1004)]
    rng = np.random.default_rng(8)
    ctxs, Us, xs = [], [], []
    for dims, kappa, nr, seed in lats:
        ctx, U = context(dims, 0.3, seed, kappa)
        ctxs.append(ctx)
        Us.append(U)
        xs.append(rng.standard_normal((nr,) + ctx.shape) + 1j * rng.standard_normal((nr,) + ctx.shape))
    batch = Batch(ctxs)
    batch.set_tile(tile)
    say("batch wilson apply", [l[0] for l in lats], "tile", tile)
    ys = batch.wilson_apply([to_gpu(x) for x in xs])
    for (dims, kappa, nr, seed), U, x, y in zip(lats, Us, xs, ys):
        ref = W.apply_Mhat(U, kappa, x, dims)
        assert rel_err(to_host(y), ref) < 5e-6, dims


@pytest.mark.parametrize("tile", [0, 16])
@pytest.mark.parametrize("graph", [True, False])
def test_batch_solve(graph, tile):
    require_gpu()
    from paper_1903_06986_amd import Batch
    ctxs, Us, defls, etas = _setup(LATS)
    batch = Batch(ctxs)
    batch.set_tile(tile)
    say("batch solve graph=%s tile=%d" % (graph, tile))
    xs, st = batch.solve([to_gpu(e) for e in etas], defls, m=20, k=10, tol=1e-11, inner_tol=1e-4,
                         rhs_block=4, graph=graph)
    i = 0
    for (dims, kappa, nr, seed), U, eta, x in zip(LATS, Us, etas, xs):
        M = W.dense_M(U, kappa, dims)
        xref = np.linalg.solve(M, eta.reshape(nr, -1).T).T.reshape(eta.shape)
        xg = to_host(x)
        for r in range(nr):
            assert rel_err(xg[r], xref[r]) < 1e-9, (dims, r)
            assert st[i]["true_resid"] < 1e-11, (dims, r, st[i])
            assert st[i]["refinements"] >= 1
            i += 1


@pytest.mark.parametrize("tile", [0, 32])
def test_batch_graph_matches_eager(tile):
    require_gpu()
    from paper_1903_06986_amd import Batch
    ctxs, Us, defls, etas = _setup(LATS)
    batch = Batch(ctxs)
    batch.set_tile(tile)
    say("batch graph vs eager tile", tile)
    xa, sa = batch.solve([to_gpu(e) for e in etas], defls, tol=1e-11, rhs_block=5, graph=True)
    xb, sb = batch.solve([to_gpu(e) for e in etas], defls, tol=1e-11, rhs_block=5, graph=False)
    assert [s["matvecs"] for s in sa] == [s["matvecs"] for s in sb]
    for a, b in zip(xa, xb):
        assert np.array_equal(to_host(a), to_host(b))


def test_batch_autotune():
    require_gpu()
    from paper_1903_06986_amd import Batch
    ctxs, Us, defls, etas = _setup(LATS)
    batch = Batch(ctxs)
    say("batch autotune")
    blk, tile, table = batch.autotune([to_gpu(e) for e in etas], defls, tol=1e-10)
    assert blk in Batch.TUNE_BLOCKS and tile in Batch.TUNE_TILES
    assert set(table) == {(b, t) for b in Batch.TUNE_BLOCKS for t in Batch.TUNE_TILES}
    assert table[(blk, tile)] == max(table.values()) > 0
    assert all(v > 0 for (b, t), v in table.items() if b <= 12)
    with pytest.raises(Exception):
        batch.set_tile(24)
