"""GPU parity of the point-split vector operator (operator codes 5..8,
mu = x, y, z, t; Table 2) against the oracle.

* loop_estimate samples and estimates against the oracle's estimator;
* exact trace corrections of PS and POLY (closed walks up to length 8,
  windings on extents of 2 included) against dense traces;
* hermitian-forced corrections against the dense eigenpairs' bilinears;
* a mixed request of local and point-split codes keeps both right.
Tolerances as for the local operators (rounding: 1e-12 on the estimator,
1e-10 on traces, 1e-9 with independently computed eigenvectors).
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, context, to_gpu, to_host, say, rel_err
from oracle import lattice as L
from oracle import wilson as W
from oracle import subtract as S
from oracle import krylov as K
from oracle import estimate as E
from oracle import pointsplit as PSO
from oracle.noise import z4_noise

pytestmark = pytest.mark.gpu

PS = (5, 6, 7, 8)


@pytest.mark.parametrize("dims", [(4, 2, 6, 4), (2, 2, 2, 4)])
def test_loop_estimate_point_split(dims):
    require_gpu()
    kappa = 0.11
    ctx, U = context(dims, 0.3, 3, kappa)
    rng = np.random.default_rng(8)
    shape = (4,) + ctx.shape
    eta = z4_noise(4, dims, 0, 4)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    xt = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    corr = rng.standard_normal((4, dims[3])) + 1j * rng.standard_normal((4, dims[3]))
    say("loop_estimate point-split", dims)
    est, err, smp = ctx.loop_estimate(to_gpu(eta), to_gpu(x), to_gpu(xt), corr, PS, samples=True)
    t = PSO.samples_ps(U, kappa, eta, x, xt, range(4), dims)
    e_ref, s_ref = E.estimate(t, corr)
    assert np.abs(smp - t).max() < 1e-12 * np.abs(t).max()
    assert np.abs(est - e_ref).max() < 1e-12 * np.abs(e_ref).max()
    assert np.abs(err - s_ref).max() < 1e-12 * np.abs(s_ref).max()
    # mixed local and point-split codes, in any order
    mixed = (7, 0, 5, 4)
    est2, _, smp2 = ctx.loop_estimate(to_gpu(eta), to_gpu(x), to_gpu(xt), None, mixed, samples=True)
    tl = E.samples(eta, x, xt, (0, 4), dims)
    assert np.abs(smp2[:, 1] - tl[:, 0]).max() < 1e-12 * np.abs(tl).max()
    assert np.abs(smp2[:, 3] - tl[:, 1]).max() < 1e-12 * np.abs(tl).max()
    assert np.abs(smp2[:, 0] - t[:, 2]).max() < 1e-12 * np.abs(t).max()
    assert np.abs(smp2[:, 2] - t[:, 0]).max() < 1e-12 * np.abs(t).max()


@pytest.mark.parametrize("dims", [(4, 4, 2, 4), (2, 2, 2, 4), (4, 2, 2, 2)])
def test_trace_corrections_point_split(dims):
    require_gpu()
    kappa = 0.12
    ctx, U = context(dims, 0.3, 21, kappa)
    Pd = W.dense_P(U, dims)
    eta = z4_noise(9, dims, 0, 2)
    say("pert_subtract point-split", dims)
    _, corr = ctx.pert_subtract(7, to_gpu(eta), PS)
    A = S.poly_dense(Pd, kappa, S.pert_coeffs(7))
    ref = np.stack([PSO.trace_ps_dense(U, kappa, dims, mu, A) for mu in range(4)])
    assert np.abs(corr - ref).max() < 1e-10 * np.abs(ref).max()
    say("poly_subtract point-split", dims)
    _, corr2, c, _ = ctx.poly_subtract(7, to_gpu(eta), b=to_gpu(eta[0:1]), thetas=PS)
    A2 = S.poly_dense(Pd, kappa, c)
    ref2 = np.stack([PSO.trace_ps_dense(U, kappa, dims, mu, A2) for mu in range(4)])
    assert np.abs(corr2 - ref2).max() < 1e-10 * np.abs(ref2).max()
    # the local codes are unchanged by the longer walk table
    _, corr3 = ctx.pert_subtract(7, to_gpu(eta), (0, 4))
    ref3 = S.trace_correction_dense(A, dims, (0, 4))
    assert np.abs(corr3 - ref3).max() < 1e-10 * np.abs(ref3).max()


def test_hermitian_forced_point_split():
    require_gpu()
    import torch
    dims, kappa, Q = (4, 4, 2, 4), 0.125, 6
    ctx, U = context(dims, 0.3, 31, kappa)
    eta = z4_noise(5, dims, 0, 2)
    say("deflate_project point-split", dims)
    _, hdefl, _ = ctx.gmresdr_solve(to_gpu(eta[0:1]), op="MG5", m=40, k=20, tol=1e-12, tol_super=1e-13,
                                    eig_tol=1e-11, n_eig=Q + 2, max_cycles=300)
    M = W.dense_M(U, kappa, dims)
    Mp = M @ W.dense_gamma(L.GAMMA5, L.volume(dims))
    lam, Ev = K.hermitian_eigpairs_dense(Mp, Q)
    Et = Ev.T.reshape((Q,) + eta[0].shape)
    _, corr, _ = ctx.deflate_project(hdefl, Q, to_gpu(eta), xt=torch.zeros_like(to_gpu(eta)), thetas=PS)
    ref = PSO.site_bilinear_ps(U, kappa, Et, range(4), dims, 1.0 / lam + 0j)
    assert np.abs(corr - ref).max() < 1e-9 * np.abs(ref).max()
