"""GPU eigenvalue subtraction (ES, Sec. 5.3) against the oracle.

The GPU builds its eigenpairs of M from the Ritz pairs of the even/odd
GMRES-DR deflation space; the oracle builds them from the exact (dense)
eigenpairs of Mhat with the same reconstruction, so the comparison also
checks that the super-converged Ritz pairs are the low eigenpairs.  The
subtraction matrix sum_q r_q l_q^+ / lambda_q does not depend on how each
eigenvector is scaled, so xt and the trace corrections compare directly
(1e-8 relative, set by the eigen-residuals ~1e-11 over gaps ~1e-3); Q is
taken where |lambda| has a gap, so no complex-conjugate pair is split.
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, context, to_gpu, to_host, say
from oracle import lattice as L
from oracle import wilson as W
from oracle import es as ES
from oracle.noise import z4_noise

pytestmark = pytest.mark.gpu


def test_eigenvalue_subtraction_matches_oracle():
    require_gpu()
    import torch
    from paper_1903_06986_amd import lqcd
    dims, kappa = (4, 4, 2, 4), 0.125
    ctx, U = context(dims, 0.3, 31, kappa)
    M = W.dense_M(U, kappa, dims)
    ev, od = L.eo_tables(dims)
    idx_e = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in ev])
    idx_o = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in od])
    Mhat = np.eye(idx_e.size) - M[np.ix_(idx_e, idx_o)] @ M[np.ix_(idx_o, idx_e)]
    lh, Sr = np.linalg.eig(Mhat)
    Sl = np.linalg.inv(Sr).conj().T
    n = M.shape[0]
    Rh = np.zeros((n, lh.size), complex)
    Lh = np.zeros((n, lh.size), complex)
    Rh[idx_e], Lh[idx_e] = Sr, Sl
    lam_all, R_all, L_all = ES.full_pairs(U, kappa, dims, lh, Rh, Lh)
    a = np.sort(np.abs(lam_all))
    Q = next(q for q in range(4, 12) if a[q] - a[q - 1] > 1e-3 * a[q])
    lam_o, R_o, L_o = ES.smallest(lam_all, R_all, L_all, Q)
    eta = z4_noise(7, dims, 0, 3)
    say("ES: even/odd GMRES-DR", dims, "Q", Q)
    _, defl, _ = ctx.gmresdr_solve(to_gpu(eta[0:1]), op="schur", m=40, k=20, tol=1e-12, tol_super=1e-13,
                                   eig_tol=1e-11, n_eig=Q + 2, max_cycles=400)
    th = tuple(range(9))
    xt, corr, lam_g = ctx.deflate_project(defl, Q, to_gpu(eta), xt=torch.zeros_like(to_gpu(eta)),
                                          mode=lqcd.DEFL_ES, thetas=th)
    assert np.abs(np.sort_complex(lam_g) - np.sort_complex(lam_o)).max() < 1e-9
    xt_o = ES.es_vector(R_o, L_o, lam_o, eta)
    assert np.abs(to_host(xt) - xt_o).max() < 1e-8 * np.abs(xt_o).max()
    corr_o = ES.es_trace(U, kappa, R_o, L_o, lam_o, th, dims)
    assert np.abs(corr - corr_o).max() < 1e-8 * np.abs(corr_o).max()
    # accumulation into an existing xt / trace, and the scalar trace's closed form
    xt2, corr2, _ = ctx.deflate_project(defl, Q, to_gpu(eta), xt=to_gpu(xt_o), corr=corr_o, mode=lqcd.DEFL_ES,
                                        thetas=th)
    assert np.abs(to_host(xt2) - 2 * xt_o).max() < 1e-8 * np.abs(xt_o).max()
    assert abs(corr[0].sum() - np.sum(1.0 / lam_o)) < 1e-8 * abs(np.sum(1.0 / lam_o))


def test_eigenvalue_subtraction_rejects_hermitian_space():
    require_gpu()
    import torch
    from paper_1903_06986_amd import lqcd
    from paper_1903_06986_amd.lqcd import LqcdError
    dims = (4, 4, 2, 4)
    ctx, U = context(dims, 0.3, 31, 0.125)
    eta = z4_noise(7, dims, 0, 1)
    _, hdefl, _ = ctx.gmresdr_solve(to_gpu(eta), op="MG5", m=20, k=10, tol=1e-8, tol_super=1e-8,
                                    max_cycles=50)
    with pytest.raises(LqcdError):
        ctx.deflate_project(hdefl, 4, to_gpu(eta), xt=torch.zeros_like(to_gpu(eta)), mode=lqcd.DEFL_ES)
