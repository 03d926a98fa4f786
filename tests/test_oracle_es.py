"""Pins for the oracle's eigenvalue subtraction (ES, Sec. 5.3), CPU.

Fixed by dense linear algebra on a small lattice, independently of the
reconstruction formulas: the full pairs built from Mhat's eigenpairs are
right and left eigenpairs of the dense M (a wrong root, a missing kappa or
a dropped g5 in D_eo^+ breaks this); with both roots of every reduced mode
the subtraction matrix is M^{-1} itself and Tr = sum 1/lambda (the paper's
closed form); the Ritz pairs from the even/odd GMRES-DR data reach the
smallest eigenvalues of dense M; the per-timeslice trace equals the dense
trace of the subtraction matrix for all nine operators.
"""
import numpy as np
import pytest

from synth import random_su3_links
from oracle import lattice as L
from oracle import wilson as W
from oracle import krylov as K
from oracle import subtract as S
from oracle import pointsplit as PSO
from oracle import es as ES
from oracle.noise import z4_noise

DIMS = (4, 4, 2, 4)
KAPPA = 0.125


@pytest.fixture(scope="module")
def setup():
    U = random_su3_links(DIMS, 0.3, 31)
    M = W.dense_M(U, KAPPA, DIMS)
    ev, od = L.eo_tables(DIMS)
    idx_e = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in ev])
    idx_o = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in od])
    Mhat = np.eye(idx_e.size) - M[np.ix_(idx_e, idx_o)] @ M[np.ix_(idx_o, idx_e)]
    return U, M, idx_e, Mhat


def _embed(vecs_e, idx_e, n):
    out = np.zeros((n, vecs_e.shape[1]), dtype=np.complex128)
    out[idx_e] = vecs_e
    return out


def _dense_reduced_pairs(M, idx_e, Mhat):
    lh, Sr = np.linalg.eig(Mhat)
    Sl = np.linalg.inv(Sr).conj().T
    n = M.shape[0]
    return lh, _embed(Sr, idx_e, n), _embed(Sl, idx_e, n)


@pytest.mark.parametrize("branch", [1, -1])
def test_full_pairs_are_eigenpairs_of_M(setup, branch):
    U, M, idx_e, Mhat = setup
    lh, Rh, Lh = _dense_reduced_pairs(M, idx_e, Mhat)
    q = np.argsort(np.abs(lh))[:8]
    lam, R, Lv = ES.full_pairs(U, KAPPA, DIMS, lh[q], Rh[:, q], Lh[:, q], branch=branch)
    Rf, Lf = R.reshape(len(q), -1), Lv.reshape(len(q), -1)
    spec = np.linalg.eigvals(M)
    for i in range(len(q)):
        r, l = Rf[i], Lf[i]
        assert np.linalg.norm(M @ r - lam[i] * r) < 1e-10 * np.linalg.norm(r)
        assert np.linalg.norm(l.conj() @ M - lam[i] * l.conj()) < 1e-10 * np.linalg.norm(l)
        assert abs(np.vdot(l, r) - 1) < 1e-10
        assert np.min(np.abs(spec - lam[i])) < 1e-10


def test_all_pairs_give_the_inverse(setup):
    U, M, idx_e, Mhat = setup
    lh, Rh, Lh = _dense_reduced_pairs(M, idx_e, Mhat)
    a = ES.full_pairs(U, KAPPA, DIMS, lh, Rh, Lh, branch=1)
    b = ES.full_pairs(U, KAPPA, DIMS, lh, Rh, Lh, branch=-1)
    lam = np.concatenate([a[0], b[0]])
    R = np.concatenate([a[1], b[1]])
    Lv = np.concatenate([a[2], b[2]])
    assert lam.size == M.shape[0]
    eta = z4_noise(3, DIMS, 0, 2)
    xt = ES.es_vector(R, Lv, lam, eta)
    x = np.linalg.solve(M, eta.reshape(2, -1).T).T.reshape(eta.shape)
    assert np.abs(xt - x).max() < 1e-10 * np.abs(x).max()
    # the paper's closed form of the trace, and the per-timeslice scalar trace
    Minv = np.linalg.inv(M)
    assert abs(np.sum(1.0 / lam) - np.trace(Minv)) < 1e-10 * abs(np.trace(Minv))
    tr = ES.es_trace(U, KAPPA, R, Lv, lam, (0,), DIMS)
    assert np.abs(tr[0] - S.trace_correction_dense(Minv, DIMS, (0,))[0]).max() < 1e-10


def test_ritz_pairs_from_gmres_dr_data(setup):
    U, M, idx_e, Mhat = setup
    shape = (DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 3)
    Ahat = lambda v: W.apply_Mhat(U, KAPPA, v.reshape(shape), DIMS).ravel()
    eta = z4_noise(5, DIMS, 0, 1)[0]
    src = W.eo_source(U, KAPPA, eta, DIMS).ravel()
    _, info = K.gmres_dr(Ahat, src, 40, 20, 1e-13, max_cycles=300, eig_tol=1e-11, n_eig=10)
    g5 = lambda v: W.g5(v.reshape(shape)).ravel()
    lh, Rh, Lh = ES.ritz_pairs_eo(info["V"], info["H"], g5)
    assert np.abs(np.diag(Lh.conj().T @ Rh) - 1).max() < 1e-12
    lam, R, Lv = ES.smallest(*ES.full_pairs(U, KAPPA, DIMS, lh, Rh, Lh), 6)
    spec = np.linalg.eigvals(M)
    ref = spec[np.argsort(np.abs(spec))][:6]
    assert np.abs(np.sort_complex(lam) - np.sort_complex(ref)).max() < 1e-8
    Rf, Lf = R.reshape(6, -1), Lv.reshape(6, -1)
    for i in range(6):
        # right AND left eigenvectors of M (the left ones are not in the
        # Krylov space; they come from the g5 partner)
        assert np.linalg.norm(M @ Rf[i] - lam[i] * Rf[i]) < 1e-8 * np.linalg.norm(Rf[i])
        assert np.linalg.norm(Lf[i].conj() @ M - lam[i] * Lf[i].conj()) < 1e-8 * np.linalg.norm(Lf[i])
        assert abs(np.vdot(Lf[i], Rf[i]) - 1) < 1e-10


def test_trace_matches_dense_subtraction_matrix(setup):
    U, M, idx_e, Mhat = setup
    lh, Rh, Lh = _dense_reduced_pairs(M, idx_e, Mhat)
    lam, R, Lv = ES.smallest(*ES.full_pairs(U, KAPPA, DIMS, lh, Rh, Lh), 10)
    Rf, Lf = R.reshape(10, -1), Lv.reshape(10, -1)
    Mt = (Rf.T / lam) @ Lf.conj()
    th = tuple(range(9))
    tr = ES.es_trace(U, KAPPA, R, Lv, lam, th, DIMS)
    ref = np.concatenate([S.trace_correction_dense(Mt, DIMS, (0, 1, 2, 3, 4)),
                          np.stack([PSO.trace_ps_dense(U, KAPPA, DIMS, mu, Mt) for mu in range(4)])])
    assert np.abs(tr - ref).max() < 1e-10 * np.abs(ref).max()
    eta = z4_noise(9, DIMS, 0, 3)
    xt = ES.es_vector(R, Lv, lam, eta)
    assert np.abs(xt.reshape(3, -1) - (Mt @ eta.reshape(3, -1).T).T).max() < 1e-10 * np.abs(xt).max()
