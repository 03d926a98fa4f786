"""Pins for the oracle's deflated Krylov solvers (CPU).

Fixed by dense linear algebra on small lattices: solutions vs LU, harmonic
Ritz values vs the smallest-|lambda| eigenvalues of Mhat, the Arnoldi
relation Mhat V_k = V_{k+1} Hbar_k, hermitian Ritz pairs of M' vs dense
eigh, and the free-field M' spectrum in closed form.  Iteration counts are
parity-unpinned (rounding dependent) and are not compared.
"""
import itertools

import numpy as np
import pytest

from synth import random_su3_links, unit_links
from oracle import lattice as L
from oracle import wilson as W
from oracle import krylov as K
from oracle.noise import z4_noise

DIMS = (4, 4, 2, 4)
KAPPA = 0.125


@pytest.fixture(scope="module")
def setup():
    U = random_su3_links(DIMS, 0.3, 31)
    M = W.dense_M(U, KAPPA, DIMS)
    eta = z4_noise(5, DIMS, 0, 3)
    ev, od = L.eo_tables(DIMS)
    idx_e = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in ev])
    idx_o = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in od])
    # dense Mhat from the block form of M
    Mee = M[np.ix_(idx_e, idx_e)]
    Meo = M[np.ix_(idx_e, idx_o)]
    Moe = M[np.ix_(idx_o, idx_e)]
    assert np.abs(Mee - np.eye(idx_e.size)).max() == 0   # no even-even hopping
    Mhat = np.eye(idx_e.size) - Meo @ Moe
    return U, M, eta, idx_e, Mhat


def _Ahat(U):
    shape = (DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 3)
    return lambda v: W.apply_Mhat(U, KAPPA, v.reshape(shape), DIMS).ravel()


def test_gmres_dr_solution_and_eigenvalues(setup):
    U, M, eta, idx_e, Mhat = setup
    src = W.eo_source(U, KAPPA, eta[0], DIMS).ravel()
    xe, info = K.gmres_dr(_Ahat(U), src, 24, 10, 1e-13)
    assert info["converged"]
    xref = np.zeros_like(src)
    xref[idx_e] = np.linalg.solve(Mhat, src[idx_e])
    assert np.linalg.norm(xe - xref) / np.linalg.norm(xref) < 1e-11
    # Arnoldi relation of the deflation data
    Vk1, Hk = info["V"], info["H"]
    k = Hk.shape[1]
    AV = np.stack([_Ahat(U)(Vk1[:, i]) for i in range(k)], axis=1)
    assert np.abs(AV - Vk1 @ Hk).max() < 1e-12
    assert np.abs(Vk1.conj().T @ Vk1 - np.eye(k + 1)).max() < 1e-12


def test_harmonic_ritz_values_are_low_eigenvalues(setup):
    """Super-converged GMRES-DR: harmonic Ritz pairs with small residual are
    eigenpairs of Mhat at the small-|lambda| end of its spectrum."""
    U, M, eta, idx_e, Mhat = setup
    kappa = 0.13
    shape = eta[0].shape
    A = lambda v: W.apply_Mhat(U, kappa, v.reshape(shape), DIMS).ravel()
    src = W.eo_source(U, kappa, eta[0], DIMS).ravel()
    _, info = K.gmres_dr(A, src, 14, 7, 1e-13, max_cycles=400, eig_tol=1e-11, n_eig=3)
    Me = np.eye(Mhat.shape[0]) - (np.eye(Mhat.shape[0]) - Mhat) * (kappa / KAPPA) ** 2
    lam = np.linalg.eigvals(Me)
    lam = lam[np.argsort(np.abs(lam))]
    conv = info["theta_resid"] < 1e-10
    assert conv[:3].all()
    for t in info["theta"][conv]:
        assert np.min(np.abs(lam - t)) < 1e-9
        # among the 2k smallest in modulus
        assert np.min(np.abs(lam[:14] - t)) < 1e-9


def test_gmres_proj_matches_dense(setup):
    U, M, eta, idx_e, Mhat = setup
    src0 = W.eo_source(U, KAPPA, eta[0], DIMS).ravel()
    _, info = K.gmres_dr(_Ahat(U), src0, 24, 10, 1e-13)
    for n in (1, 2):
        src = W.eo_source(U, KAPPA, eta[n], DIMS).ravel()
        xe, inf = K.gmres_proj(_Ahat(U), src, info["V"], info["H"], 14, 1e-12)
        assert inf["converged"]
        x = W.eo_reconstruct(U, KAPPA, xe.reshape(eta[n].shape), eta[n], DIMS)
        xref = np.linalg.solve(M, eta[n].ravel())
        assert np.linalg.norm(x.ravel() - xref) / np.linalg.norm(xref) < 1e-10


def test_hermitian_ritz_pairs_vs_dense(setup):
    U, M, eta, idx_e, Mhat = setup
    G5 = W.dense_gamma(L.GAMMA5, L.volume(DIMS))
    Mp = M @ G5
    shape = eta[0].shape
    Ap = lambda v: W.apply_Mprime(U, KAPPA, v.reshape(shape)).ravel()
    _, info = K.gmres_dr(Ap, eta[0].ravel(), 40, 20, 1e-13, max_cycles=300, eig_tol=1e-11, n_eig=8)
    Q = 6
    lam, Ev, resid = K.rayleigh_ritz_hermitian(info["V"], info["H"], Q)
    lam_d, E_d = K.hermitian_eigpairs_dense(Mp, Q)
    good = resid < 1e-9
    assert good.all()
    assert np.abs(lam[good] - lam_d[:good.sum()]).max() < 1e-9
    # projector invariant on the converged pairs
    z = np.random.default_rng(2).standard_normal(Mp.shape[0]) + 0j
    ng = int(np.argmin(good)) if not good.all() else Q
    P1 = Ev[:, :ng] @ ((Ev[:, :ng].conj().T @ z) / lam[:ng])
    P2 = E_d[:, :ng] @ ((E_d[:, :ng].conj().T @ z) / lam_d[:ng])
    assert np.linalg.norm(P1 - P2) / np.linalg.norm(P2) < 1e-8


def test_free_field_hermitian_spectrum():
    dims = (4, 4, 2, 2)
    kappa = 0.1
    M = W.dense_M(unit_links(dims), kappa, dims)
    Mp = M @ W.dense_gamma(L.GAMMA5, L.volume(dims))
    lam = np.sort(np.linalg.eigvalsh(Mp))
    ref = []
    for p in itertools.product(*[2 * np.pi * np.arange(n) / n for n in dims]):
        a = 1 - 2 * kappa * np.cos(p).sum()
        b = 4 * kappa ** 2 * (np.sin(p) ** 2).sum()
        ref += [np.sqrt(a * a + b)] * 6 + [-np.sqrt(a * a + b)] * 6
    assert np.abs(lam - np.sort(ref)).max() < 1e-13
