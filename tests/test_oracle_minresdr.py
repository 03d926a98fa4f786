"""Pins for the oracle's MINRES-DR (hermitian deflated restarted solver, CPU).

Fixed by dense linear algebra, independently of the recurrence itself:
  * solutions of hermitian indefinite systems vs LU;
  * its harmonic Ritz values vs the smallest-|lambda| eigenvalues (eigh);
  * the first cycle vs the minimum-residual solution over an explicitly
    built Krylov space (a wrong or dropped recurrence term moves it);
  * the restart relation A V_k = V_{k+1} Hbar_k, orthonormal V, hermitian
    H_k after several cycles;
  * the hermitian harmonic pencil vs scipy's generalized eigensolver, also
    with an exactly singular H_m (where a solve with H_m^* has no answer);
  * agreement with the pinned GMRES-DR on the same hermitian problem;
  * Ritz pairs of M' = M g5 on a small lattice vs dense eigh, also at a
    near-critical kappa.
Iteration counts depend on rounding and are not compared.
"""
import numpy as np
import pytest
import scipy.linalg

from synth import random_su3_links
from oracle import lattice as L
from oracle import wilson as W
from oracle import krylov as K
from oracle.noise import z4_noise


def _hermitian_indefinite(n, seed, small=(1e-3, -2e-3, 5e-3, -8e-3, 1.2e-2, -2e-2)):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, _ = np.linalg.qr(Z)
    rest = n - len(small)
    bulk = np.concatenate([rng.uniform(-3.0, -0.2, rest // 2), rng.uniform(0.2, 4.0, rest - rest // 2)])
    lam = np.concatenate([np.asarray(small), bulk])
    A = (Q * lam) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, lam, b


def test_solution_matches_lu():
    A, lam, b = _hermitian_indefinite(150, 1)
    x, info = K.minres_dr(lambda v: A @ v, b, 30, 10, 1e-11, max_cycles=400)
    assert info["converged"]
    xr = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-7
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 2e-11


def test_harmonic_ritz_values_are_the_smallest_eigenvalues():
    A, lam, b = _hermitian_indefinite(150, 2)
    _, info = K.minres_dr(lambda v: A @ v, b, 30, 10, 1e-12, max_cycles=600, eig_tol=1e-9, n_eig=6)
    ref = lam[np.argsort(np.abs(lam))][:6]
    th = info["theta"][:6]
    assert np.abs(th.imag).max() < 1e-12
    assert np.abs(np.sort(th.real) - np.sort(ref)).max() < 1e-8 * np.abs(ref).max() + 1e-12
    assert (info["theta_resid"][:6] <= 1e-9 * np.abs(th)).all()


def test_first_cycle_is_minimum_residual_over_krylov_space():
    rng = np.random.default_rng(3)
    n, m = 60, 8
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, _ = np.linalg.qr(Z)
    lam = np.concatenate([rng.uniform(-2.0, -0.5, 30), rng.uniform(0.5, 3.0, 30)])
    A = (Q * lam) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x1, _ = K.minres_dr(lambda v: A @ v, b, m, 3, 0.0, max_cycles=1)
    # K_m(A, b) from explicit powers, orthonormalised; min |b - A Kq y|
    Kr = np.empty((n, m), dtype=np.complex128)
    v = b.copy()
    for j in range(m):
        Kr[:, j] = v
        v = A @ v
    Kq, _ = np.linalg.qr(Kr)
    y = np.linalg.lstsq(A @ Kq, b, rcond=None)[0]
    xr = Kq @ y
    assert np.linalg.norm(x1 - xr) / np.linalg.norm(xr) < 1e-10


def test_restart_relation_after_cycles():
    A, lam, b = _hermitian_indefinite(120, 4)
    m, k = 24, 8
    _, info = K.minres_dr(lambda v: A @ v, b, m, k, 0.0, max_cycles=5)
    V, H = info["V"], info["H"]
    assert V.shape == (120, k + 1) and H.shape == (k + 1, k)
    lhs = A @ V[:, :k]
    assert np.linalg.norm(lhs - V @ H) / np.linalg.norm(lhs) < 1e-11
    assert np.abs(V.conj().T @ V - np.eye(k + 1)).max() < 1e-11
    Hk = H[:k, :k]
    assert np.abs(Hk - Hk.conj().T).max() < 1e-10 * np.abs(Hk).max()


@pytest.mark.parametrize("singular", [False, True])
def test_hermitian_harmonic_pencil_vs_scipy(singular):
    rng = np.random.default_rng(5)
    m = 12
    Z = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    Hm = 0.5 * (Z + Z.conj().T)
    if singular:  # make H_m exactly singular
        w, S = np.linalg.eigh(Hm)
        w[3] = 0.0
        Hm = (S * w) @ S.conj().T
        Hm = 0.5 * (Hm + Hm.conj().T)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    H[:m] = Hm
    H[m, m - 1] = 0.7
    theta, g, w = K.harmonic_ritz_hermitian(H, m)
    # scipy: Hbar^* Hbar g = theta H_m g
    tr = scipy.linalg.eig(H.conj().T @ H, Hm, right=False)
    fin = np.isfinite(theta)
    ref = np.sort_complex(tr[np.isfinite(tr) & (np.abs(tr) < 1e8)])
    ours = np.sort_complex(theta[fin & (np.abs(theta) < 1e8)])
    assert ours.size == ref.size == (m - 1 if singular else m)
    assert np.abs(ours - ref).max() < 1e-8 * np.abs(ref).max()
    # each pair with a finite theta (away from the mu = 0 direction, where
    # theta is 1 / rounding) satisfies the pencil, and w spans the
    # orthogonal complement of range(Hbar)
    for q in np.nonzero(fin & (np.abs(theta) < 1e8))[0]:
        r = H.conj().T @ H @ g[:, q] - theta[q] * Hm @ g[:, q]
        assert np.linalg.norm(r) < 1e-9 * np.linalg.norm(H.conj().T @ H @ g[:, q])
    assert abs(np.linalg.norm(w) - 1) < 1e-13
    assert np.abs(H.conj().T @ w).max() < 1e-12


def test_agrees_with_gmres_dr_on_hermitian_problem():
    A, lam, b = _hermitian_indefinite(140, 6)
    Af = lambda v: A @ v
    x1, i1 = K.minres_dr(Af, b, 28, 10, 1e-11, max_cycles=400, eig_tol=1e-8, n_eig=5)
    x2, i2 = K.gmres_dr(Af, b, 28, 10, 1e-11, max_cycles=400, eig_tol=1e-8, n_eig=5)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x2) < 1e-8
    assert np.abs(np.sort(i1["theta"][:5].real) - np.sort(i2["theta"][:5].real)).max() < 1e-7


@pytest.mark.parametrize("kappa", [0.125, 0.255])
def test_lattice_hermitian_eigpairs_vs_dense(kappa):
    """kappa = 0.255 puts an eigenvalue of M' of this lattice at 1.25e-3
    (near-critical): a restart built from pairs of a hermitised H_m loses
    the Arnoldi relation there within a few hundred cycles."""
    dims = (4, 4, 2, 4)
    U = random_su3_links(dims, 0.3, 31)
    M = W.dense_M(U, kappa, dims)
    Mp = M @ W.dense_gamma(L.GAMMA5, L.volume(dims))
    eta = z4_noise(5, dims, 0, 1)[0]
    shape = eta.shape
    Ap = lambda v: W.apply_Mprime(U, kappa, v.reshape(shape)).ravel()
    _, info = K.minres_dr(Ap, eta.ravel(), 40, 20, 1e-13, max_cycles=400, eig_tol=1e-11, n_eig=8)
    Q = 6
    lam, Ev, resid = K.rayleigh_ritz_hermitian(info["V"], info["H"], Q)
    lam_d, E_d = K.hermitian_eigpairs_dense(Mp, Q)
    assert (resid < 1e-9).all()
    assert np.abs(lam - lam_d).max() < 1e-9
    overlap = np.abs(np.einsum("iq,iq->q", E_d.conj(), Ev))
    assert np.abs(overlap - 1).max() < 1e-8
