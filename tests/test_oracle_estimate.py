"""Pins for the oracle's subtracted estimator (CPU, fixed seeds).

* Unbiasedness (Eqs. (14), (23)): for every method the mean over many Z(4)
  noises of eta^dagger Theta (x - xt) + Tr(Theta tilde-M^{-1}) approaches the
  exact Tr(Theta M^{-1}) from a dense inverse.
* Variance law for Z(4) noise (Eq. (13) with one noise vector): with
  q = Theta (M^{-1} - tilde-M^{-1}), Var t = sum_{i != j} |q_ij|^2, and
  Var Re t, Var Im t = 1/2 sum_{i != j} (|q_ij|^2 +- Re q_ij q_ji).  The
  standard errors the estimator reports satisfy N err^2 = Var (Re / Im).
* 1/xi' (Sec. 5.5): once p(kappa P) is M^{-1}, e'^dagger g5 p e' is
  e'^dagger M'^{-1} e' = 1/lambda' (M' = M g5), and HFPS / HFPOLY collapse
  to their polynomial part.
* HFES with every eigenpair of M' reproduces x exactly (zero variance).
* Sec. 6: per site, tr(M^{-1})_xx is real and tr(g_mu M^{-1})_xx imaginary.
* The estimate is unchanged by a gauge transformation of links and noise.
"""
import numpy as np
import pytest

from synth import random_su3_links
from oracle import lattice as L
from oracle import wilson as W
from oracle import subtract as S
from oracle import estimate as E
from oracle import krylov as K
from oracle.noise import z4_noise

DIMS = (2, 2, 2, 2)
KAPPA = 0.11
THETAS = (0, 4)


@pytest.fixture(scope="module")
def dense():
    U = random_su3_links(DIMS, 0.3, 61)
    V = L.volume(DIMS)
    Pd = W.dense_P(U, DIMS)
    M = np.eye(12 * V) - KAPPA * Pd
    Minv = np.linalg.inv(M)
    G5 = W.dense_gamma(L.GAMMA5, V)
    lam, Ev = K.hermitian_eigpairs_dense(M @ G5, 24)
    return U, Pd, M, Minv, G5, lam, Ev


def _methods(U, Pd, G5, lam, Ev, b):
    """Dense tilde-M^{-1} per method and the callables producing xt."""
    V = L.volume(DIMS)
    shape = (DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 3)
    Q = lam.size
    Et = Ev.T.reshape((Q,) + shape)
    cpert = S.pert_coeffs(4)
    cpoly, _ = S.poly_coeffs(U, KAPPA, b, 4)
    inv_lam = 1.0 / lam + 0j
    xi_pert = S.xi_inverse(U, KAPPA, Et, cpert)
    xi_poly = S.xi_inverse(U, KAPPA, Et, cpoly)
    eig = lambda w: G5 @ Ev @ np.diag(w) @ Ev.conj().T
    Ppert = S.poly_dense(Pd, KAPPA, cpert)
    Ppoly = S.poly_dense(Pd, KAPPA, cpoly)
    dense = {
        "NS": np.zeros_like(Pd), "PS": Ppert, "POLY": Ppoly, "HFES": eig(inv_lam),
        "HFPS": eig(inv_lam) + Ppert - eig(xi_pert), "HFPOLY": eig(inv_lam) + Ppoly - eig(xi_poly),
    }
    xt = {
        "NS": lambda eta: np.zeros_like(eta),
        "PS": lambda eta: S.horner(U, KAPPA, eta, cpert),
        "POLY": lambda eta: S.horner(U, KAPPA, eta, cpoly),
        "HFES": lambda eta: S.eig_vector(Et, inv_lam, eta),
        "HFPS": lambda eta: S.eig_vector(Et, inv_lam, eta) + S.horner(U, KAPPA, eta, cpert)
        - S.eig_vector(Et, xi_pert, eta),
        "HFPOLY": lambda eta: S.eig_vector(Et, inv_lam, eta) + S.horner(U, KAPPA, eta, cpoly)
        - S.eig_vector(Et, xi_poly, eta),
    }
    sb = lambda w: S.site_bilinear(Et, THETAS, DIMS, w)
    cp = S.trace_correction_probe(U, KAPPA, cpert, DIMS, THETAS)
    cq = S.trace_correction_probe(U, KAPPA, cpoly, DIMS, THETAS)
    corr = {
        "NS": np.zeros((len(THETAS), DIMS[3]), complex), "PS": cp, "POLY": cq, "HFES": sb(inv_lam),
        "HFPS": sb(inv_lam) + cp - sb(xi_pert), "HFPOLY": sb(inv_lam) + cq - sb(xi_poly),
    }
    return dense, xt, corr


def test_unbiased_and_variance_law(dense):
    U, Pd, M, Minv, G5, lam, Ev = dense
    lam, Ev = lam[:8], Ev[:, :8]
    V = L.volume(DIMS)
    b = z4_noise(100, DIMS, 0, 1)[0]
    dense_mats, xt_fns, corr = _methods(U, Pd, G5, lam, Ev, b)
    exact = S.trace_correction_dense(Minv, DIMS, THETAS)
    exact = np.concatenate([exact, exact.sum(-1, keepdims=True)], -1)
    # the oracle's subtraction vectors equal the dense matrices applied to eta
    eta = z4_noise(8, DIMS, 0, 4)
    for m, f in xt_fns.items():
        ref = (dense_mats[m] @ eta.reshape(4, -1).T).T.reshape(eta.shape)
        assert np.abs(f(eta) - ref).max() < 1e-12, m
    N, chunk = 100000, 25000
    tsum = {m: [] for m in dense_mats}
    for c0 in range(0, N, chunk):
        eta = z4_noise(7, DIMS, c0, chunk)
        ef = eta.reshape(chunk, -1).T
        x = (Minv @ ef).T.reshape(eta.shape)
        for m, D in dense_mats.items():
            xt = (D @ ef).T.reshape(eta.shape)
            tsum[m].append(E.samples(eta, x, xt, THETAS, DIMS))
    for m in dense_mats:
        t = np.concatenate(tsum[m])
        est, err = E.estimate(t, corr[m])
        for a, th in enumerate(THETAS):
            Th = W.dense_gamma(S.theta_matrix(th), V)
            q = Th @ (Minv - dense_mats[m])
            off = q - np.diag(np.diag(q))
            var_c = (np.abs(off) ** 2).sum()
            cross = (off * off.T).real.sum()
            if var_c < 1e-20:
                assert np.abs(t[:, a, -1] - t[0, a, -1]).max() < 1e-10
                continue
            # unbiased within 4.5 standard errors (Re and Im separately)
            d = est[a, -1] - exact[a, -1]
            assert abs(d.real) < 4.5 * err[a, -1, 0] + 1e-12, (m, th)
            assert abs(d.imag) < 4.5 * err[a, -1, 1] + 1e-12, (m, th)
            # Z(4) variance law
            emp = np.var(t[:, a, -1])
            assert abs(emp / var_c - 1) < 0.04, (m, th, emp / var_c)
            for c, (part, pred) in enumerate(((t[:, a, -1].real, 0.5 * (var_c + cross)),
                                              (t[:, a, -1].imag, 0.5 * (var_c - cross)))):
                if pred > 1e-3 * var_c:
                    assert abs(np.var(part) / pred - 1) < 0.05, (m, th)
                    # the reported standard error is sqrt(Var / N): N err^2
                    # against the predicted variance (a missing 1/sqrt(N),
                    # or a Re/Im swap, misses by orders of magnitude)
                    assert abs(N * err[a, -1, c] ** 2 / pred - 1) < 0.05, (m, th, c)
                else:
                    assert N * err[a, -1, c] ** 2 < 2e-3 * var_c, (m, th, c)


def test_xi_inverse_is_inverse_eigenvalue_when_p_inverts_M():
    """With p(kappa P) = z M^{-1} (the hopping series of order 60 at kappa =
    0.05 times a complex z; kappa ||P|| <= 0.05 * 8 sqrt(2) < 0.57, so the
    truncation is below 0.57^61 ~ 1e-15), 1/xi'_q = e'^dagger g5 p e'_q must
    equal z / lambda'_q: M' = M g5 gives M'^{-1} = g5 M^{-1} (Sec. 5.5).  A
    missing g5 flips the sign for the negative lambda', a conjugated
    bilinear gives conj(z) / lambda'.  The HFPS / HFPOLY overlap term then
    cancels the HFES term exactly, vector and trace correction."""
    kappa = 0.05
    U = random_su3_links(DIMS, 0.3, 65)
    V = L.volume(DIMS)
    M = W.dense_M(U, kappa, DIMS)
    G5 = W.dense_gamma(L.GAMMA5, V)
    lam, Ev = K.hermitian_eigpairs_dense(M @ G5, 12)
    assert (lam < 0).any() and (lam > 0).any()
    shape = (DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 3)
    Et = Ev.T.reshape((lam.size,) + shape)
    z = 0.3 + 0.7j
    coeffs = z * S.pert_coeffs(60)
    xi = S.xi_inverse(U, kappa, Et, coeffs)
    assert np.abs(xi - z / lam).max() < 1e-12 * np.abs(z / lam).max()
    # HFPOLY with p -> z M^{-1} and weights z / lambda': the eigen part and
    # the overlap cancel, leaving x_poly and Tr(Theta p)
    eta = z4_noise(9, DIMS, 0, 3)
    eig = S.eig_vector(Et, z / lam + 0j, eta)
    assert np.abs(eig - S.eig_vector(Et, xi, eta)).max() < 1e-12
    sb = S.site_bilinear(Et, (0, 1, 2, 3, 4), DIMS, z / lam + 0j)
    assert np.abs(sb - S.site_bilinear(Et, (0, 1, 2, 3, 4), DIMS, xi)).max() < 1e-12
    # and the truncated series is M^{-1} to the same accuracy
    Minv = np.linalg.inv(M)
    ref = z * (Minv @ eta.reshape(3, -1).T).T.reshape(eta.shape)
    assert np.abs(S.horner(U, kappa, eta, coeffs) - ref).max() < 1e-13


def test_hfes_all_modes_is_exact(dense):
    U, Pd, M, Minv, G5, lam, Ev = dense
    V = L.volume(DIMS)
    lam_all, E_all = K.hermitian_eigpairs_dense(M @ G5, 12 * V)
    shape = (DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 3)
    Et = E_all.T.reshape((12 * V,) + shape)
    eta = z4_noise(3, DIMS, 0, 4)
    x = (Minv @ eta.reshape(4, -1).T).T.reshape(eta.shape)
    xt = S.eig_vector(Et, 1.0 / lam_all + 0j, eta)
    assert np.abs(x - xt).max() < 1e-12
    corr = S.site_bilinear(Et, THETAS, DIMS, 1.0 / lam_all + 0j)
    exact = S.trace_correction_dense(Minv, DIMS, THETAS)
    assert np.abs(corr - exact).max() < 1e-11


def test_site_traces_real_or_imaginary():
    dims = (4, 4, 2, 2)
    U = random_su3_links(dims, 0.3, 62)
    V = L.volume(dims)
    Minv = np.linalg.inv(W.dense_M(U, 0.13, dims))
    blocks = S.diag_blocks_dense(Minv, V)
    tr = S.block_traces(blocks, (0, 1, 2, 3, 4))
    assert np.abs(tr[0].imag).max() < 1e-13
    assert np.abs(tr[1:].real).max() < 1e-13


def test_estimate_gauge_invariant():
    dims = (4, 2, 2, 2)
    U = random_su3_links(dims, 0.3, 63)
    g = random_su3_links(dims, 1.0, 64)[..., 2, :, :]
    Ug = np.empty_like(U)
    for mu in range(4):
        gp = np.roll(g, -1, axis=3 - mu)
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gp, -1, -2))
    eta = z4_noise(5, dims, 0, 3)
    geta = np.einsum("...ab,n...sb->n...sa", g, eta)
    M, Mg = W.dense_M(U, 0.12, dims), W.dense_M(Ug, 0.12, dims)
    x = np.linalg.solve(M, eta.reshape(3, -1).T).T.reshape(eta.shape)
    xg = np.linalg.solve(Mg, geta.reshape(3, -1).T).T.reshape(eta.shape)
    c = S.pert_coeffs(4)
    t1 = E.samples(eta, x, S.horner(U, 0.12, eta, c), (0, 1, 4), dims)
    t2 = E.samples(geta, xg, S.horner(Ug, 0.12, geta, c), (0, 1, 4), dims)
    assert np.abs(t1 - t2).max() < 1e-12


def test_relative_efficiency():
    assert abs(E.relative_efficiency(0.5, 1.0) - 300.0) < 1e-12
    assert abs(E.relative_efficiency(1.0, 1.0)) < 1e-15
