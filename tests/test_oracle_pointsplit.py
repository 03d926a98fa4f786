"""Pins for the oracle's point-split vector operator (CPU).

* the shift form of Theta(mu) equals its matrix elements;
* free field: the dense trace Tr(Theta(mu) p(kappa P)) equals the
  momentum-space sum (an independent construction), for the PS polynomial;
* Tr(Theta(mu) M^{-1}) is purely imaginary (Theta(mu)^dagger =
  -g5 Theta(mu) g5 with g5-hermiticity of M), the "Im" of Table 2;
* only odd powers of kappa P contribute to Tr(Theta(mu) (kappa P)^j);
* with every unit vector as noise the estimator equals the dense trace;
* the hermitian-forced bilinear equals the dense trace of
  Theta(mu) g5 sum_q w_q e_q e_q^dagger.
"""
import numpy as np
import pytest

from synth import random_su3_links, unit_links
from oracle import lattice as L
from oracle import wilson as W
from oracle import subtract as S
from oracle import pointsplit as PSO

KAPPA = 0.11


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (4, 2, 2, 4)])
def test_shift_form_matches_matrix_elements(dims):
    U = random_su3_links(dims, 0.3, 12)
    rng = np.random.default_rng(3)
    shape = (2, dims[3], dims[2], dims[1], dims[0], 4, 3)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    for mu in range(4):
        D = PSO.dense_theta_ps(U, KAPPA, dims, mu)
        ref = (D @ v.reshape(2, -1).T).T.reshape(shape)
        assert np.abs(PSO.apply_theta_ps(U, KAPPA, mu, v) - ref).max() < 1e-14


@pytest.mark.parametrize("mu", [0, 3])
def test_constant_phase_trace_closed_form(mu):
    """Constant abelian links keep momentum space diagonal: the dense trace
    equals the plane-wave sum; the phases make it nonzero."""
    dims = (4, 2, 2, 4)
    phases = (0.3, -0.5, 0.7, 0.9)
    U = PSO.phase_links(dims, phases)
    coeffs = S.pert_coeffs(7)
    A = S.poly_dense(W.dense_P(U, dims), KAPPA, coeffs)
    dense = PSO.trace_ps_dense(U, KAPPA, dims, mu, A).sum()
    closed = PSO.free_trace_ps(dims, KAPPA, mu, coeffs, phases)
    assert abs(closed) > 1e-4
    assert abs(dense - closed) < 1e-12 * abs(closed)
    # unit links: the free current has no expectation
    U0 = unit_links(dims)
    A0 = S.poly_dense(W.dense_P(U0, dims), KAPPA, coeffs)
    assert abs(PSO.trace_ps_dense(U0, KAPPA, dims, mu, A0).sum()) < 1e-12


def test_trace_is_imaginary_and_odd_orders_only():
    dims = (2, 2, 2, 4)
    U = random_su3_links(dims, 0.3, 14)
    M = W.dense_M(U, KAPPA, dims)
    Minv = np.linalg.inv(M)
    Pd = W.dense_P(U, dims)
    for mu in range(4):
        t = PSO.trace_ps_dense(U, KAPPA, dims, mu, Minv).sum()
        assert abs(t.real) < 1e-12 * abs(t)
        for j in range(0, 7):
            c = np.zeros(j + 1)
            c[j] = 1.0
            tj = PSO.trace_ps_dense(U, KAPPA, dims, mu, S.poly_dense(Pd, KAPPA, c)).sum()
            if j % 2 == 0:
                assert abs(tj) < 1e-12
    # at small kappa the hopping expansion of the trace converges to it
    k2 = 0.05
    coeffs = S.pert_coeffs(25)
    approx = PSO.trace_ps_dense(U, k2, dims, 3, S.poly_dense(Pd, k2, coeffs)).sum()
    exact = PSO.trace_ps_dense(U, k2, dims, 3, np.linalg.inv(W.dense_M(U, k2, dims))).sum()
    assert abs(approx - exact) < 1e-8 * abs(exact)


def test_estimator_with_unit_vectors_is_exact():
    dims = (2, 2, 2, 4)
    U = random_su3_links(dims, 0.3, 15)
    V = L.volume(dims)
    n = 12 * V
    shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    eta = np.eye(n, dtype=np.complex128).reshape((n,) + shape)
    Minv = np.linalg.inv(W.dense_M(U, KAPPA, dims))
    x = (Minv @ eta.reshape(n, -1).T).T.reshape(eta.shape)
    smp = PSO.samples_ps(U, KAPPA, eta, x, np.zeros_like(x), range(4), dims)
    for mu in range(4):
        ref = PSO.trace_ps_dense(U, KAPPA, dims, mu, Minv)
        assert np.abs(smp[:, mu, :-1].sum(axis=0) - ref).max() < 1e-11 * np.abs(ref).max()


def test_hermitian_forced_bilinear_matches_dense():
    dims = (2, 2, 2, 4)
    U = random_su3_links(dims, 0.3, 16)
    rng = np.random.default_rng(5)
    Q = 3
    shape = (Q, dims[3], dims[2], dims[1], dims[0], 4, 3)
    E = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    w = rng.standard_normal(Q) + 1j * rng.standard_normal(Q)
    Ef = E.reshape(Q, -1)
    G5 = W.dense_gamma(L.GAMMA5, L.volume(dims))
    A = G5 @ (Ef.T * w) @ np.conj(Ef)
    got = PSO.site_bilinear_ps(U, KAPPA, E, range(4), dims, w)
    for mu in range(4):
        assert np.abs(got[mu] - PSO.trace_ps_dense(U, KAPPA, dims, mu, A)).max() < 1e-11 * np.abs(got).max()
