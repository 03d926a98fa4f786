"""Pins for the oracle's derivatives of Tr(Theta M^{-1}) (CPU).

* dense d/dkappa and d/dw^a against Richardson-extrapolated central finite
  differences (h = 1e-3 and 5e-4, error O(h^4));
* the per-noise estimator (y^dagger P x, i tr[T^a (U F1 - F2 U^dagger)]) with
  every unit vector as a noise vector reproduces the dense derivatives
  exactly (sum_i e_i^dagger A e_i = Tr A).
"""
import numpy as np
import pytest

from synth import random_su3_links
from oracle import lattice as L
from oracle import wilson as W
from oracle import gradient as G

DIMS = (2, 2, 2, 4)
KAPPA = 0.09


@pytest.fixture(scope="module")
def links():
    return random_su3_links(DIMS, 0.3, 71)


def _richardson(f, h):
    """Central differences at h and h/2 combined to cancel the h^2 term."""
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3, d1, d2


@pytest.mark.parametrize("theta", [0, 4])
def test_dkappa_dense_vs_finite_difference(links, theta):
    an = G.dkappa_dense(links, KAPPA, DIMS, theta)
    r, d1, d2 = _richardson(lambda h: G.trace_dense(links, KAPPA + h, DIMS, theta), 1e-3)
    assert abs(r - an) < 1e-5 * abs(an)
    # the plain central differences converge to it as h^2
    assert 3.5 < abs(d1 - an) / abs(d2 - an) < 4.5


@pytest.mark.parametrize("theta,site,mu,a", [(0, 3, 0, 0), (0, 7, 3, 7), (4, 5, 2, 4), (2, 0, 1, 2)])
def test_dlink_dense_vs_finite_difference(links, theta, site, mu, a):
    an = G.dlink_dense(links, KAPPA, DIMS, theta, site, mu, a)
    f = lambda h: G.trace_dense(G.rotate_link(links, site, mu, a, h, DIMS), KAPPA, DIMS, theta)
    r, _, _ = _richardson(f, 1e-3)
    assert abs(r - an) < 1e-6 * max(abs(an), 1e-3)


@pytest.mark.parametrize("theta", [0, 1, 4])
def test_estimator_with_unit_vectors_is_exact(links, theta):
    V = L.volume(DIMS)
    n = 12 * V
    shape = (DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 3)
    eta = np.eye(n, dtype=np.complex128).reshape((n,) + shape)
    M = W.dense_M(links, KAPPA, DIMS)
    Minv = np.linalg.inv(M)
    solve = lambda b: (Minv @ b.reshape(b.shape[0], -1).T).T.reshape(b.shape)
    x = solve(eta)
    y = G.adjoint_vectors(links, KAPPA, DIMS, theta, eta, solve)
    dk, dw = G.grad_estimate(links, KAPPA, DIMS, eta, x, y)
    # the estimator averages over N = n noises; unit vectors sum to the trace
    assert abs(dk * n - G.dkappa_dense(links, KAPPA, DIMS, theta)) < 1e-10 * abs(dk * n)
    Lx, Ly, Lz, Lt = DIMS
    for site, mu, a in ((3, 0, 0), (7, 3, 7), (12, 1, 5)):
        c = [site % Lx, (site // Lx) % Ly, (site // (Lx * Ly)) % Lz, site // (Lx * Ly * Lz)]
        est = dw[c[3], c[2], c[1], c[0], mu, a] * n
        ref = G.dlink_dense(links, KAPPA, DIMS, theta, site, mu, a)
        assert abs(est - ref) < 1e-10 * max(abs(ref), 1e-6)


def test_weighted_theta_reduces_to_plain_theta():
    V = L.volume(DIMS)
    ones = np.ones((1, DIMS[3]))
    for th in range(5):
        assert np.array_equal(G.theta_weighted_dense((th,), ones, DIMS), G.theta_dense(th, V))
    # linear in the weights and site-diagonal in time: weight one timeslice only
    w = np.zeros((2, DIMS[3]), dtype=np.complex128)
    w[0, 1] = 2 - 1j
    w[1, 3] = 0.5j
    D = G.theta_weighted_dense((0, 3), w, DIMS)
    Vs = V // DIMS[3]
    blk = slice(12 * Vs, 24 * Vs)
    assert np.allclose(D[blk, blk], (2 - 1j) * np.eye(12 * Vs))
    assert np.count_nonzero(D[:12 * Vs]) == 0 and np.count_nonzero(D[24 * Vs:36 * Vs]) == 0


def test_weighted_estimator_with_unit_vectors_is_exact(links):
    rng = np.random.default_rng(5)
    thetas = (0, 2, 4)
    w = rng.normal(size=(3, DIMS[3])) + 1j * rng.normal(size=(3, DIMS[3]))
    V = L.volume(DIMS)
    n = 12 * V
    shape = (DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 3)
    eta = np.eye(n, dtype=np.complex128).reshape((n,) + shape)
    Minv = np.linalg.inv(W.dense_M(links, KAPPA, DIMS))
    solve = lambda b: (Minv @ b.reshape(b.shape[0], -1).T).T.reshape(b.shape)
    x = solve(eta)
    y = G.adjoint_vectors_weighted(links, KAPPA, DIMS, thetas, w, eta, solve)
    dk, dw = G.grad_estimate(links, KAPPA, DIMS, eta, x, y)
    Tw = G.theta_weighted_dense(thetas, w, DIMS)
    ref = G.dkappa_dense(links, KAPPA, DIMS, Tw)
    assert abs(dk * n - ref) < 1e-10 * abs(ref)
    for site, mu, a in ((3, 0, 0), (9, 2, 6)):
        c = [site % 2, (site // 2) % 2, (site // 4) % 2, site // 8]
        ref = G.dlink_dense(links, KAPPA, DIMS, Tw, site, mu, a)
        assert abs(dw[c[3], c[2], c[1], c[0], mu, a] * n - ref) < 1e-10 * max(abs(ref), 1e-6)
