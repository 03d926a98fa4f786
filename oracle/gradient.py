"""Derivatives of Tr(Theta M^{-1}) (oracle; test infrastructure only).

Not in the paper; derived from its M = 1 - kappa P (Sec. 5.1, Eqs.
(24)-(25)) and g5-hermiticity M^dagger = g5 M g5 (Sec. 5.4):

  d/dkappa Tr(Theta M^{-1}) = Tr(Theta M^{-1} P M^{-1}),
  estimated per noise vector as y^dagger P x with x = M^{-1} eta and
  y = (M^{-1})^dagger Theta^dagger eta = g5 M^{-1} g5 Theta^dagger eta.

Link derivative for U_mu(x) -> exp(i w^a T^a) U_mu(x) (left multiplication,
T^a = lambda^a / 2 with the Gell-Mann matrices): only the forward hop out
of x and the backward hop into x + mu contain the link, so

  d/dw^a Tr(Theta M^{-1}) = kappa Tr(Theta M^{-1} (dP/dw^a) M^{-1}),
  (dP/dw^a) psi (x)      = (1 - g_mu) i T^a U_mu(x) psi(x + mu),
  (dP/dw^a) psi (x + mu) = (1 + g_mu) (-i) U_mu(x)^dagger T^a psi(x),

and per noise vector y^dagger (dP/dw^a) x = i tr[T^a (U F1 - F2 U^dagger)]
with the colour outer products F1 = sum_s ((1 - g_mu) x(x+mu))_s y(x)_s^dagger,
F2 = sum_s ((1 + g_mu) x(x))_s y(x+mu)_s^dagger.

Pinned by tests/test_oracle_gradient.py: dense derivatives against central
finite differences, and the per-noise formulas against the dense traces with
a complete set of unit vectors as noise (which makes the estimate exact).
"""
import numpy as np

from .lattice import GAMMA, GAMMA5, volume
from .wilson import hop, dense_P, g5, apply_theta

_I4 = np.eye(4, dtype=np.complex128)


def gell_mann():
    L = np.zeros((8, 3, 3), dtype=np.complex128)
    L[0][0, 1] = L[0][1, 0] = 1
    L[1][0, 1] = -1j
    L[1][1, 0] = 1j
    L[2][0, 0], L[2][1, 1] = 1, -1
    L[3][0, 2] = L[3][2, 0] = 1
    L[4][0, 2] = -1j
    L[4][2, 0] = 1j
    L[5][1, 2] = L[5][2, 1] = 1
    L[6][1, 2] = -1j
    L[6][2, 1] = 1j
    L[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return L


T_GEN = gell_mann() / 2


def theta_dense(theta, V):
    T = _I4 if theta == 0 else GAMMA[theta - 1]
    return np.kron(np.eye(V), np.kron(T, np.eye(3)))


def theta_weighted_dense(thetas, weights, dims):
    """Site-diagonal Theta_w = sum_a w[a][t(x)] Theta_a (dense), with t(x)
    the timeslice of site x; weights complex [len(thetas)][Lt]."""
    V = volume(dims)
    Vs = V // dims[3]
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    for a, th in enumerate(thetas):
        T = np.kron(_I4 if th == 0 else GAMMA[th - 1], np.eye(3))
        for x in range(V):
            D[12 * x:12 * x + 12, 12 * x:12 * x + 12] += weights[a][x // Vs] * T
    return D


def _theta(theta, dims):
    return theta_dense(theta, volume(dims)) if np.isscalar(theta) else theta


def trace_dense(U, kappa, dims, theta):
    """Tr(Theta M^{-1}); theta an operator code or a dense matrix."""
    V = volume(dims)
    M = np.eye(12 * V) - kappa * dense_P(U, dims)
    return np.trace(_theta(theta, dims) @ np.linalg.inv(M))


def dkappa_dense(U, kappa, dims, theta):
    V = volume(dims)
    P = dense_P(U, dims)
    Minv = np.linalg.inv(np.eye(12 * V) - kappa * P)
    return np.trace(_theta(theta, dims) @ Minv @ P @ Minv)


def dP_dw(U, dims, site, mu, a):
    """dP/dw^a for the link U_mu(site) (site lexicographic), dense."""
    Lx, Ly, Lz, Lt = dims
    L = (Lx, Ly, Lz, Lt)
    V = volume(dims)
    c = [site % Lx, (site // Lx) % Ly, (site // (Lx * Ly)) % Lz, site // (Lx * Ly * Lz)]
    cp = list(c)
    cp[mu] = (cp[mu] + 1) % L[mu]
    sp = cp[0] + Lx * (cp[1] + Ly * (cp[2] + Lz * cp[3]))
    Ux = U[c[3], c[2], c[1], c[0], mu]
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    Ta = T_GEN[a]
    D[12 * site:12 * site + 12, 12 * sp:12 * sp + 12] += np.kron(_I4 - GAMMA[mu], 1j * Ta @ Ux)
    D[12 * sp:12 * sp + 12, 12 * site:12 * site + 12] += np.kron(_I4 + GAMMA[mu], -1j * Ux.conj().T @ Ta)
    return D


def dlink_dense(U, kappa, dims, theta, site, mu, a):
    V = volume(dims)
    Minv = np.linalg.inv(np.eye(12 * V) - kappa * dense_P(U, dims))
    return kappa * np.trace(_theta(theta, dims) @ Minv @ dP_dw(U, dims, site, mu, a) @ Minv)


def rotate_link(U, site, mu, a, h, dims):
    """Copy of U with U_mu(site) -> exp(i h T^a) U_mu(site)."""
    Lx, Ly, Lz, Lt = dims
    c = [site % Lx, (site // Lx) % Ly, (site // (Lx * Ly)) % Lz, site // (Lx * Ly * Lz)]
    w, v = np.linalg.eigh(T_GEN[a])
    R = v @ np.diag(np.exp(1j * h * w)) @ v.conj().T
    U2 = U.copy()
    U2[c[3], c[2], c[1], c[0], mu] = R @ U[c[3], c[2], c[1], c[0], mu]
    return U2


def adjoint_vectors(U, kappa, dims, theta, eta, solve):
    """y = g5 M^{-1} g5 Theta^dagger eta, with `solve` a callable M^{-1}."""
    src = g5(apply_theta(theta, eta))  # Theta is hermitian
    return g5(solve(src))


def adjoint_vectors_weighted(U, kappa, dims, thetas, weights, eta, solve):
    """y = g5 M^{-1} g5 Theta_w^dagger eta for Theta_w of theta_weighted_dense:
    Theta_w^dagger eta (x) = sum_a conj(w[a][t(x)]) Theta_a eta(x)."""
    src = np.zeros_like(eta)
    for a, th in enumerate(thetas):
        wt = np.conj(np.asarray(weights[a], dtype=np.complex128))
        src += wt[None, :, None, None, None, None, None] * apply_theta(th, eta)
    return g5(solve(g5(src)))


def grad_estimate(U, kappa, dims, eta, x, y):
    """Per-noise-averaged (dkappa, dw[Lt,Lz,Ly,Lx,mu,a]) from x = M^{-1} eta
    and y = g5 M^{-1} g5 Theta eta (fields of shape (N, Lt, Lz, Ly, Lx, 4, 3))."""
    N = eta.shape[0]
    dk = np.mean([np.vdot(y[n].ravel(), hop(U, x[n]).ravel()) for n in range(N)])
    dw = np.zeros(U.shape[:4] + (4, 8), dtype=np.complex128)
    for mu in range(4):
        ax = 3 - mu
        Umu = U[..., mu, :, :]
        for n in range(N):
            xp = np.roll(x[n], -1, axis=ax)           # x(site + mu)
            yp = np.roll(y[n], -1, axis=ax)           # y(site + mu)
            z1 = np.einsum("st,...tb->...sb", _I4 - GAMMA[mu], xp)
            z2 = np.einsum("st,...tb->...sb", _I4 + GAMMA[mu], x[n])
            F1 = np.einsum("...sa,...sb->...ab", z1, np.conj(y[n]))
            F2 = np.einsum("...sa,...sb->...ab", z2, np.conj(yp))
            G = 1j * (Umu @ F1 - F2 @ np.conj(np.swapaxes(Umu, -1, -2)))
            dw[..., mu, :] += np.einsum("kab,...ba->...k", T_GEN, G)
    dw *= kappa / N
    return dk, dw
