"""Pins for the oracle's Wilson operator (CPU).

What fixes the operator, independently of the code that applies it:
* two constructions of P (array shifts vs matrix elements) agree;
* the free-field (unit-link) spectrum of P is the closed form
  2 sum_mu cos p_mu +- 2i sqrt(sum_mu sin^2 p_mu), 6-fold each
  (plane waves, p_mu = 2 pi n / L_mu), and plane waves are eigenvectors;
* g5 M g5 = M^dagger, so M' = M g5 is hermitian;
* gauge covariance M[U^g] = G M[U] G^dagger;
* Tr P^4 = -64 sum_plaquettes Re tr U_P for extents >= 5 (a closed-loop
  identity: only the 1x1 loops survive, each with spin trace -64/... and
  backtracking walks vanish because (1 - g)(1 + g) = 0);
* the even/odd reduction reproduces the full solution.
"""
import itertools

import numpy as np
import pytest

from synth import random_su3_links, unit_links
from oracle import lattice as L
from oracle import wilson as W


def _rand_field(dims, lead=(), seed=0):
    Lx, Ly, Lz, Lt = dims
    rng = np.random.default_rng(seed)
    shape = lead + (Lt, Lz, Ly, Lx, 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4), (4, 4, 4, 4)])
def test_hop_equals_dense_matrix(dims):
    U = random_su3_links(dims, 0.3, 5)
    Pd = W.dense_P(U, dims)
    psi = _rand_field(dims)
    assert np.abs(Pd @ psi.ravel() - W.hop(U, psi).ravel()).max() < 1e-13


def test_links_are_su3():
    U = random_su3_links((4, 4, 2, 2), 0.3, 3).reshape(-1, 3, 3)
    I = np.einsum("nba,nbc->nac", np.conj(U), U)
    assert np.abs(I - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


def free_field_eigs(dims):
    ps = [2 * np.pi * np.arange(Ln) / Ln for Ln in dims]
    vals = []
    for p in itertools.product(*ps):
        C = 2 * np.cos(p).sum()
        S = 2 * np.sqrt((np.sin(p) ** 2).sum())
        vals += [C + 1j * S] * 6 + [C - 1j * S] * 6
    return np.array(vals)


def _sorted(z):
    z = np.round(z, 9)
    return z[np.lexsort((z.imag, z.real))]


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 2, 6)])
def test_free_field_spectrum(dims):
    Pd = W.dense_P(unit_links(dims), dims)
    ev = np.linalg.eigvals(Pd)
    assert np.abs(_sorted(ev) - _sorted(free_field_eigs(dims))).max() < 1e-8


def test_free_field_plane_wave_eigenvector():
    """P (e^{ipx} u) = e^{ipx} P(p) u with P(p) = sum_mu [(1-g)e^{ip} + (1+g)e^{-ip}]."""
    dims = (4, 6, 2, 8)
    x, y, z, t = L.coords(dims)
    n = (1, 2, 1, 3)
    p = [2 * np.pi * n[i] / dims[i] for i in range(4)]
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    rng = np.random.default_rng(1)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = phase[..., None, None] * u
    Pp = sum((np.eye(4) - L.GAMMA[m]) * np.exp(1j * p[m]) + (np.eye(4) + L.GAMMA[m]) * np.exp(-1j * p[m])
             for m in range(4))
    ref = phase[..., None, None] * (Pp @ u)
    assert np.abs(W.hop(unit_links(dims), psi) - ref).max() < 1e-13


def test_g5_hermiticity_dense():
    dims = (4, 4, 2, 2)
    U = random_su3_links(dims, 0.3, 9)
    M = W.dense_M(U, 0.13, dims)
    G5 = W.dense_gamma(L.GAMMA5, L.volume(dims))
    assert np.abs(G5 @ M @ G5 - M.conj().T).max() < 1e-14
    Mp = M @ G5
    assert np.abs(Mp - Mp.conj().T).max() < 1e-14


def test_gauge_covariance():
    dims = (4, 2, 4, 2)
    U = random_su3_links(dims, 0.4, 4)
    g = random_su3_links(dims, 1.0, 8)[..., 0, :, :]        # one SU(3) per site
    Ug = np.empty_like(U)
    for mu in range(4):
        ax = 3 - mu
        gp = np.roll(g, -1, axis=ax)                          # g(x + mu)
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gp, -1, -2))
    psi = _rand_field(dims)
    Gpsi = np.einsum("...ab,...sb->...sa", g, psi)
    lhs = W.hop(Ug, Gpsi)
    rhs = np.einsum("...ab,...sb->...sa", g, W.hop(U, psi))
    assert np.abs(lhs - rhs).max() < 1e-13


def plaquette_sum(U):
    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            amu, anu = 3 - mu, 3 - nu
            Umu, Unu = U[..., mu, :, :], U[..., nu, :, :]
            P = Umu @ np.roll(Unu, -1, axis=amu) @ np.conj(np.swapaxes(np.roll(Umu, -1, axis=anu), -1, -2)) \
                @ np.conj(np.swapaxes(Unu, -1, -2))
            tot += np.trace(P, axis1=-2, axis2=-1).real.sum()
    return tot


def test_trace_P4_plaquettes_L6():
    dims = (6, 6, 6, 6)
    U = random_su3_links(dims, 0.3, 12)
    P = W.sparse_P(U, dims)
    P2 = (P @ P).tocsr()
    trP4 = P2.multiply(P2.T).sum()
    assert abs(trP4 - (-64.0 * plaquette_sum(U))) < 1e-11 * abs(trP4)
    # the local vector g4 sees no closed path of length 4 at L >= 5
    G4 = W.sparse_P(U, dims).copy()
    import scipy.sparse as sp
    G = sp.kron(sp.identity(L.volume(dims)), sp.kron(sp.csr_matrix(L.GAMMA[3]), sp.identity(3))).tocsr()
    trG4P4 = (G @ P2).multiply(P2.T).sum()
    assert abs(trG4P4) < 1e-10 * abs(trP4)


def test_free_field_trace_P4_closed_form():
    """Tr P^4 / V = -1152 at L >= 5 (= -64 * 18 unit plaquettes per site)."""
    dims = (6, 6, 6, 6)
    P = W.sparse_P(unit_links(dims), dims)
    P2 = (P @ P).tocsr()
    assert abs(P2.multiply(P2.T).sum() / L.volume(dims) + 1152.0) < 1e-9


def test_even_odd_solution_matches_full():
    dims = (4, 4, 2, 2)
    U = random_su3_links(dims, 0.3, 21)
    kappa = 0.12
    eta = _rand_field(dims, seed=3)
    M = W.dense_M(U, kappa, dims)
    x = np.linalg.solve(M, eta.ravel()).reshape(eta.shape)
    # reduced system on even sites, dense in the even subspace
    ev, od = L.eo_tables(dims)
    par = L.parity(dims).ravel()
    idx_e = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in ev])
    Mhat = np.zeros((idx_e.size, idx_e.size), dtype=complex)
    for col in range(idx_e.size):
        e = np.zeros(12 * L.volume(dims), dtype=complex)
        e[idx_e[col]] = 1
        Mhat[:, col] = W.apply_Mhat(U, kappa, e.reshape(eta.shape), dims).ravel()[idx_e]
    rhs = W.eo_source(U, kappa, eta, dims).ravel()[idx_e]
    xe = np.zeros(12 * L.volume(dims), dtype=complex)
    xe[idx_e] = np.linalg.solve(Mhat, rhs)
    xfull = W.eo_reconstruct(U, kappa, xe.reshape(eta.shape), eta, dims)
    assert np.abs(xfull - x).max() < 1e-12
