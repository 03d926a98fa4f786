"""Pins for the oracle's subtraction polynomials and trace corrections (CPU).

* POLY: the QR minimiser equals numpy's least-squares solution and satisfies
  the paper's normal equations (v^dagger v) a = v^dagger b with
  v = (Mb ... M^{d+1} b) in the M basis (Eq. (44)); degree 0 reduces to
  c0 = (Mb)^dagger b / |Mb|^2.
* Trace corrections: dense matrix powers and unit-vector probes agree;
  free-field Tr P^j = 12 sum_p Re (C + i|S|)^j (C = 2 sum cos p,
  S_mu = 2 sin p_mu); on 4^4 random links
  Tr P^4 = -64 sum_plaq Re tr U_P + 64 sum_{x,mu} Re tr L_mu(x) and
  Tr g4 P^4 = -64 i sum_x Im tr L_4(x) (L_mu the length-4 Polyakov loops);
  odd orders have no diagonal; gauge invariance.
* Hopping expansion: Tr(Theta M^{-1}) - sum_{j<=n} kappa^j Tr(Theta P^j)
  falls like kappa^{n+2} (n even, odd orders vanish).
"""
import itertools

import numpy as np
import pytest

from synth import random_su3_links, unit_links
from oracle import lattice as L
from oracle import wilson as W
from oracle import subtract as S
from oracle.noise import z4_noise

THETAS = (0, 1, 2, 3, 4)


def test_poly_coefficients_least_squares():
    dims = (4, 2, 2, 4)
    U = random_su3_links(dims, 0.3, 41)
    kappa = 0.12
    b = z4_noise(9, dims, 0, 1)[0]
    d = 5
    c, a = S.poly_coeffs(U, kappa, b, d)
    # same minimiser as a library least-squares solve on the M^k b basis
    cols = []
    y = b.copy()
    for j in range(d + 2):
        cols.append(y.ravel())
        y = W.apply_M(U, kappa, y)
    v = np.stack(cols[1:], axis=1)          # (Mb ... M^{d+1} b)
    a_ls = np.linalg.lstsq(v, b.ravel(), rcond=None)[0]
    assert np.abs(a - a_ls).max() < 1e-8 * np.abs(a).max()
    # normal equations (v^dagger v) a = v^dagger b hold as orthogonality
    r = b.ravel() - v @ a
    assert np.abs(v.conj().T @ r).max() < 1e-10 * np.linalg.norm(b) * np.linalg.norm(v)
    # basis maps are inverse to each other
    assert np.abs(S.m_to_kp_basis(S.kp_to_m_basis(c)) - c).max() < 1e-10 * np.abs(c).max()


def test_poly_degree_zero_closed_form():
    dims = (2, 2, 2, 4)
    U = random_su3_links(dims, 0.3, 42)
    kappa = 0.11
    b = z4_noise(3, dims, 0, 1)[0]
    c, a = S.poly_coeffs(U, kappa, b, 0)
    Mb = W.apply_M(U, kappa, b).ravel()
    assert abs(c[0] - np.vdot(Mb, b.ravel()) / np.vdot(Mb, Mb)) < 1e-14
    assert abs(a[0] - c[0]) < 1e-15


def _free_trace(dims, j):
    tot = 0.0
    for p in itertools.product(*[2 * np.pi * np.arange(n) / n for n in dims]):
        C = 2 * np.cos(p).sum()
        Sm = 2 * np.sqrt((np.sin(p) ** 2).sum())
        tot += 12 * ((C + 1j * Sm) ** j).real
    return tot


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 2, 2, 2), (4, 2, 6, 2)])
def test_free_field_trace_powers(dims):
    V = L.volume(dims)
    Pd = W.dense_P(unit_links(dims), dims)
    A = np.eye(12 * V, dtype=complex)
    for j in range(1, 7):
        A = Pd @ A
        tr = S.trace_correction_dense(A, dims, (0,)).sum()
        assert abs(tr - _free_trace(dims, j)) < 1e-8 * max(1.0, abs(tr))
    if dims == (4, 4, 4, 4):
        # published-size check values: -384 and -9216 per site on 4^4
        assert abs(_free_trace(dims, 4) / V + 384) < 1e-9
        assert abs(_free_trace(dims, 6) / V + 9216) < 1e-9


def test_free_field_large_L_by_probe():
    """Tr P^4 / V = -1152 and Tr P^6 / V = -50688 once L >= 7 (8^4);
    translation invariance lets one site's diagonal block stand for all."""
    dims = (8, 8, 8, 8)
    U = unit_links(dims)
    V = L.volume(dims)
    for j, ref in ((4, -1152.0), (6, -50688.0)):
        coeffs = np.zeros(j + 1, dtype=complex)
        coeffs[j] = 1.0
        blk = S.diag_blocks_probe(U, 1.0, coeffs, dims, [0])
        assert abs(np.trace(blk[0]).real - ref) < 1e-8
        assert abs(_free_trace(dims, j) / V - ref) < 1e-7


def _polyakov(U, mu):
    ax = 3 - mu
    Umu = U[..., mu, :, :]
    P = Umu.copy()
    for s in range(1, 4):
        P = P @ np.roll(Umu, -s, axis=ax)
    return np.trace(P, axis1=-2, axis2=-1)


def test_random_links_4x4_windings():
    from tests.test_oracle_wilson import plaquette_sum
    dims = (4, 4, 4, 4)
    U = random_su3_links(dims, 0.3, 17)
    Ps = W.sparse_P(U, dims)
    P2 = (Ps @ Ps).tocsr()
    trP4 = P2.multiply(P2.T).sum()
    poly = sum(_polyakov(U, mu).real.sum() for mu in range(4))
    assert abs(trP4 - (-64 * plaquette_sum(U) + 64 * poly)) < 1e-10 * abs(trP4)
    import scipy.sparse as sp
    G4 = sp.kron(sp.identity(L.volume(dims)), sp.kron(sp.csr_matrix(L.GAMMA[3]), sp.identity(3))).tocsr()
    trG4P4 = (G4 @ P2).multiply(P2.T).sum()
    assert abs(trG4P4 - (-64j * _polyakov(U, 3).imag.sum())) < 1e-10 * abs(trP4)


@pytest.fixture(scope="module")
def small():
    dims = (4, 4, 2, 2)
    U = random_su3_links(dims, 0.35, 51)
    return dims, U, W.dense_P(U, dims)


def test_dense_and_probe_corrections_agree(small):
    dims, U, Pd = small
    kappa = 0.13
    rng = np.random.default_rng(4)
    for coeffs in (S.pert_coeffs(6), rng.standard_normal(6) + 1j * rng.standard_normal(6)):
        A = S.poly_dense(Pd, kappa, coeffs)
        dense = S.trace_correction_dense(A, dims, THETAS)
        probe = S.trace_correction_probe(U, kappa, coeffs, dims, THETAS)
        assert np.abs(dense - probe).max() < 1e-12 * np.abs(dense).max()


def test_odd_orders_have_no_diagonal(small):
    dims, U, Pd = small
    V = L.volume(dims)
    A = np.eye(12 * V, dtype=complex)
    for j in range(1, 8):
        A = Pd @ A
        if j % 2:
            assert np.abs(S.diag_blocks_dense(A, V)).max() < 1e-12


def test_corrections_gauge_invariant(small):
    dims, U, Pd = small
    g = random_su3_links(dims, 1.0, 77)[..., 1, :, :]
    Ug = np.empty_like(U)
    for mu in range(4):
        gp = np.roll(g, -1, axis=3 - mu)
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gp, -1, -2))
    c = S.pert_coeffs(6)
    a = S.trace_correction_dense(S.poly_dense(Pd, 0.12, c), dims, THETAS)
    b = S.trace_correction_dense(S.poly_dense(W.dense_P(Ug, dims), 0.12, c), dims, THETAS)
    assert np.abs(a - b).max() < 1e-11 * np.abs(a).max()


def test_hopping_expansion_slope(small):
    """Tr(Theta M^{-1}) minus its expansion through kappa^4 scales as kappa^6."""
    dims, U, Pd = small
    V = L.volume(dims)
    Id = np.eye(12 * V)
    for th in (0, 4):
        errs = []
        for kappa in (0.004, 0.008):
            Minv = np.linalg.inv(Id - kappa * Pd)
            exact = S.trace_correction_dense(Minv, dims, (th,)).sum()
            series = S.trace_correction_dense(S.poly_dense(Pd, kappa, S.pert_coeffs(4)), dims, (th,)).sum()
            errs.append(abs(exact - series))
        slope = np.log(errs[1] / errs[0]) / np.log(2.0)
        assert abs(slope - 6.0) < 0.1
