"""Subtraction matrices and their trace corrections (oracle; test infra only).

Sec. 4, Eqs. (14)-(15): subtracting tilde-M^{-1} eta from the solution keeps
the trace estimate unbiased once Tr(Theta tilde-M^{-1}) is added back, and
the variance then depends only on the off-diagonal part of
Theta (M^{-1} - tilde-M^{-1}).  The methods differ in tilde-M^{-1}:

PS (Sec. 5.1, Eqs. (27)-(31)):  sum_{j=0}^{n} (kappa P)^j; "order" n is the
    highest power (the paper's seventh order is n = 6).
POLY (Sec. 5.2, Eqs. (40)-(46)): the minimum-residual polynomial
    p(M) = sum_k a_k M^k minimising |(M p(M) - 1) b| for one noise vector b
    (the normal equations of Eq. (44) with v = (Mb ... M^{d+1} b)).  The same
    minimiser is computed by Householder QR in the kappa P basis
    (sum_j c_j (kappa P)^j, kappa P = 1 - M), which is better conditioned;
    a_k are recovered by the binomial map for reporting (Eq. (46) read in
    reverse).
HFES (Sec. 5.4, Eqs. (66)-(68)): g5 sum_q e'_q e'_q^dagger / lambda'_q with
    (lambda'_q, e'_q) the Q eigenpairs of M' = M g5 of smallest |lambda'|.
HFPOLY / HFPS (Sec. 5.5, Eqs. (69)-(72)): HFES + POLY (or PS) minus the
    overlap g5 sum_q e'_q e'_q^dagger / xi'_q, 1/xi'_q = e'_q^dagger g5 p e'_q
    (M'_poly^{-1} = (p^{-1} g5)^{-1} = g5 p).

Trace corrections (Eqs. (34), (47), the HFES term of Eq. (66) and the last
two terms of Eq. (70)) are returned per timeslice for Theta in {1, g_1..g_4}
(theta code 0..4).  The polynomial ones are computed exactly from the
diagonal 12x12 blocks of p(kappa P): by dense matrix powers (small
lattices) or by unit-vector probes at chosen sites.
"""
import numpy as np
from math import comb

from .lattice import GAMMA, GAMMA5, volume
from .wilson import hop, apply_M, g5


def theta_matrix(theta):
    return np.eye(4, dtype=np.complex128) if theta == 0 else GAMMA[theta - 1]


# ------------------------------------------------------------- polynomials
def horner(U, kappa, eta, coeffs):
    """sum_j coeffs[j] (kappa P)^j eta by Horner's rule."""
    y = coeffs[-1] * eta
    for cj in coeffs[-2::-1]:
        y = cj * eta + kappa * hop(U, y)
    return y


def pert_coeffs(order):
    return np.ones(order + 1, dtype=np.complex128)


def pert_vector(U, kappa, eta, order):
    """x_pert = sum_{j=0}^{order} (kappa P)^j eta (Eq. (31))."""
    return horner(U, kappa, eta, pert_coeffs(order))


def poly_coeffs(U, kappa, b, degree):
    """Min-Res polynomial of degree d for the noise vector b.

    Returns (c, a): c[j] multiplies (kappa P)^j, a[k] multiplies M^k; both
    describe the same polynomial.  Columns w_j = M (kappa P)^j b, j = 0..d;
    c = argmin |b - W c| by Householder QR.
    """
    cols = []
    y = b.astype(np.complex128)
    for j in range(degree + 1):
        cols.append(apply_M(U, kappa, y).ravel())
        y = kappa * hop(U, y)
    W = np.stack(cols, axis=1)
    Qm, R = np.linalg.qr(W)
    c = np.linalg.solve(R, Qm.conj().T @ b.ravel())
    return c, kp_to_m_basis(c)


def kp_to_m_basis(c):
    """(kappa P)^j = (1 - M)^j = sum_k C(j,k) (-1)^k M^k."""
    d = len(c) - 1
    a = np.zeros(d + 1, dtype=np.complex128)
    for j in range(d + 1):
        for k in range(j + 1):
            a[k] += c[j] * comb(j, k) * (-1) ** k
    return a


def m_to_kp_basis(a):
    """M^k = (1 - kappa P)^k = sum_j C(k,j) (-1)^j (kappa P)^j."""
    d = len(a) - 1
    c = np.zeros(d + 1, dtype=np.complex128)
    for k in range(d + 1):
        for j in range(k + 1):
            c[j] += a[k] * comb(k, j) * (-1) ** j
    return c


def poly_vector(U, kappa, eta, c):
    return horner(U, kappa, eta, c)


# -------------------------------------------------------- exact corrections
def block_traces(blocks, thetas):
    """tr(Theta B) for 12x12 site blocks B[..., 12, 12] (spin-major)."""
    B = blocks.reshape(blocks.shape[:-2] + (4, 3, 4, 3))
    out = []
    for th in thetas:
        T = theta_matrix(th)
        out.append(np.einsum("st,...tasa->...", T, B))
    return np.stack(out, axis=0)


def diag_blocks_dense(A, V):
    """12x12 diagonal blocks of a dense 12V x 12V matrix, shape (V, 12, 12)."""
    idx = np.arange(V)
    A4 = A.reshape(V, 12, V, 12)
    return A4[idx, :, idx, :]


def poly_dense(Pd, kappa, coeffs):
    """Dense p(kappa P) = sum_j coeffs[j] (kappa P)^j by Horner on matrices."""
    n = Pd.shape[0]
    R = coeffs[-1] * np.eye(n, dtype=np.complex128)
    for cj in coeffs[-2::-1]:
        R = cj * np.eye(n) + kappa * (Pd @ R)
    return R


def per_timeslice(site_values, dims):
    """Sum per-site values (..., V) into (..., Lt) timeslice sums."""
    Lx, Ly, Lz, Lt = dims
    sv = np.asarray(site_values)
    return sv.reshape(sv.shape[:-1] + (Lt, Lx * Ly * Lz)).sum(axis=-1)


def trace_correction_dense(A, dims, thetas):
    """Tr_t(Theta A) per timeslice for a dense 12V x 12V matrix A."""
    V = volume(dims)
    return per_timeslice(block_traces(diag_blocks_dense(A, V), thetas), dims)


def diag_blocks_probe(U, kappa, coeffs, dims, sites):
    """Diagonal blocks of p(kappa P) at the given lexicographic sites, from
    12 unit-vector probes per site (Eqs. (32)-(34)): column alpha of block
    x is (p(kappa P) e_{x,alpha})(x)."""
    Lx, Ly, Lz, Lt = dims
    V = volume(dims)
    out = np.zeros((len(sites), 12, 12), dtype=np.complex128)
    for n, s in enumerate(sites):
        probes = np.zeros((12, V * 12), dtype=np.complex128)
        probes[np.arange(12), 12 * s + np.arange(12)] = 1.0
        probes = probes.reshape(12, Lt, Lz, Ly, Lx, 4, 3)
        y = horner(U, kappa, probes, coeffs).reshape(12, V, 12)
        out[n] = y[:, s, :].T
    return out


def trace_correction_probe(U, kappa, coeffs, dims, thetas):
    """Exact Tr_t(Theta p(kappa P)) from unit-vector probes at every site."""
    V = volume(dims)
    blocks = diag_blocks_probe(U, kappa, coeffs, dims, range(V))
    return per_timeslice(block_traces(blocks, thetas), dims)


# ---------------------------------------------------------- hermitian forced
def site_bilinear(E, thetas, dims, weights):
    """sum_q w_q e_q(x)^dagger Theta g5 e_q(x) per timeslice.

    E: (Q, Lt, Lz, Ly, Lx, 4, 3) eigenvectors; weights: (Q,)."""
    V = volume(dims)
    Ef = E.reshape(E.shape[0], V, 4, 3)
    res = []
    for th in thetas:
        T = theta_matrix(th) @ GAMMA5
        v = np.einsum("qxsa,st,qxta->qx", np.conj(Ef), T, Ef)
        res.append(np.einsum("q,qx->x", weights, v))
    return per_timeslice(np.stack(res, axis=0), dims)


def eig_vector(E, inv_vals, eta):
    """g5 sum_q inv_vals[q] e_q (e_q^dagger eta) for eta of shape (n, field)."""
    Q = E.shape[0]
    Ef = E.reshape(Q, -1)
    ef = eta.reshape(eta.shape[0], -1)
    coef = (np.conj(Ef) @ ef.T) * inv_vals[:, None]       # (Q, n)
    y = (coef.T @ Ef).reshape(eta.shape)
    return g5(y)


def xi_inverse(U, kappa, E, coeffs):
    """1/xi'_q = e'_q^dagger g5 p(kappa P) e'_q (Eq. (69))."""
    out = np.zeros(E.shape[0], dtype=np.complex128)
    for q in range(E.shape[0]):
        y = g5(horner(U, kappa, E[q], coeffs))
        out[q] = np.vdot(E[q].ravel(), y.ravel())
    return out
