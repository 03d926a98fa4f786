"""The Wilson matrix and its reductions (oracle; test infrastructure only).

Sec. 5.1, Eqs. (24)-(25): M = 1 - kappa P with the hopping matrix

  (P psi)(x) = sum_mu [ (1 - g_mu) U_mu(x) psi(x + mu)
                      + (1 + g_mu) U_mu(x - mu)^dagger psi(x - mu) ].

(Sec. 5.2 once writes "M = I + kappa P"; the sign of Eq. (24), also implied
by the expansion I + kappa P + (kappa P)^2 + ... of Eq. (27), is the one
used throughout.)

Sec. 7: even/odd preconditioning gives the reduced system
  Mhat x_e = eta_e + kappa D_eo eta_o,   Mhat = 1 - kappa^2 D_eo D_oe,
  x_o = eta_o + kappa D_oe x_e,
with D_eo (D_oe) the block of P from odd to even (even to odd) sites.
Sec. 5.4, Eq. (63): M' = M g5 (multiplication on the right).

Two independent constructions of P are given: `hop` (array shifts) and
`dense_P` (matrix elements filled from the index form of Eq. (25)); the
tests pin them to each other, to the free-field plane-wave spectrum, to
g5-hermiticity, to gauge covariance and to the plaquette form of Tr P^4.
"""
import numpy as np

from .lattice import GAMMA, GAMMA5, volume

_ONE = np.eye(4, dtype=np.complex128)
_PROJ_MINUS = np.array([_ONE - GAMMA[mu] for mu in range(4)])  # forward hop
_PROJ_PLUS = np.array([_ONE + GAMMA[mu] for mu in range(4)])   # backward hop


def _axis(mu):
    # field axes are (t, z, y, x, spin, colour); direction mu = x,y,z,t
    return 3 - mu


def hop(U, psi):
    """P psi for fields of shape (..., Lt, Lz, Ly, Lx, 4, 3).

    Per site the field is a 4x3 (spin x colour) matrix F, so the colour
    rotation U F^T is written F @ U^T and the spin factor (1 -+ g) @ F."""
    out = np.zeros(psi.shape, dtype=np.complex128)
    nlead = psi.ndim - 6
    for mu in range(4):
        ax = nlead + _axis(mu)
        Umu = U[..., mu, :, :]
        UmuT = np.swapaxes(Umu, -1, -2)
        fwd = np.roll(psi, -1, axis=ax)                  # psi(x + mu)
        out += _PROJ_MINUS[mu] @ (fwd @ UmuT)             # (1 - g) U_mu(x) psi(x + mu)
        t = psi @ np.conj(Umu)                           # U_mu(x)^dagger psi(x)
        t = np.roll(t, +1, axis=ax)                      # at x: from x - mu
        out += _PROJ_PLUS[mu] @ t                        # (1 + g) U_mu(x - mu)^+ psi(x - mu)
    return out


def apply_M(U, kappa, psi):
    """M psi = psi - kappa P psi (Eq. (24))."""
    return psi - kappa * hop(U, psi)


def apply_Mdag(U, kappa, psi):
    """M^dagger psi = g5 M g5 psi."""
    return g5(apply_M(U, kappa, g5(psi)))


def g5(psi):
    return np.einsum("st,...tb->...sb", GAMMA5, psi)


def apply_Mprime(U, kappa, psi):
    """M' psi = M (g5 psi) (Eq. (63)); M' is hermitian."""
    return apply_M(U, kappa, g5(psi))


def apply_theta(theta, psi):
    """Theta psi for theta = 0 (identity) or 1..4 (g_mu, mu = theta-1)."""
    if theta == 0:
        return psi.copy()
    return np.einsum("st,...tb->...sb", GAMMA[theta - 1], psi)


# ---------------------------------------------------------------- even / odd
def parity_mask(dims):
    from .lattice import parity
    p = parity(dims)
    return p[..., None, None]


def D_eo(U, psi_odd_full, dims):
    """Hop restricted to even output sites of a field supported on odd sites.

    Works on full-lattice arrays (zeros on the other parity) so that the
    definitions stay visible; returns a full array that is zero on odd sites.
    """
    par = parity_mask(dims)
    return np.where(par == 0, hop(U, np.where(par == 1, psi_odd_full, 0)), 0)


def D_oe(U, psi_even_full, dims):
    par = parity_mask(dims)
    return np.where(par == 1, hop(U, np.where(par == 0, psi_even_full, 0)), 0)


def apply_Mhat(U, kappa, xe_full, dims):
    """Mhat x_e = x_e - kappa^2 D_eo D_oe x_e on even sites (full-lattice array)."""
    par = parity_mask(dims)
    xe = np.where(par == 0, xe_full, 0)
    return xe - kappa * kappa * D_eo(U, D_oe(U, xe, dims), dims)


def eo_source(U, kappa, eta, dims):
    """eta_hat_e = eta_e + kappa D_eo eta_o (full array, zero on odd sites)."""
    par = parity_mask(dims)
    return np.where(par == 0, eta, 0) + kappa * D_eo(U, eta, dims)


def eo_reconstruct(U, kappa, xe_full, eta, dims):
    """Full solution from the even part: x_o = eta_o + kappa D_oe x_e."""
    par = parity_mask(dims)
    xe = np.where(par == 0, xe_full, 0)
    return xe + np.where(par == 1, eta, 0) + kappa * D_oe(U, xe, dims)


# ------------------------------------------------------------ dense builders
def dense_P(U, dims):
    """The hopping matrix as a dense (12V x 12V) array, element by element.

    Row/column index (s * 4 + spin) * 3 + colour.  Entries accumulate, so
    on L = 2 extents (where x + mu and x - mu coincide) both terms land on
    the same block, as the sum in Eq. (25) requires.
    """
    Lx, Ly, Lz, Lt = dims
    L = (Lx, Ly, Lz, Lt)
    V = volume(dims)
    P = np.zeros((12 * V, 12 * V), dtype=np.complex128)

    def site(c):
        return c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]))

    for t in range(Lt):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    c = (x, y, z, t)
                    s = site(c)
                    for mu in range(4):
                        cp = list(c); cp[mu] = (cp[mu] + 1) % L[mu]
                        cm = list(c); cm[mu] = (cm[mu] - 1) % L[mu]
                        sp, sm = site(cp), site(cm)
                        Uf = U[t, z, y, x, mu]
                        Ub = U[cm[3], cm[2], cm[1], cm[0], mu]
                        P[12 * s:12 * s + 12, 12 * sp:12 * sp + 12] += np.kron(_PROJ_MINUS[mu], Uf)
                        P[12 * s:12 * s + 12, 12 * sm:12 * sm + 12] += np.kron(_PROJ_PLUS[mu], Ub.conj().T)
    return P


def dense_gamma(op, V):
    """Block-diagonal 12V x 12V matrix of a 4x4 spin matrix."""
    return np.kron(np.eye(V), np.kron(op, np.eye(3)))


def dense_M(U, kappa, dims):
    V = volume(dims)
    return np.eye(12 * V, dtype=np.complex128) - kappa * dense_P(U, dims)


def sparse_P(U, dims):
    """The hopping matrix as a scipy.sparse CSR matrix (same index order).

    Built from the same matrix elements as `dense_P` but vectorised over
    sites, for lattices where a dense 12V x 12V array does not fit."""
    import scipy.sparse as sp
    from .lattice import coords
    Lx, Ly, Lz, Lt = dims
    L = (Lx, Ly, Lz, Lt)
    V = volume(dims)
    x, y, z, t = (a.ravel() for a in coords(dims))
    c = [x, y, z, t]

    def site(cc):
        return cc[0] + Lx * (cc[1] + Ly * (cc[2] + Lz * cc[3]))

    s = site(c)
    Uf = U.reshape(V, 4, 3, 3)
    rows, cols, vals = [], [], []
    ii = np.arange(12)
    for mu in range(4):
        cp = list(c); cp[mu] = (c[mu] + 1) % L[mu]
        cm = list(c); cm[mu] = (c[mu] - 1) % L[mu]
        sp_, sm = site(cp), site(cm)
        fwd = np.einsum("st,xab->xsatb", _PROJ_MINUS[mu], Uf[:, mu]).reshape(V, 12, 12)
        bwd = np.einsum("st,xba->xsatb", _PROJ_PLUS[mu], np.conj(Uf[sm, mu])).reshape(V, 12, 12)
        for nb, blk in ((sp_, fwd), (sm, bwd)):
            rows.append(np.repeat((12 * s)[:, None] + ii, 12, axis=1).reshape(V, 12, 12))
            cols.append(np.tile((12 * nb)[:, None, None] + ii[None, None, :], (1, 12, 1)))
            vals.append(blk)
    r = np.concatenate([a.ravel() for a in rows])
    cc = np.concatenate([a.ravel() for a in cols])
    v = np.concatenate([a.ravel() for a in vals])
    return sp.csr_matrix((v, (r, cc)), shape=(12 * V, 12 * V))
