"""Eigenvalue subtraction, ES (Sec. 5.3) (oracle; test infrastructure only).

The subtraction matrix is built from the Q eigenpairs of the full Wilson
matrix M with smallest |lambda| and biorthonormal right and left
eigenvectors (e_L^(q)^+ e_R^(q') = delta):
    Mt_eig^{-1} = sum_q (1 / lambda_q) e_R^(q) e_L^(q)^+,
    xt^(n) = sum_q (1 / lambda_q) e_R^(q) (e_L^(q)^+ eta^(n)),
    Tr_t(Theta Mt_eig^{-1}) = sum_q (1 / lambda_q) sum_{x in t} e_L^(q)(x)^+ (Theta e_R^(q))(x)
(with all N pairs, Tr(Mt^{-1}) = sum 1/lambda, the paper's closed form).

The pairs come from the even/odd GMRES-DR data of the first noise vector
(Sec. 7), with the relation between reduced and full eigenvectors written
out here (the paper only states that it exists):
  * Ritz pairs of Mhat in span(V_k): H_k = V_k^+ Mhat V_k = S diag(lh) S^{-1},
    right vectors rh = V_k S.  The Krylov space holds the right
    eigenvectors, not the left ones (Mhat is not normal), so the left
    vectors come from g5-hermiticity, Mhat^+ = g5 Mhat g5: the left
    eigenvector of lh is g5 times the right one of conj(lh) (the Ritz value
    closest to conj(lh)), scaled so that lh_vec^+ rh = 1;
  * M = [[1, -kappa D_eo], [-kappa D_oe, 1]] in (even, odd) blocks and
    Mhat = 1 - kappa^2 D_eo D_oe: for Mhat rh = lh rh, the full vector
    r = (rh, kappa / (1 - lambda) D_oe rh) is a right eigenvector of M
    whenever (1 - lambda)^2 = 1 - lh; the small-|lambda| branch is
    lambda = 1 - sqrt(1 - lh) (principal square root);
  * the left vector of the same lambda, l^+ M = lambda l^+, is
    (lh_vec, kappa / (1 - conj lambda) D_eo^+ lh_vec) with D_eo^+ = g5 D_oe g5
    (g5-hermiticity of the hop); then l^+ r = 2 lh_vec^+ rh, so l is halved.
"""
import numpy as np

from .lattice import volume
from . import wilson as W
from . import subtract as S
from . import pointsplit as PSO


def ritz_pairs_eo(defl_V, defl_H, g5):
    """Right/left Ritz pairs of Mhat from A V_k = V_{k+1} Hbar_k: (lh, Rh, Lh)
    with Rh, Lh of shape (n, k) and diag(Lh^+ Rh) = 1.  g5 applies gamma_5
    to a flattened field."""
    k = defl_H.shape[1]
    Hk = defl_H[:k, :k]
    lh, Sr = np.linalg.eig(Hk)
    Rh = defl_V[:, :k] @ Sr
    Lh = np.empty_like(Rh)
    for q in range(k):
        p = int(np.argmin(np.abs(lh - np.conj(lh[q]))))   # the conjugate partner
        l = g5(Rh[:, p])
        Lh[:, q] = l / np.conj(np.vdot(l, Rh[:, q]))
    return lh, Rh, Lh


def full_pairs(U, kappa, dims, lh, Rh, Lh, branch=1):
    """Full-lattice eigenpairs of M from even-site Ritz pairs of Mhat.

    Rh, Lh: (n, k) columns that are full-lattice fields (zero on odd sites)
    flattened.  branch = 1 takes lambda = 1 - sqrt(1 - lh) (the small
    eigenvalues), -1 the other root 1 + sqrt(1 - lh).  Returns lam (k,), R, L
    of shape (k, field) with L[q]^+ R[q] = 1."""
    shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    lam = 1.0 - branch * np.sqrt(1.0 - lh.astype(np.complex128))
    R, L = [], []
    for q in range(lh.size):
        rh = Rh[:, q].reshape(shape)
        lv = Lh[:, q].reshape(shape)
        r = rh + kappa / (1.0 - lam[q]) * W.D_oe(U, rh, dims)
        l = lv + kappa / (1.0 - np.conj(lam[q])) * W.g5(W.D_oe(U, W.g5(lv), dims))
        R.append(r)
        L.append(0.5 * l)
    return lam, np.stack(R), np.stack(L)


def smallest(lam, R, L, Q):
    """The Q pairs of smallest |lambda| (ties: index order)."""
    order = np.lexsort((np.arange(lam.size), np.abs(lam)))[:Q]
    return lam[order], R[order], L[order]


def es_vector(R, L, lam, eta):
    """xt^(n) = sum_q (1/lambda_q) R[q] (L[q]^+ eta^(n)), eta of shape (n, field)."""
    Q = lam.size
    Rf, Lf = R.reshape(Q, -1), L.reshape(Q, -1)
    ef = eta.reshape(eta.shape[0], -1)
    coef = (np.conj(Lf) @ ef.T) / lam[:, None]          # (Q, n)
    return (coef.T @ Rf).reshape(eta.shape)


def es_trace(U, kappa, R, L, lam, thetas, dims):
    """Tr_t(Theta Mt_eig^{-1}) per operator code (0..8) and timeslice."""
    V = volume(dims)
    Q = lam.size
    rows = []
    for th in thetas:
        acc = np.zeros(V, dtype=np.complex128)
        for q in range(Q):
            if th < 5:
                y = W.apply_theta(th, R[q])
            else:
                y = PSO.apply_theta_ps(U, kappa, th - 5, R[q])
            acc += np.einsum("xi,xi->x", np.conj(L[q].reshape(V, 12)), y.reshape(V, 12)) / lam[q]
        rows.append(acc)
    return S.per_timeslice(np.stack(rows), dims)
