"""Deflated restarted Krylov solvers (oracle; test infrastructure only).

Sec. 7 solves the first noise vector with GMRES-DR(m, k) to
"super-convergence", keeping its k approximate low eigenvectors, and the
remaining noise vectors with GMRES-Proj, which alternates a minimum-residual
projection over those vectors with GMRES(m - k) cycles; the algorithms
themselves are only cited there (Morgan, SIAM J. Sci. Comput. 24 (2002) 20
for GMRES-DR; Morgan and Wilcox for GMRES-Proj).  The steps below follow
those published methods in plain FP64:

GMRES-DR(m, k)
  1. Arnoldi from v_1 = r0 / |r0| with classical Gram-Schmidt applied twice,
     giving A V_m = V_{m+1} Hbar_m; c = |r0| e_1.
  2. d = argmin |c - Hbar_m d|, x += V_m d, s = c - Hbar_m d (|s| = |r|).
  3. Harmonic Ritz pairs: (H_m + |h_{m+1,m}|^2 f e_m^T) g = theta g with
     H_m^* f = e_m; keep the k of smallest |theta|.
  4. P_{k+1}: orthonormalise the k vectors g (padded with a zero row) and
     the residual direction (s, or the parallel vector w of `harmonic_ritz`).
  5. V_{k+1} <- V_{m+1} P_{k+1}, Hbar_k <- P_{k+1}^* Hbar_m P_k,
     c <- P_{k+1}^* s; Arnoldi continues from v_{k+1} to v_{m+1}
     (orthogonalising against all previous vectors); back to 2.
  After the last cycle one more step 3-5 leaves the deflation data
  (V_{k+1}, Hbar_k) with A V_k = V_{k+1} Hbar_k.

GMRES-Proj(m - k, k) for every later right-hand side
  repeat { c = V_{k+1}^* r; d = argmin |c - Hbar_k d|; x += V_k d;
           one GMRES(m - k) cycle from the new residual;
           r = b - A x } until |r| <= tol |b|.

MINRES-DR(m, k) for a hermitian (indefinite) A, e.g. M' = M g5 near the
critical kappa, where Sec. 8 switches from GMRES-DR to it (the method is
only cited there; the steps below are this module's reading of deflated
restarting with a symmetric Lanczos recurrence):
  1. as GMRES-DR step 1, except that after the first new column of a cycle
     (which is orthogonalised against every kept vector) each new vector is
     orthogonalised by the three-term recurrence against v_{j-1}, v_j, then
     once more against those two and against the k + 1 kept vectors of the
     last restart (selective reorthogonalisation against the approximate
     eigenvectors, which is where a Lanczos basis loses orthogonality);
  2. as GMRES-DR step 2;
  3. harmonic Ritz pairs from the pencil H_m^* g = mu Hbar_m^* Hbar_m g
     with the positive definite Hbar_m^* Hbar_m = L L^*, as the eigenproblem
     of L^{-1} H_m^* L^{-*}, theta = 1 / mu (equivalent to step 3 of
     GMRES-DR, but it never solves with H_m, which turns singular when a
     Ritz value of an indefinite A crosses zero).  H_m is used as computed,
     not made hermitian: pairs of a hermitised H_m are not exact for the
     computed Hbar_m, their residuals leave the kept residual direction, and
     the restart relation then degrades from cycle to cycle;
  4. the residual direction is the unit vector orthogonal to the range of
     Hbar_m (last column of its complete QR); then as GMRES-DR steps 4-5.

Hermitian eigenpairs (Sec. 5.4): GMRES-DR on M' (full lattice) followed by
Rayleigh-Ritz in V_k: T = V_k^* M' V_k = (Hbar_k)[:k, :k], hermitised,
eigh(T) = (lambda', s), e' = V_k s; the Q of smallest |lambda'| are kept.

Iteration counts are not pinned (they depend on rounding); tests compare
only converged quantities (solutions, harmonic Ritz values, eigenpairs).
"""
import numpy as np


def _cgs2(V, w):
    h = V.conj().T @ w
    w = w - V @ h
    h2 = V.conj().T @ w
    w = w - V @ h2
    return w, h + h2


def arnoldi(A, V, H, j0, m, stats):
    """Extend the Arnoldi relation from column j0 to column m (in place)."""
    for j in range(j0, m):
        w = A(V[:, j])
        stats["matvecs"] += 1
        w, h = _cgs2(V[:, :j + 1], w)
        H[:j + 1, j] = h
        nrm = np.linalg.norm(w)
        H[j + 1, j] = nrm
        if nrm == 0.0:
            raise FloatingPointError("Arnoldi breakdown at column %d" % j)
        V[:, j + 1] = w / nrm


def _lstsq(H, c):
    return np.linalg.lstsq(H, c, rcond=None)[0]


def harmonic_ritz(H, m):
    """Harmonic Ritz values/vectors of the (m+1) x m Hessenberg matrix H.

    Also returns w = [-|h|^2 f; h] (h = H[m, m-1]), the common direction of
    every harmonic residual Hbar_m g - theta [g; 0] and of the GMRES
    least-squares residual c - Hbar_m d (both are orthogonal to the range
    of Hbar_m)."""
    Hm = H[:m, :m]
    em = np.zeros(m, dtype=np.complex128)
    em[-1] = 1.0
    f = np.linalg.solve(Hm.conj().T, em)
    h = H[m, m - 1]
    G = Hm + abs(h) ** 2 * np.outer(f, em)
    theta, g = np.linalg.eig(G)
    w = np.concatenate([-abs(h) ** 2 * f, [h]])
    return theta, g, w


def _deflation_restart(V, H, s, m, k):
    theta, g, w = harmonic_ritz(H, m)
    order = np.lexsort((np.arange(m), np.abs(theta)))[:k]
    Pm = np.zeros((m + 1, k + 1), dtype=np.complex128)
    Pm[:m, :k] = g[:, order]
    # The (k+1)-th column spans the residual direction.  s = c - Hbar d is
    # parallel to w in exact arithmetic but loses its direction to
    # cancellation once |s| << |c|; w carries the same direction accurately.
    Pm[:, k] = w
    Q, _ = np.linalg.qr(Pm)
    Hk = Q.conj().T @ H @ Q[:m, :k]
    Vnew = V @ Q
    cnew = Q.conj().T @ s
    # |A y - theta y| for y = V_m g / |g|: |e_m^T g| |w| / |g|
    gk = g[:, order]
    resid = np.abs(gk[m - 1, :]) * np.linalg.norm(w) / np.linalg.norm(gk, axis=0)
    return Vnew, Hk, cnew, theta[order], resid


def gmres_dr(A, b, m, k, tol, max_cycles=500, x0=None, eig_tol=None, n_eig=None):
    """Solve A x = b; returns (x, info) with info['V'], info['H'] the
    deflation data (V_{k+1}: n x (k+1), Hbar_k: (k+1) x k) and
    info['theta'] the k harmonic Ritz values of the final restart and
    info['theta_resid'] their residual norms |A y - theta y| (|y| = 1).

    Super-convergence: with eig_tol set, cycles continue after the residual
    test passes until the n_eig (default k) harmonic Ritz pairs of smallest
    |theta| also satisfy |A y - theta y| <= eig_tol |theta|."""
    n = b.size
    x = np.zeros(n, dtype=np.complex128) if x0 is None else x0.astype(np.complex128).copy()
    stats = {"matvecs": 0, "cycles": 0}
    r = b - A(x) if x0 is not None else b.astype(np.complex128).copy()
    if x0 is not None:
        stats["matvecs"] += 1
    bnorm = np.linalg.norm(b)
    V = np.zeros((n, m + 1), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    beta = np.linalg.norm(r)
    V[:, 0] = r / beta
    c = np.zeros(m + 1, dtype=np.complex128)
    c[0] = beta
    j0 = 0
    hist = []
    while True:
        arnoldi(A, V, H, j0, m, stats)
        d = _lstsq(H, c)
        x += V[:, :m] @ d
        s = c - H @ d
        res = np.linalg.norm(s)
        hist.append(res / bnorm)
        stats["cycles"] += 1
        Vk1, Hk, ck, theta, theta_res = _deflation_restart(V, H, s, m, k)
        done = res <= tol * bnorm
        if done and eig_tol is not None:
            ne = k if n_eig is None else n_eig
            done = bool(np.all(theta_res[:ne] <= eig_tol * np.abs(theta[:ne])))
        if done or stats["cycles"] >= max_cycles:
            break
        V[:, :k + 1] = Vk1
        V[:, k + 1:] = 0
        H[:] = 0
        H[:k + 1, :k] = Hk
        c[:] = 0
        c[:k + 1] = ck
        j0 = k
    info = dict(V=Vk1, H=Hk, theta=theta, theta_resid=theta_res, history=hist, converged=res <= tol * bnorm, **stats)
    return x, info


def lanczos_extend(A, V, H, j0, m, kept, stats):
    """MINRES-DR basis extension from column j0 to column m (in place).

    Column j0 is orthogonalised (twice) against v_0 .. v_j0; every later
    column against v_{j-1}, v_j, then once more against v_{j-1}, v_j and the
    first `kept` vectors (the kept vectors of the last restart, 0 before the
    first restart).  Coefficients of both passes add into H, so
    A V_m = V_{m+1} Hbar_m holds to rounding."""
    for j in range(j0, m):
        w = A(V[:, j])
        stats["matvecs"] += 1
        if j == j0:
            w, h = _cgs2(V[:, :j + 1], w)
            H[:j + 1, j] = h
        else:
            near = [j - 1, j]
            h1 = V[:, near].conj().T @ w
            w = w - V[:, near] @ h1
            second = sorted(set(range(kept)) | set(near))
            h2 = V[:, second].conj().T @ w
            w = w - V[:, second] @ h2
            H[near, j] += h1
            H[second, j] += h2
        nrm = np.linalg.norm(w)
        H[j + 1, j] = nrm
        if nrm == 0.0:
            raise FloatingPointError("Lanczos breakdown at column %d" % j)
        V[:, j + 1] = w / nrm


def harmonic_ritz_hermitian(H, m):
    """Harmonic Ritz pairs of a hermitian operator from its (m+1) x m Hbar_m.

    The pencil H_m^* g = mu (Hbar_m^* Hbar_m) g with Hbar_m^* Hbar_m positive
    definite (Hbar_m has full column rank): with the Cholesky factor
    L L^* = Hbar_m^* Hbar_m it is the eigenproblem of the (hermitian up to
    rounding) L^{-1} H_m^* L^{-*}, y = L^* g, theta = 1 / mu.  Returns theta
    (inf where mu = 0), g and the unit vector w orthogonal to the range of
    Hbar_m, the common direction of the harmonic residuals."""
    Hm = H[:m, :m]
    B = H.conj().T @ H
    L = np.linalg.cholesky(B)
    Li = np.linalg.inv(L)
    mu, Y = np.linalg.eig(Li @ Hm.conj().T @ Li.conj().T)
    g = Li.conj().T @ Y
    with np.errstate(divide="ignore", invalid="ignore"):
        theta = np.where(mu != 0, 1.0 / np.where(mu != 0, mu, 1.0), np.inf)
    Qc, _ = np.linalg.qr(H, mode="complete")
    w = Qc[:, m]
    return theta.astype(np.complex128), g, w


def _deflation_restart_hermitian(V, H, s, m, k):
    theta, g, w = harmonic_ritz_hermitian(H, m)
    order = np.lexsort((np.arange(m), np.abs(theta)))[:k]
    gk = g[:, order]
    Pm = np.zeros((m + 1, k + 1), dtype=np.complex128)
    Pm[:m, :k] = gk
    Pm[:, k] = w
    Q, _ = np.linalg.qr(Pm)
    Hk = Q.conj().T @ H @ Q[:m, :k]
    Vnew = V @ Q
    cnew = Q.conj().T @ s
    gp = np.vstack([gk, np.zeros((1, k))])
    resid = np.linalg.norm(H @ gk - gp * theta[order], axis=0) / np.linalg.norm(gk, axis=0)
    return Vnew, Hk, cnew, theta[order], resid


def minres_dr(A, b, m, k, tol, max_cycles=500, x0=None, eig_tol=None, n_eig=None):
    """MINRES-DR(m, k) for hermitian A: same interface and outputs as gmres_dr."""
    n = b.size
    x = np.zeros(n, dtype=np.complex128) if x0 is None else x0.astype(np.complex128).copy()
    stats = {"matvecs": 0, "cycles": 0}
    r = b - A(x) if x0 is not None else b.astype(np.complex128).copy()
    if x0 is not None:
        stats["matvecs"] += 1
    bnorm = np.linalg.norm(b)
    V = np.zeros((n, m + 1), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    beta = np.linalg.norm(r)
    V[:, 0] = r / beta
    c = np.zeros(m + 1, dtype=np.complex128)
    c[0] = beta
    j0, kept = 0, 0
    hist = []
    while True:
        lanczos_extend(A, V, H, j0, m, kept, stats)
        d = _lstsq(H, c)
        x += V[:, :m] @ d
        s = c - H @ d
        res = np.linalg.norm(s)
        hist.append(res / bnorm)
        stats["cycles"] += 1
        Vk1, Hk, ck, theta, theta_res = _deflation_restart_hermitian(V, H, s, m, k)
        done = res <= tol * bnorm
        if done and eig_tol is not None:
            ne = k if n_eig is None else n_eig
            done = bool(np.all(theta_res[:ne] <= eig_tol * np.abs(theta[:ne])))
        if done or stats["cycles"] >= max_cycles:
            break
        V[:, :k + 1] = Vk1
        V[:, k + 1:] = 0
        H[:] = 0
        H[:k + 1, :k] = Hk
        c[:] = 0
        c[:k + 1] = ck
        j0, kept = k, k + 1
    info = dict(V=Vk1, H=Hk, theta=theta, theta_resid=theta_res, history=hist, converged=res <= tol * bnorm, **stats)
    return x, info


def gmres_cycle(A, r, p, stats):
    """One GMRES(p) cycle from residual r: returns the correction dx."""
    n = r.size
    V = np.zeros((n, p + 1), dtype=np.complex128)
    H = np.zeros((p + 1, p), dtype=np.complex128)
    beta = np.linalg.norm(r)
    V[:, 0] = r / beta
    arnoldi(A, V, H, 0, p, stats)
    c = np.zeros(p + 1, dtype=np.complex128)
    c[0] = beta
    d = _lstsq(H, c)
    return V[:, :p] @ d


def gmres_proj(A, b, defl_V, defl_H, p, tol, max_cycles=1000, x0=None):
    """GMRES-Proj: projection over (V_{k+1}, Hbar_k) alternated with GMRES(p)."""
    n = b.size
    k = defl_H.shape[1]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else x0.astype(np.complex128).copy()
    stats = {"matvecs": 0, "cycles": 0}
    r = b.astype(np.complex128) - (A(x) if x0 is not None else 0)
    bnorm = np.linalg.norm(b)
    hist = []
    while np.linalg.norm(r) > tol * bnorm and stats["cycles"] < max_cycles:
        c = defl_V.conj().T @ r
        d = _lstsq(defl_H, c)
        x = x + defl_V[:, :k] @ d
        r = r - defl_V @ (defl_H @ d)
        x = x + gmres_cycle(A, r, p, stats)
        r = b - A(x)
        stats["matvecs"] += 1
        stats["cycles"] += 1
        hist.append(np.linalg.norm(r) / bnorm)
    return x, dict(history=hist, converged=np.linalg.norm(r) <= tol * bnorm, **stats)


def rayleigh_ritz_hermitian(defl_V, defl_H, Q):
    """Ritz pairs of a hermitian operator in span(V_k) from A V_k = V_{k+1} Hbar_k.

    Returns (lam[Q], E[n, Q], resid[Q]) sorted by |lambda| (ties: lambda,
    then index)."""
    k = defl_H.shape[1]
    T = defl_H[:k, :k]
    T = 0.5 * (T + T.conj().T)
    lam, S = np.linalg.eigh(T)
    order = np.lexsort((np.arange(k), lam, np.abs(lam)))[:Q]
    lam, S = lam[order], S[:, order]
    E = defl_V[:, :k] @ S
    Sp = np.vstack([S, np.zeros((1, S.shape[1]))])
    resid = np.linalg.norm(defl_H @ S - Sp[:k + 1] * lam, axis=0)
    return lam, E, resid


def hermitian_eigpairs_dense(Mp, Q):
    """Q eigenpairs of a dense hermitian matrix with smallest |lambda|."""
    lam, E = np.linalg.eigh(0.5 * (Mp + Mp.conj().T))
    order = np.lexsort((np.arange(lam.size), lam, np.abs(lam)))[:Q]
    return lam[order], E[:, order]
