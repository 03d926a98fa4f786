"""The point-split vector operator (oracle; test infrastructure only).

Table 2 of the paper defines the point-split vector current in direction
mu by the two link-crossing bilinears
    kappa psibar(x + mu) (1 + g_mu) U_mu(x)^dagger psi(x)
  - kappa psibar(x) (1 - g_mu) U_mu(x) psi(x + mu),
whose expectation is -Tr(Theta(mu) M^{-1}) (Sec. 6) with the matrix
    (Theta(mu) psi)(x) = kappa [ (1 + g_mu) U_mu(x - mu)^dagger psi(x - mu)
                               - (1 - g_mu) U_mu(x) psi(x + mu) ],
i.e. kappa times the backward minus the forward hop of P (Eq. (25)) along
mu only.  The trace and its subtraction follow Secs. 5.1-5.2 with Theta
replaced by Theta(mu) (the paper's sums over e_{i+mu} Theta(mu) ... e_i);
the stochastic estimate is (1/N) sum_n eta_n^dagger Theta(mu) (x_n - xt_n).
Per timeslice, the term of row site x is attributed to the timeslice of x.

Pins (tests/test_oracle_pointsplit.py): the shift form against matrix
elements; with constant abelian links, the trace against a momentum-space
closed form (and zero for unit links);
Tr(Theta(mu) M^{-1}) purely imaginary (g5-hermiticity: Theta(mu)^dagger =
-g5 Theta(mu) g5); only odd orders of kappa P contribute to its
perturbative trace; the estimator with unit vectors equals the dense trace.
"""
import numpy as np

from .lattice import GAMMA, volume
from .subtract import per_timeslice

_I4 = np.eye(4, dtype=np.complex128)


def apply_theta_ps(U, kappa, mu, psi):
    """Theta(mu) psi for fields (..., Lt, Lz, Ly, Lx, 4, 3) (array shifts)."""
    nlead = psi.ndim - 6
    ax = nlead + 3 - mu
    Umu = U[..., mu, :, :]
    # backward: (1 + g) U_mu(x - mu)^dagger psi(x - mu)
    t = np.einsum("...ba,...sb->...sa", np.conj(Umu), psi)        # U^dagger psi at x
    bwd = np.einsum("st,...tb->...sb", _I4 + GAMMA[mu], np.roll(t, 1, axis=ax))
    # forward: (1 - g) U_mu(x) psi(x + mu)
    f = np.roll(psi, -1, axis=ax)
    fwd = np.einsum("st,...tb->...sb", _I4 - GAMMA[mu], np.einsum("...ab,...sb->...sa", Umu, f))
    return kappa * (bwd - fwd)


def dense_theta_ps(U, kappa, dims, mu):
    """Theta(mu) as a dense 12V x 12V matrix, filled element by element."""
    Lx, Ly, Lz, Lt = dims
    V = volume(dims)
    L = (Lx, Ly, Lz, Lt)
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    for s in range(V):
        c = [s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)]
        f = list(c)
        f[mu] = (c[mu] + 1) % L[mu]
        b = list(c)
        b[mu] = (c[mu] - 1) % L[mu]
        sf = f[0] + Lx * (f[1] + Ly * (f[2] + Lz * f[3]))
        sb = b[0] + Lx * (b[1] + Ly * (b[2] + Lz * b[3]))
        Uf = U[c[3], c[2], c[1], c[0], mu]
        Ub = U[b[3], b[2], b[1], b[0], mu]
        D[12 * s:12 * s + 12, 12 * sb:12 * sb + 12] += kappa * np.kron(_I4 + GAMMA[mu], Ub.conj().T)
        D[12 * s:12 * s + 12, 12 * sf:12 * sf + 12] -= kappa * np.kron(_I4 - GAMMA[mu], Uf)
    return D


def trace_ps_dense(U, kappa, dims, mu, A):
    """Tr_t(Theta(mu) A) per timeslice for a dense 12V x 12V matrix A."""
    V = volume(dims)
    T = dense_theta_ps(U, kappa, dims, mu) @ A
    diag = np.einsum("xixi->x", T.reshape(V, 12, V, 12))
    return per_timeslice(diag, dims)


def samples_ps(U, kappa, eta, x, xt, mus, dims):
    """t_n[mu][t] = sum_{x in t} eta_n(x)^dagger (Theta(mu) (x_n - xt_n))(x);
    shape (N, len(mus), Lt + 1), last column the total."""
    N = eta.shape[0]
    V = volume(dims)
    diff = x - xt
    out = []
    for mu in mus:
        y = apply_theta_ps(U, kappa, mu, diff).reshape(N, V, 12)
        site = np.einsum("nxi,nxi->nx", np.conj(eta.reshape(N, V, 12)), y)
        ts = per_timeslice(site, dims)
        out.append(np.concatenate([ts, ts.sum(axis=-1, keepdims=True)], axis=-1))
    return np.stack(out, axis=1)


def site_bilinear_ps(U, kappa, E, mus, dims, weights):
    """sum_q w_q sum_{x in t} e_q(x)^dagger (Theta(mu) g5 e_q)(x), (len(mus), Lt)."""
    from .wilson import g5
    V = volume(dims)
    res = []
    for mu in mus:
        y = apply_theta_ps(U, kappa, mu, g5(E)).reshape(E.shape[0], V, 12)
        v = np.einsum("qxi,qxi->qx", np.conj(E.reshape(E.shape[0], V, 12)), y)
        res.append(np.einsum("q,qx->x", weights, v))
    return per_timeslice(np.stack(res, axis=0), dims)


def phase_links(dims, phases):
    """Constant abelian links U_mu(x) = exp(i phases[mu]) times the identity."""
    Lx, Ly, Lz, Lt = dims
    U = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        U[..., mu, :, :] = np.exp(1j * phases[mu]) * np.eye(3)
    return U


def free_trace_ps(dims, kappa, mu, coeffs, phases=(0.0, 0.0, 0.0, 0.0)):
    """Tr(Theta(mu) p(kappa P)) for the constant links of phase_links, from
    plane waves, p(z) = sum_j coeffs[j] z^j.  A plane wave of momentum p sees
    the phases as a shift q = p + phases, so per momentum the operators act on
    spin as Theta(mu) -> kappa [(1 + g_mu) e^{-i q_mu} - (1 - g_mu) e^{+i q_mu}]
    and P -> sum_nu [(1 - g_nu) e^{+i q_nu} + (1 + g_nu) e^{-i q_nu}], times
    the 3 x 3 colour identity; the trace sums over the V momenta.  (With zero
    phases the trace vanishes: the free current has no expectation.)"""
    Lx, Ly, Lz, Lt = dims
    total = 0.0 + 0.0j
    for nx in range(Lx):
        for ny in range(Ly):
            for nz in range(Lz):
                for nt in range(Lt):
                    p = 2 * np.pi * np.array([nx / Lx, ny / Ly, nz / Lz, nt / Lt]) + np.asarray(phases)
                    Pp = sum((_I4 - GAMMA[nu]) * np.exp(1j * p[nu]) + (_I4 + GAMMA[nu]) * np.exp(-1j * p[nu])
                             for nu in range(4))
                    Th = kappa * ((_I4 + GAMMA[mu]) * np.exp(-1j * p[mu]) - (_I4 - GAMMA[mu]) * np.exp(1j * p[mu]))
                    poly = np.zeros((4, 4), dtype=np.complex128)
                    Kp = np.eye(4, dtype=np.complex128)
                    for cj in coeffs:
                        poly += cj * Kp
                        Kp = Kp @ (kappa * Pp)
                    total += 3 * np.trace(Th @ poly)
    return total
