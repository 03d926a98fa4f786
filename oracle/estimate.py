"""The subtracted trace estimator (oracle; test infrastructure only).

Sec. 5, Eq. (23) (and its per-method forms, Eqs. (30), (49), (66), (70)):

  Tr(Theta M^{-1}) ~ (1/N) sum_n eta^(n)dagger Theta (x^(n) - xt^(n))
                     + Tr(Theta tilde-M^{-1}),

with x^(n) = M^{-1} eta^(n) and xt^(n) = tilde-M^{-1} eta^(n).  Sec. 6,
Eq. (73): <psibar Theta psi> = -Tr(Theta M^{-1}); Table 2: the scalar
(Theta = 1) carries its signal in the real part, the local vector
(Theta = g_mu) in the imaginary part.  The per-timeslice split sums the
site terms over the spatial volume of each timeslice; the last entry of
every estimate row is the whole-lattice total.

Standard error: s / sqrt(N) with the unbiased sample variance, separately
for the real and imaginary parts.  Relative efficiency, Eq. (74):
RE = (1 / dy^2 - 1) * 100 with dy the ratio of error bars.
"""
import numpy as np

from .lattice import volume
from .wilson import apply_theta
from .subtract import per_timeslice


def samples(eta, x, xt, thetas, dims):
    """t_n[theta][t] = sum_{x in t} eta_n(x)^dagger Theta (x_n - xt_n)(x).

    eta, x, xt: (N, Lt, Lz, Ly, Lx, 4, 3).  Returns complex (N, ntheta, Lt+1),
    last column the total."""
    N = eta.shape[0]
    V = volume(dims)
    diff = x - xt
    out = []
    for th in thetas:
        y = apply_theta(th, diff).reshape(N, V, 12)
        site = np.einsum("nxi,nxi->nx", np.conj(eta.reshape(N, V, 12)), y)
        ts = per_timeslice(site, dims)
        out.append(np.concatenate([ts, ts.sum(axis=-1, keepdims=True)], axis=-1))
    return np.stack(out, axis=1)


def estimate(t_samples, correction):
    """Mean + correction and standard errors.

    t_samples: (N, ntheta, Lt+1) complex; correction: (ntheta, Lt) complex
    per-timeslice trace correction.  Returns (est (ntheta, Lt+1) complex,
    stderr (ntheta, Lt+1, 2) [Re, Im])."""
    N = t_samples.shape[0]
    corr = np.concatenate([correction, correction.sum(axis=-1, keepdims=True)], axis=-1)
    est = t_samples.mean(axis=0) + corr
    if N > 1:
        se_re = t_samples.real.std(axis=0, ddof=1) / np.sqrt(N)
        se_im = t_samples.imag.std(axis=0, ddof=1) / np.sqrt(N)
    else:
        se_re = np.zeros(est.shape)
        se_im = np.zeros(est.shape)
    return est, np.stack([se_re, se_im], axis=-1)


def relative_efficiency(err_method, err_ref):
    """RE = (1 / dy^2 - 1) * 100 with dy = err_method / err_ref (Eq. (74))."""
    dy = np.asarray(err_method) / np.asarray(err_ref)
    return (1.0 / dy ** 2 - 1.0) * 100.0
