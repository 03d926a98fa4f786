"""The whole loop-estimation path in FP64 (oracle; test infrastructure only).

Follows Sec. 7's procedure: noise eta^(0..N-1) (Sec. 2); even/odd reduced
solves, GMRES-DR on eta^(0) and GMRES-Proj on the rest; odd-site
reconstruction; hermitian eigenpairs of M' = M g5 from a second, full-lattice
GMRES-DR solve on eta^(0) (Sec. 5.4: the hermitian system is solved
unreduced); PS and POLY subtraction vectors and trace corrections; the
HFES, HFPS and HFPOLY combinations (Sec. 5.5); the subtracted estimator for
Theta in {1, g_1, .., g_4} (Sec. 5, Eq. (23); Sec. 6).

Method codes: 0 NS, 1 PS, 2 POLY, 3 HFES, 4 HFPS, 5 HFPOLY.
"""
import numpy as np

from . import lattice as L
from . import wilson as W
from . import krylov as K
from . import subtract as S
from . import estimate as E
from .noise import z4_noise

METHODS = ("NS", "PS", "POLY", "HFES", "HFPS", "HFPOLY")


def solve_all(U, dims, kappa, eta, m, k, tol, tol_super, max_cycles=400):
    """x^(n) = M^{-1} eta^(n) via the even/odd system; returns (x, info)."""
    shape = eta.shape[1:]
    par = W.parity_mask(dims)

    def Ahat(v):
        return W.apply_Mhat(U, kappa, v.reshape(shape), dims).ravel()

    xs = np.zeros_like(eta)
    src0 = W.eo_source(U, kappa, eta[0], dims).ravel()
    xe, info0 = K.gmres_dr(Ahat, src0, m, k, tol_super, max_cycles=max_cycles)
    xs[0] = W.eo_reconstruct(U, kappa, xe.reshape(shape), eta[0], dims)
    infos = [info0]
    for n in range(1, eta.shape[0]):
        src = W.eo_source(U, kappa, eta[n], dims).ravel()
        xe, inf = K.gmres_proj(Ahat, src, info0["V"], info0["H"], m - k, tol, max_cycles=max_cycles)
        xs[n] = W.eo_reconstruct(U, kappa, xe.reshape(shape), eta[n], dims)
        infos.append(inf)
    return xs, infos


def hermitian_modes(U, dims, kappa, b, m, k, Q, tol_super, eig_tol=1e-10, max_cycles=400):
    """Q eigenpairs of M' from a super-converged full-lattice GMRES-DR solve
    (continued until the Q lowest harmonic Ritz pairs have relative
    residual <= eig_tol) and Rayleigh-Ritz in its deflation space."""
    shape = b.shape

    def Ap(v):
        return W.apply_Mprime(U, kappa, v.reshape(shape)).ravel()

    _, info = K.gmres_dr(Ap, b.ravel(), m, k, tol_super, max_cycles=max_cycles,
                         eig_tol=eig_tol, n_eig=Q)
    lam, Ev, resid = K.rayleigh_ritz_hermitian(info["V"], info["H"], Q)
    return lam, Ev.T.reshape((Q,) + shape), resid, info


def trace_poly(U, dims, kappa, coeffs, thetas):
    """Exact Tr_t(Theta p(kappa P)): dense powers up to 4^4, probes beyond."""
    V = L.volume(dims)
    if V <= 256:
        A = S.poly_dense(W.dense_P(U, dims), kappa, coeffs)
        return S.trace_correction_dense(A, dims, thetas)
    return S.trace_correction_probe(U, kappa, coeffs, dims, thetas)


def run(U, dims, kappa, noise_seed, n_noise, m, k, pert_order, poly_degree, Q,
        thetas=(0, 1, 2, 3, 4), tol=1e-12, tol_super=1e-13, herm_m=None, herm_k=None,
        modes=None):
    """Returns a dict with per-method estimates, errors, samples and the
    intermediate objects (x, subtraction vectors, coefficients, modes)."""
    eta = z4_noise(noise_seed, dims, 0, n_noise)
    x, infos = solve_all(U, dims, kappa, eta, m, k, tol, tol_super)
    if modes is None:
        lam, Ev, resid, hinfo = hermitian_modes(U, dims, kappa, eta[0], herm_m or m, herm_k or k,
                                                Q, tol_super)
    else:
        lam, Ev = modes
        resid = None
    cp = S.pert_coeffs(pert_order)
    cpoly, apoly = S.poly_coeffs(U, kappa, eta[0], poly_degree)
    xt_pert = S.horner(U, kappa, eta, cp)
    xt_poly = S.horner(U, kappa, eta, cpoly)
    corr_pert = trace_poly(U, dims, kappa, cp, thetas)
    corr_poly = trace_poly(U, dims, kappa, cpoly, thetas)
    inv_lam = (1.0 / lam).astype(np.complex128)
    xt_eig = S.eig_vector(Ev, inv_lam, eta)
    corr_eig = S.site_bilinear(Ev, thetas, dims, inv_lam)
    xi_pert = S.xi_inverse(U, kappa, Ev, cp)
    xi_poly = S.xi_inverse(U, kappa, Ev, cpoly)
    xt = {
        "NS": np.zeros_like(eta),
        "PS": xt_pert,
        "POLY": xt_poly,
        "HFES": xt_eig,
        "HFPS": xt_eig + xt_pert - S.eig_vector(Ev, xi_pert, eta),
        "HFPOLY": xt_eig + xt_poly - S.eig_vector(Ev, xi_poly, eta),
    }
    Lt = dims[3]
    zero = np.zeros((len(thetas), Lt), dtype=np.complex128)
    corr = {
        "NS": zero,
        "PS": corr_pert,
        "POLY": corr_poly,
        "HFES": corr_eig,
        "HFPS": corr_eig + corr_pert - S.site_bilinear(Ev, thetas, dims, xi_pert),
        "HFPOLY": corr_eig + corr_poly - S.site_bilinear(Ev, thetas, dims, xi_poly),
    }
    out = {}
    for meth in METHODS:
        t = E.samples(eta, x, xt[meth], thetas, dims)
        est, err = E.estimate(t, corr[meth])
        out[meth] = dict(samples=t, est=est, err=err, corr=corr[meth])
    return dict(methods=out, x=x, eta=eta, xt=xt, lam=lam, modes=Ev, mode_resid=resid,
                poly_c=cpoly, poly_a=apoly, xi_pert=xi_pert, xi_poly=xi_poly, solve_info=infos)
