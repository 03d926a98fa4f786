"""The whole loop-estimation path on the GPU, as a sequence of C-ABI calls.

Sec. 7's procedure: Z(4) noise; even/odd solves (GMRES-DR on the first
noise vector, super-converged, GMRES-Proj on the rest); hermitian
eigenpairs of M' = M g5 from a second super-converged solve on the full
lattice (Sec. 5.4); PS and POLY subtraction vectors with exact trace
corrections (Sec. 5.1-5.2); HFES, HFPS and HFPOLY (Sec. 5.4-5.5); the
subtracted estimator for Theta = 1, g_1..g_4 (Sec. 5 Eq. (23), Sec. 6).

This module only sequences library calls; every computation runs in
liblqcd.so.  fused=True (the default) serves the six methods with the
library's combined calls: PS and POLY vectors from one chain of powers of
kappa P (poly_subtract_multi, written twice: as they are and as the bases
of HFPS and HFPOLY), the three hermitian-forced projections with one set of
overlaps (deflate_project_multi) and the six estimates in one call
(loop_estimate_multi).  fused=False makes one call per method (the PS and
POLY estimates are then taken before their vectors are extended in place
into HFPS and HFPOLY) and also returns 1/xi'.
"""
import numpy as np

from . import lqcd

METHODS = ("NS", "PS", "POLY", "HFES", "HFPS", "HFPOLY")


def run(ctx, noise_seed, n_noise, m, k, pert_order, poly_degree, Q, herm_m, herm_k,
        thetas=(0, 1, 2, 3, 4), tol=1e-10, tol_super=1e-13, inner="f64", inner_tol=1e-5,
        rhs_block=8, eig_tol=1e-10, max_cycles=2000, defl=None, hdefl=None, samples=False, fused=True):
    """Run the path; returns a dict of per-method (est, err[, samples]) and
    the intermediate objects."""
    import torch
    eta = ctx.noise_z4(noise_seed, 0, n_noise)
    x, defl, st = ctx.gmresdr_solve(eta, op="schur", m=m, k=k, tol=tol, tol_super=tol_super,
                                    inner=inner, inner_tol=inner_tol, rhs_block=rhs_block,
                                    max_cycles=max_cycles, defl=defl)
    if hdefl is None:
        _, hdefl, hst = ctx.gmresdr_solve(eta[0:1], op="MG5", m=herm_m, k=herm_k, tol=tol,
                                          tol_super=tol_super, eig_tol=eig_tol, n_eig=Q,
                                          max_cycles=max_cycles)
    lam, lam_res = hdefl.eigpairs(Q)
    out = {}
    ones = np.ones(pert_order + 1, dtype=np.complex128)
    if fused:
        # trace corrections and the Min-Res coefficients (no vectors)
        _, corr_ps = ctx.pert_subtract(pert_order, eta[0:0], thetas)
        _, corr_poly, cpoly, apoly = ctx.poly_subtract(poly_degree, eta[0:0], b=eta[0:1], thetas=thetas)
        xt_ps, xt_poly, base_ps, base_poly = ctx.poly_subtract_multi(eta, [ones, cpoly, ones, cpoly])
        hf = ctx.deflate_project_multi(hdefl, Q, eta, [(lqcd.DEFL_HFES, None, None, None),
                                                       (lqcd.DEFL_EIGPOLY, ones, base_ps, corr_ps),
                                                       (lqcd.DEFL_EIGPOLY, cpoly, base_poly, corr_poly)], thetas)
        xts = [None, xt_ps, xt_poly] + [h[0] for h in hf]
        corrs = [None, corr_ps, corr_poly] + [h[1] for h in hf]
        res = ctx.loop_estimate_multi(eta, x, xts, corrs, thetas, samples=samples)
        for name, r in zip(METHODS, res):
            out[name] = dict(est=r[0], err=r[1], samples=r[2] if samples else None)
        return dict(methods=out, x=x, eta=eta, defl=defl, hdefl=hdefl, solve_stats=st, lam=lam,
                    lam_resid=lam_res, poly_c=cpoly, poly_a=apoly, xi_pert=None, xi_poly=None)

    def est(name, xt, corr):
        r = ctx.loop_estimate(eta, x, xt, corr, thetas, samples=samples)
        out[name] = dict(est=r[0], err=r[1], samples=r[2] if samples else None)

    est("NS", None, None)
    xt_ps, corr_ps = ctx.pert_subtract(pert_order, eta, thetas)
    est("PS", xt_ps, corr_ps)
    xt_poly, corr_poly, cpoly, apoly = ctx.poly_subtract(poly_degree, eta, b=eta[0:1], thetas=thetas)
    est("POLY", xt_poly, corr_poly)
    xt_hf, corr_hf, _ = ctx.deflate_project(hdefl, Q, eta, xt=torch.zeros_like(eta), corr=None,
                                            mode=lqcd.DEFL_HFES, thetas=thetas)
    est("HFES", xt_hf, corr_hf)
    del xt_hf
    xt_ps, corr_hfps, xi_ps = ctx.deflate_project(hdefl, Q, eta, xt=xt_ps, corr=corr_ps,
                                                  mode=lqcd.DEFL_EIGPOLY, coeffs=ones, thetas=thetas)
    est("HFPS", xt_ps, corr_hfps)
    xt_poly, corr_hfpoly, xi_poly = ctx.deflate_project(hdefl, Q, eta, xt=xt_poly, corr=corr_poly,
                                                        mode=lqcd.DEFL_EIGPOLY, coeffs=cpoly,
                                                        thetas=thetas)
    est("HFPOLY", xt_poly, corr_hfpoly)
    return dict(methods=out, x=x, eta=eta, defl=defl, hdefl=hdefl, solve_stats=st, lam=lam,
                lam_resid=lam_res, poly_c=cpoly, poly_a=apoly, xi_pert=xi_ps, xi_poly=xi_poly)
