"""Differentiable trace estimate (torch.autograd.Function over the C ABI).

``trace_estimate(lat, kappa, omega, seed, nnoise, thetas)`` returns the
unsubtracted stochastic estimate of Tr_t(Theta M^{-1}) (Sec. 5 Eq. (23)),
per operator and timeslice, as a real tensor [ntheta, Lt, 2] (real and
imaginary parts).  It is differentiable in

* ``kappa``: a 0-d float64 tensor, the hopping parameter of M = 1 - kappa P;
* ``omega``: a float64 tensor [Lt, Lz, Ly, Lx, 4, 8] of su(3) coordinates of
  a left rotation of every link, U_mu(x) -> exp(i omega^a T^a) U_mu(x)
  (T^a = lambda^a / 2), taken at omega = 0: its gradient is the force on
  the links of the context (omega must be zero).

Forward solves M x = eta with the library's deflated GMRES and estimates.
Only the noise seed is saved; backward regenerates the noise and solves
the forward and adjoint systems again in one batched call (loop_gradient),
with the weighting that the incoming gradient defines.  The gradient is the
exact derivative of the fixed-noise estimate, so it is itself an unbiased
estimate of the derivative of the trace.
"""
import numpy as np
import torch


class TraceEstimate(torch.autograd.Function):
    @staticmethod
    def forward(fctx, kappa, omega, lat, seed, first, nnoise, thetas, solve_kw):
        if float(omega.detach().abs().max()) != 0.0:
            raise ValueError("omega are coordinates of the tangent space at the context's links: "
                             "only omega = 0 is evaluated")
        lat.set_kappa(float(kappa.detach()))
        eta = lat.noise_z4(seed, first, nnoise)
        x, defl, _ = lat.gmresdr_solve(eta, op="schur", **solve_kw)
        defl.free()
        est, _ = lat.loop_estimate(eta, x, thetas=thetas)
        Lt = lat.dims[3]
        e = est[:, :Lt]
        out = np.stack([e.real, e.imag], axis=-1)
        fctx.lat, fctx.seed, fctx.first, fctx.nnoise = lat, seed, first, nnoise
        fctx.thetas, fctx.solve_kw = tuple(thetas), dict(solve_kw)
        fctx.kappa = float(kappa.detach())
        fctx.kdev, fctx.odev = kappa.device, omega.device
        return torch.from_numpy(out).to(kappa.device)

    @staticmethod
    def backward(fctx, grad):
        lat = fctx.lat
        g = grad.detach().to("cpu", torch.float64).numpy()
        # L = sum g0 Re T + g1 Im T = Re sum (g0 - i g1) T
        w = g[..., 0] - 1j * g[..., 1]
        lat.set_kappa(fctx.kappa)
        eta = lat.noise_z4(fctx.seed, fctx.first, fctx.nnoise)
        need_links = fctx.needs_input_grad[1]
        dk, dl, defl, _ = lat.loop_gradient(eta, None, thetas=fctx.thetas, weights=w, links=need_links,
                                            **fctx.solve_kw)
        if defl is not None:
            defl.free()
        gk = torch.tensor(dk.real, dtype=torch.float64, device=fctx.kdev)
        go = dl.real.contiguous().to(fctx.odev) if need_links else None
        return gk, go, None, None, None, None, None, None


def trace_estimate(lat, kappa, omega, seed, nnoise, thetas=(0,), first=0, **solve_kw):
    """Differentiable unsubtracted estimate, [ntheta, Lt, 2] (see module doc).
    solve_kw are gmresdr_solve's keyword arguments (m, k, tol, ...)."""
    return TraceEstimate.apply(kappa, omega, lat, seed, first, nnoise, tuple(thetas), solve_kw)
