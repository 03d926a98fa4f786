"""GPU parity of loop_gradient and the autograd wrapper (differentiation of
the trace estimate) against the oracle.

* GPU derivatives against the oracle's per-noise estimator with LU solves
  and the same Z(4) noise (weighted operators, several timeslice weights);
* unit vectors as noise make the estimate exact: GPU derivatives against
  the dense Tr(Theta M^-1 P M^-1) and kappa Tr(Theta M^-1 dP/dw M^-1);
* finite differences of the GPU estimate itself (fixed noise) in kappa and
  in one link rotation, Richardson-extrapolated;
* torch.autograd through TraceEstimate against the oracle's weighted
  derivatives.
Solves run at 1e-12 (the derivatives inherit the solver's relative error).
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, context, to_gpu, to_host, say, rel_err
from oracle import wilson as W
from oracle import gradient as G
from oracle.noise import z4_noise

pytestmark = pytest.mark.gpu

SOLVE = dict(m=20, k=10, tol=1e-12, tol_super=1e-13, rhs_block=2)


def _oracle_grad(U, kappa, dims, eta, thetas, weights):
    M = W.dense_M(U, kappa, dims)
    lu = np.linalg.inv(M)
    solve = lambda b: (lu @ b.reshape(b.shape[0], -1).T).T.reshape(b.shape)
    x = solve(eta)
    y = G.adjoint_vectors_weighted(U, kappa, dims, thetas, weights, eta, solve)
    return G.grad_estimate(U, kappa, dims, eta, x, y)


@pytest.mark.parametrize("dims,kappa,nrhs,thetas", [((4, 4, 4, 4), 0.12, 4, (0, 4)),
                                                     ((6, 4, 2, 8), 0.13, 3, (1, 2, 3))])
def test_gradient_vs_oracle(dims, kappa, nrhs, thetas):
    require_gpu()
    ctx, U = context(dims, 0.3, 1001, kappa)
    rng = np.random.default_rng(17)
    w = rng.normal(size=(len(thetas), dims[3])) + 1j * rng.normal(size=(len(thetas), dims[3]))
    eta = z4_noise(2001, dims, 0, nrhs)
    say("loop_gradient vs oracle", dims, kappa, nrhs, thetas)
    dk, dl, defl, st = ctx.loop_gradient(to_gpu(eta), None, thetas=thetas, weights=w, **SOLVE)
    for s in st:
        assert s["true_resid"] < 1e-11, s
    dk_ref, dw_ref = _oracle_grad(U, kappa, dims, eta, thetas, w)
    assert abs(dk - dk_ref) < 1e-9 * abs(dk_ref)
    assert rel_err(to_host(dl), dw_ref) < 1e-9
    # given solutions (x from the solver) give the same derivatives
    say("loop_gradient with x given", dims)
    x, _, _ = ctx.gmresdr_solve(to_gpu(eta), op="schur", defl=defl, **SOLVE)
    dk2, dl2, _, _ = ctx.loop_gradient(to_gpu(eta), x, thetas=thetas, weights=w, defl=defl, **SOLVE)
    assert abs(dk2 - dk_ref) < 1e-9 * abs(dk_ref)
    assert rel_err(to_host(dl2), dw_ref) < 1e-9
    # kappa only
    dk3, dl3, _, _ = ctx.loop_gradient(to_gpu(eta), x, thetas=thetas, weights=w, defl=defl, links=False,
                                       **SOLVE)
    assert dl3 is None and abs(dk3 - dk_ref) < 1e-9 * abs(dk_ref)


def test_gradient_unit_vectors_exact():
    """With every unit vector as a noise vector the estimate is the trace:
    the GPU derivatives times N equal the dense derivatives."""
    require_gpu()
    dims, kappa = (2, 2, 2, 4), 0.09
    ctx, U = context(dims, 0.3, 71, kappa)
    n = 12 * 32
    eta = np.eye(n, dtype=np.complex128).reshape((n, dims[3], dims[2], dims[1], dims[0], 4, 3))
    thetas = (0, 3)
    w = np.array([[1, 2, 0.5, -1], [0.5j, 0, 1, 1 - 1j]], dtype=np.complex128)
    say("loop_gradient unit vectors", dims, n)
    dk, dl, _, _ = ctx.loop_gradient(to_gpu(eta), None, thetas=thetas, weights=w,
                                     **dict(SOLVE, rhs_block=8))
    dl = to_host(dl)
    Tw = G.theta_weighted_dense(thetas, w, dims)
    ref = G.dkappa_dense(U, kappa, dims, Tw)
    assert abs(dk * n - ref) < 1e-9 * abs(ref)
    for site, mu, a in ((0, 0, 0), (3, 1, 4), (13, 3, 7), (30, 2, 2)):
        c = [site % 2, (site // 2) % 2, (site // 4) % 2, site // 8]
        r = G.dlink_dense(U, kappa, dims, Tw, site, mu, a)
        assert abs(dl[c[3], c[2], c[1], c[0], mu, a] * n - r) < 1e-9 * max(abs(r), 1e-3)


def _estimate(ctx, eta_g, thetas, w):
    x, defl, _ = ctx.gmresdr_solve(eta_g, op="schur", **dict(SOLVE, tol=1e-13))
    defl.free()
    est, _ = ctx.loop_estimate(eta_g, x, thetas=thetas)
    return np.sum(w * est[:, :-1])


def test_gradient_vs_finite_differences():
    require_gpu()
    from paper_1903_06986_amd import Context
    dims, kappa = (4, 4, 4, 4), 0.11
    ctx, U = context(dims, 0.3, 1001, kappa)
    thetas = (0, 4)
    w = np.ones((2, dims[3]), dtype=np.complex128)
    eta_g = to_gpu(z4_noise(2001, dims, 0, 2))
    say("loop_gradient fd kappa", dims)
    dk, dl, _, _ = ctx.loop_gradient(eta_g, None, thetas=thetas, weights=w, **dict(SOLVE, tol=1e-13))
    dl = to_host(dl)

    def f_kappa(h):
        ctx.set_kappa(kappa + h)
        return _estimate(ctx, eta_g, thetas, w)

    h = 4e-4
    d1 = (f_kappa(h) - f_kappa(-h)) / (2 * h)
    d2 = (f_kappa(h / 2) - f_kappa(-h / 2)) / h
    ctx.set_kappa(kappa)
    assert abs((4 * d2 - d1) / 3 - dk) < 1e-6 * abs(dk)
    for site, mu, a in ((5, 2, 3), (200, 0, 7)):
        say("loop_gradient fd link", site, mu, a)
        c = [site % 4, (site // 4) % 4, (site // 16) % 4, site // 64]

        def f_link(h):
            c2 = Context(dims, G.rotate_link(U, site, mu, a, h, dims), kappa)
            return _estimate(c2, eta_g, thetas, w)

        h = 1e-3
        d1 = (f_link(h) - f_link(-h)) / (2 * h)
        d2 = (f_link(h / 2) - f_link(-h / 2)) / h
        an = dl[c[3], c[2], c[1], c[0], mu, a]
        assert abs((4 * d2 - d1) / 3 - an) < 1e-6 * max(abs(an), 1e-3)


def test_autograd_trace_estimate():
    require_gpu()
    import torch
    from paper_1903_06986_amd.autograd import trace_estimate
    dims, kappa = (4, 4, 2, 4), 0.12
    ctx, U = context(dims, 0.3, 11, kappa)
    thetas = (0, 1, 4)
    nn, seed = 3, 7
    k_t = torch.tensor(kappa, dtype=torch.float64, requires_grad=True)
    om = torch.zeros((dims[3], dims[2], dims[1], dims[0], 4, 8), dtype=torch.float64, device="cuda",
                     requires_grad=True)
    say("autograd forward", dims)
    out = trace_estimate(ctx, k_t, om, seed, nn, thetas, **SOLVE)
    eta = z4_noise(seed, dims, 0, nn)
    M = W.dense_M(U, kappa, dims)
    x = np.linalg.solve(M, eta.reshape(nn, -1).T).T.reshape(eta.shape)
    # forward: the unsubtracted per-timeslice estimate
    for a, th in enumerate(thetas):
        tx = W.apply_theta(th, x)
        ref = np.einsum("ntzyxsc,ntzyxsc->nt", np.conj(eta), tx).mean(axis=0)
        got = out[a].detach().cpu().numpy()
        assert np.abs(got[:, 0] + 1j * got[:, 1] - ref).max() < 1e-9 * np.abs(ref).max()
    rng = np.random.default_rng(3)
    gw = torch.from_numpy(rng.normal(size=tuple(out.shape)))
    loss = (out * gw).sum()
    say("autograd backward", dims)
    loss.backward()
    g = gw.numpy()
    dk_ref, dw_ref = _oracle_grad(U, kappa, dims, eta, thetas, g[..., 0] - 1j * g[..., 1])
    assert abs(k_t.grad.item() - dk_ref.real) < 1e-9 * abs(dk_ref)
    assert rel_err(om.grad.cpu().numpy(), dw_ref.real) < 1e-9
