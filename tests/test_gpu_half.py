"""GPU parity of the 16-bit (FP16 / BF16, per-site scaled) storage path.

Stencil: Mhat applied to a stored input equals the oracle's FP64 Mhat to
the storage's rounding.  A stored value is v / s rounded to p fraction bits
(p = 10 for FP16, 7 for BF16) with s the site's largest |re| or |im|, so
each component errs by at most 2^-(p+1) s; the even/odd operator
1 - kappa^2 D_eo D_oe amplifies a per-site error by at most 1 + 64 kappa^2
(|P| <= 8 per parity hop), hence the bound 2^-(p+1) (1 + 64 kappa^2) max|x|
per output component, asserted relative to max|x|.  A lower bound checks
that the 16-bit path really rounds (its error is far above the FP32
stencil's).

Solver: mixed-precision solves with a 16-bit inner basis reach the same
FP64 true residual and LU solution as the FP32 form.
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, context, to_gpu, to_host, say, rel_err
from oracle import wilson as W
from oracle.noise import z4_noise

pytestmark = pytest.mark.gpu

BITS = {"f16": 10, "bf16": 7}


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("dims", [(4, 4, 2, 4), (6, 4, 2, 8), (2, 2, 2, 4)])
def test_schur_stored_input(dims, prec):
    require_gpu()
    kappa = 0.13
    ctx, U = context(dims, 0.3, 7, kappa)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((3,) + ctx.shape) + 1j * rng.standard_normal((3,) + ctx.shape)
    # scale sites differently so the per-site scales matter
    x *= np.exp(rng.uniform(-6, 6, size=(3,) + ctx.shape[:4]))[..., None, None]
    say("schur stored", prec, dims)
    y = to_host(ctx.wilson_apply("schur", to_gpu(x), prec=prec))
    ref = W.apply_Mhat(U, kappa, x, dims)
    err = np.abs(y - ref)
    # per-site bound: each output site sees its own and its 2-hop
    # neighbours' inputs; use the global bound on every site scale
    # (sqrt 2: a complex component has two rounded parts)
    bound = 2.0 ** -(BITS[prec] + 1) * np.sqrt(2) * (1 + 64 * kappa ** 2) * np.abs(x).max()
    assert err.max() <= bound, (err.max(), bound)
    y32 = to_host(ctx.wilson_apply("schur", to_gpu(x), prec="f32"))
    assert err.max() > 100 * np.abs(y32 - ref).max()


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_schur_stored_input_relative_per_site(prec):
    """Sites of very different magnitude keep their relative accuracy: the
    scales are per site, not per vector."""
    require_gpu()
    dims, kappa = (4, 4, 2, 4), 0.0
    ctx, U = context(dims, 0.3, 7, kappa)   # kappa = 0: Mhat is the identity on even sites
    rng = np.random.default_rng(10)
    x = rng.standard_normal((1,) + ctx.shape) + 1j * rng.standard_normal((1,) + ctx.shape)
    x *= np.exp(rng.uniform(-20, 20, size=(1,) + ctx.shape[:4]))[..., None, None]
    say("schur stored per-site", prec)
    y = to_host(ctx.wilson_apply("schur", to_gpu(x), prec=prec))
    ref = W.apply_Mhat(U, kappa, x, dims)
    even = np.abs(ref).max(axis=(-1, -2), keepdims=True) > 0
    d = y - ref
    comp = np.maximum(np.abs(d.real), np.abs(d.imag))  # each real part is rounded on its own
    site_max = np.maximum(np.abs(x.real), np.abs(x.imag)).max(axis=(-1, -2), keepdims=True)
    rel = (comp / site_max)[np.broadcast_to(even, y.shape)]
    assert rel.max() <= 2.0 ** -(BITS[prec] + 1) * 1.01


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("dims,kappa", [((4, 4, 4, 4), 0.12), ((6, 4, 2, 8), 0.13)])
def test_mixed_solve_16bit_basis(dims, kappa, prec):
    require_gpu()
    ctx, U = context(dims, 0.3, 1001, kappa)
    eta = z4_noise(2001, dims, 0, 5)
    say("solve mixed", prec, dims)
    x, defl, st = ctx.gmresdr_solve(to_gpu(eta), op="schur", m=20, k=10, tol=1e-11, tol_super=1e-13,
                                    inner=prec, inner_tol=1e-3, rhs_block=4)
    x = to_host(x)
    M = W.dense_M(U, kappa, dims)
    xref = np.linalg.solve(M, eta.reshape(5, -1).T).T.reshape(eta.shape)
    for r in range(5):
        assert rel_err(x[r], xref[r]) < 1e-9
        assert st[r]["true_resid"] < 1e-11
    assert all(s["refinements"] >= 1 for s in st[1:])
    # the 16-bit path is only for the even/odd system
    with pytest.raises(Exception):
        ctx.gmresdr_solve(to_gpu(eta[:1]), op="MG5", m=20, k=10, inner=prec)


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_mixed_solve_second_pass_on_every_step(prec):
    """The second Gram-Schmidt pass of the single-step 16-bit Arnoldi works
    on the stored vector in place; forced on every GMRES-Proj step it must
    leave the solutions as accurate as the conditional pass does (the
    two-step form's block second pass: test_two_step_arnoldi)."""
    require_gpu()
    dims, kappa = (6, 4, 2, 8), 0.13
    ctx, U = context(dims, 0.3, 1001, kappa)
    eta = z4_noise(2002, dims, 0, 4)
    M = W.dense_M(U, kappa, dims)
    xref = np.linalg.solve(M, eta.reshape(4, -1).T).T.reshape(eta.shape)
    out = {}
    for forced in (0, 1):
        ctx.tune(cycle_reorth=forced, arnoldi_steps=1)
        say("solve mixed second pass", prec, forced)
        x, defl, st = ctx.gmresdr_solve(to_gpu(eta), op="schur", m=20, k=10, tol=1e-11, tol_super=1e-13,
                                        inner=prec, inner_tol=1e-3, rhs_block=3)
        x = to_host(x)
        for r in range(4):
            assert rel_err(x[r], xref[r]) < 1e-9, (forced, r)
            assert st[r]["true_resid"] < 1e-11, (forced, r)
        out[forced] = st
    ctx.tune(cycle_reorth=0, arnoldi_steps=4)
    # forced: every Arnoldi step of the GMRES-Proj solves ran the second pass
    for r in range(1, 4):
        assert out[1][r]["reorth"] > out[0][r]["reorth"]
        assert out[1][r]["reorth"] >= out[1][r]["matvecs"] // 2


@pytest.mark.parametrize("z16", [0, 1])
@pytest.mark.parametrize("m", [19, 20, 21])
@pytest.mark.parametrize("forced", [0, 1])
@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_sstep_arnoldi(prec, forced, m, z16):
    """s Arnoldi steps per pass over the 16-bit basis (s = 2 .. 6: the
    shifted powers (Mhat - 1)^k v_j, k = 1..s, projected together, then
    orthonormalised among themselves) span the same Krylov space: the
    solutions reach LU and the true residual as the single-step form does,
    in about as many matrix-vector products; with the second pass forced on
    every block, and with cycle lengths p = m - 10 = 9, 10, 11, so that the
    last block of a cycle is shorter than s (1 to 5 steps); with the powers
    kept in FP32 and stored in the basis's 16-bit form (z16)."""
    require_gpu()
    dims, kappa = (6, 4, 2, 8), 0.13
    ctx, U = context(dims, 0.3, 1001, kappa)
    eta = z4_noise(2003, dims, 0, 4)
    M = W.dense_M(U, kappa, dims)
    xref = np.linalg.solve(M, eta.reshape(4, -1).T).T.reshape(eta.shape)
    st = {}
    try:
        for steps in (1, 2, 3, 4, 5, 6):
            ctx.tune(arnoldi_steps=steps, cycle_reorth=forced, sstep_z16=z16)
            say("solve s-step", prec, forced, m, steps, z16)
            x, defl, s = ctx.gmresdr_solve(to_gpu(eta), op="schur", m=m, k=10, tol=1e-11, tol_super=1e-13,
                                           inner=prec, inner_tol=1e-3, rhs_block=3)
            x = to_host(x)
            for r in range(4):
                assert rel_err(x[r], xref[r]) < 1e-9, (steps, r)
                assert s[r]["true_resid"] < 1e-11, (steps, r)
            st[steps] = s
    finally:
        ctx.tune(arnoldi_steps=4, cycle_reorth=0, sstep_z16=0)
    for steps in (2, 3, 4, 5, 6):
        for r in range(1, 4):
            assert st[steps][r]["matvecs"] <= st[1][r]["matvecs"] + (m - 10 + 1), (steps, r, st[1][r], st[steps][r])
            if forced:
                assert st[steps][r]["reorth"] > 0


@pytest.mark.parametrize("z16", [0, 1])
@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_sstep_direct_and_explicit_paths_in_one_block(prec, z16):
    """The s-step block takes, per right-hand side, either the direct path
    (Gram matrix from the dot pass, basis vectors stored by the update pass)
    or the explicit one (update in place, second pass).  A right-hand side
    whose even/odd source is an eigenvector of Mhat of the largest modulus
    (the deflation space holds the smallest) makes its block nearly
    degenerate (z_1 = (lambda - 1) v is all but removed by the projection),
    so the DGKS test sends it down the explicit path, while the noise vectors
    beside it in the same block take the direct one.  Every solution still
    reaches LU and the true residual."""
    require_gpu()
    dims, kappa = (4, 2, 2, 4), 0.13
    ctx, U = context(dims, 0.3, 1001, kappa)
    M = W.dense_M(U, kappa, dims)
    par = np.broadcast_to(W.parity_mask(dims) == 0, ctx.shape).reshape(-1)
    E, O = np.flatnonzero(par), np.flatnonzero(~par)
    Mhat = M[np.ix_(E, E)] - M[np.ix_(E, O)] @ M[np.ix_(O, E)]
    lam, vec = np.linalg.eig(Mhat)
    v = vec[:, np.argmax(np.abs(lam))]
    eta = z4_noise(2003, dims, 0, 4).astype(np.complex128)
    e2 = np.zeros(M.shape[0], complex)
    e2[E] = v  # odd part zero: the even/odd source is v itself
    eta[2] = e2.reshape(ctx.shape)
    xref = np.linalg.solve(M, eta.reshape(4, -1).T).T.reshape(eta.shape)
    ctx.tune(arnoldi_steps=4, cycle_reorth=0, sstep_z16=z16)
    say("solve mixed paths", prec, z16)
    try:
        x, defl, s = ctx.gmresdr_solve(to_gpu(eta), op="schur", m=20, k=10, tol=1e-11, tol_super=1e-13,
                                       inner=prec, inner_tol=1e-3, rhs_block=3)
    finally:
        ctx.tune(sstep_z16=0)
    x = to_host(x)
    for r in range(4):
        assert rel_err(x[r], xref[r]) < 1e-9, r
        assert s[r]["true_resid"] < 1e-11, r
    assert s[2]["reorth"] > 0, s[2]
    assert s[1]["reorth"] == 0 and s[3]["reorth"] == 0, (s[1], s[3])
