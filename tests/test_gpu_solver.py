"""GPU parity of gmresdr_solve (GMRES-DR + GMRES-Proj, Sec. 7) against the oracle.

Solutions are compared with dense LU (|x - x_LU| / |x_LU| <= 1e-10 in
FP64), converged harmonic Ritz values with the dense spectrum of the
even/odd operator, hermitian Rayleigh-Ritz pairs with dense eigh (through
the projector sum_q e e^+ / lambda, since phases and degenerate rotations
are free).  Iteration counts are not compared.  The full-size case checks
the true residual recomputed by the oracle.
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, context, to_gpu, to_host, say, rel_err
from oracle import lattice as L
from oracle import wilson as W
from oracle import krylov as K
from oracle.noise import z4_noise

pytestmark = pytest.mark.gpu


def _dense_solve(U, kappa, dims, eta):
    M = W.dense_M(U, kappa, dims)
    n = eta.shape[0]
    return np.linalg.solve(M, eta.reshape(n, -1).T).T.reshape(eta.shape), M


@pytest.mark.parametrize("dims,kappa,nrhs,block", [((4, 4, 4, 4), 0.12, 4, 2),
                                                    ((6, 4, 2, 8), 0.13, 5, 3),
                                                    ((4, 4, 4, 4), 0.12, 13, 13)])
def test_schur_solve_fp64(dims, kappa, nrhs, block):
    """Blocks of 13 right-hand sides take the matrix-core projection in tiles
    of 8 + 5 columns."""
    require_gpu()
    ctx, U = context(dims, 0.3, 1001, kappa)
    eta = z4_noise(2001, dims, 0, nrhs)
    say("solve schur f64", dims, kappa, nrhs, block)
    x, defl, st = ctx.gmresdr_solve(to_gpu(eta), op="schur", m=20, k=10, tol=1e-12,
                                    tol_super=1e-13, rhs_block=block)
    x = to_host(x)
    xref, _ = _dense_solve(U, kappa, dims, eta)
    for r in range(nrhs):
        assert rel_err(x[r], xref[r]) < 1e-10, r
        assert st[r]["true_resid"] < 1e-11, st[r]
    # a second call reuses the deflation space (GMRES-Proj for every rhs)
    say("solve schur f64 reuse", dims)
    x2, _, st2 = ctx.gmresdr_solve(to_gpu(eta[1:2]), op="schur", m=20, k=10, tol=1e-12, defl=defl)
    assert rel_err(to_host(x2)[0], xref[1]) < 1e-10


@pytest.mark.parametrize("m", [90, 100])
def test_schur_solve_large_basis(m):
    """Restarts of bases of m + 1 = 91 vectors (recombination by the
    persistent kernel with 64-element tiles and the coefficients in LDS) and
    of 101 vectors (the general LDS-staged form): same solution as dense LU.
    On this lattice and kappa the oracle's GMRES-DR(m, 40) takes 3 cycles."""
    require_gpu()
    dims, kappa = (4, 4, 4, 4), 0.19
    ctx, U = context(dims, 0.3, 1001, kappa)
    eta = z4_noise(2001, dims, 0, 1)
    say("solve schur f64 large basis", dims, kappa, "m", m)
    x, _, st = ctx.gmresdr_solve(to_gpu(eta), op="schur", m=m, k=40, tol=1e-12, tol_super=1e-13,
                                 max_cycles=200)
    assert st[0]["cycles"] >= 2, st[0]  # at least one restart
    xref, _ = _dense_solve(U, kappa, dims, eta)
    assert rel_err(to_host(x)[0], xref[0]) < 1e-10
    assert st[0]["true_resid"] < 1e-11, st[0]


def test_harmonic_ritz_values_gpu():
    """Super-converged GMRES-DR: converged harmonic Ritz values are
    eigenvalues of Mhat (dense), like the oracle's."""
    require_gpu()
    dims, kappa = (4, 4, 2, 4), 0.13
    ctx, U = context(dims, 0.3, 31, kappa)
    eta = z4_noise(5, dims, 0, 1)
    say("ritz", dims)
    _, defl, st = ctx.gmresdr_solve(to_gpu(eta), op="schur", m=14, k=7, tol=1e-13, tol_super=1e-13,
                                    eig_tol=1e-11, n_eig=3, max_cycles=400)
    theta = defl.ritz()
    ev, od = L.eo_tables(dims)
    M = W.dense_M(U, kappa, dims)
    ie = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in ev])
    io = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in od])
    Mhat = np.eye(ie.size) - M[np.ix_(ie, io)] @ M[np.ix_(io, ie)]
    lam = np.linalg.eigvals(Mhat)
    # oracle run on the same problem
    shape = eta[0].shape
    A = lambda v: W.apply_Mhat(U, kappa, v.reshape(shape), dims).ravel()
    src = W.eo_source(U, kappa, eta[0], dims).ravel()
    _, oinfo = K.gmres_dr(A, src, 14, 7, 1e-13, max_cycles=400, eig_tol=1e-11, n_eig=3)
    for t in theta[:3]:
        assert np.min(np.abs(lam - t)) < 1e-9
        assert np.min(np.abs(oinfo["theta"] - t)) < 1e-9


def test_hermitian_solve_and_eigpairs():
    require_gpu()
    dims, kappa = (4, 4, 2, 4), 0.125
    ctx, U = context(dims, 0.3, 31, kappa)
    eta = z4_noise(5, dims, 0, 2)
    say("solve MG5", dims)
    x, defl, st = ctx.gmresdr_solve(to_gpu(eta), op="MG5", m=40, k=20, tol=1e-12, tol_super=1e-13,
                                    eig_tol=1e-11, n_eig=8, max_cycles=300)
    M = W.dense_M(U, kappa, dims)
    Mp = M @ W.dense_gamma(L.GAMMA5, L.volume(dims))
    xref = np.linalg.solve(Mp, eta.reshape(2, -1).T).T
    x = to_host(x).reshape(2, -1)
    for r in range(2):
        assert rel_err(x[r], xref[r]) < 1e-10
    Q = 6
    lam, res = defl.eigpairs(Q)
    lam_d, E_d = K.hermitian_eigpairs_dense(Mp, Q)
    assert (res < 1e-9).all()
    assert np.abs(lam - lam_d).max() < 1e-9


def _near_critical_kappa(U, dims):
    """kappa in [0.13, 0.26] where M' = M g5 of this small lattice has its
    smallest |eigenvalue| on a coarse grid (an eigenvalue crossing zero)."""
    best = None
    for kappa in np.linspace(0.13, 0.26, 27):
        M = W.dense_M(U, kappa, dims)
        lam = np.linalg.eigvalsh(M @ W.dense_gamma(L.GAMMA5, L.volume(dims)))
        v = np.abs(lam).min()
        if best is None or v < best[1]:
            best = (kappa, v)
    return best


@pytest.mark.parametrize("near_critical", [False, True])
def test_minres_dr_hermitian(near_critical):
    """MINRES-DR on M' = M g5 (full lattice): solutions vs dense LU, Ritz
    pairs vs dense eigh, harmonic Ritz values vs the oracle's MINRES-DR, at
    a moderate kappa and at a kappa where an eigenvalue of M' is near zero
    (the regime where the hermitian system needs MINRES-DR)."""
    require_gpu()
    dims = (4, 4, 2, 4)
    ctx, U = context(dims, 0.3, 31, 0.125)
    kappa = 0.125
    if near_critical:
        kappa, lmin = _near_critical_kappa(U, dims)
        ctx.set_kappa(kappa)
    eta = z4_noise(5, dims, 0, 2)
    say("MINRES-DR MG5", dims, "kappa", kappa)
    x, defl, st = ctx.gmresdr_solve(to_gpu(eta), op="MG5", m=40, k=20, tol=1e-12, tol_super=1e-13,
                                    eig_tol=1e-11, n_eig=8, max_cycles=400, method="minres-dr")
    M = W.dense_M(U, kappa, dims)
    Mp = M @ W.dense_gamma(L.GAMMA5, L.volume(dims))
    xref = np.linalg.solve(Mp, eta.reshape(2, -1).T).T
    xg = to_host(x).reshape(2, -1)
    cond = np.linalg.cond(Mp)
    for r in range(2):
        assert rel_err(xg[r], xref[r]) < 1e-13 * cond + 1e-10
        assert st[r]["true_resid"] < 1e-11
    Q = 6
    lam, res = defl.eigpairs(Q)
    lam_d, E_d = K.hermitian_eigpairs_dense(Mp, Q)
    assert (res < 1e-9).all()
    assert np.abs(lam - lam_d).max() < 1e-9
    # the oracle's MINRES-DR reaches the same harmonic Ritz values
    shape = eta[0].shape
    Ap = lambda v: W.apply_Mprime(U, kappa, v.reshape(shape)).ravel()
    _, info = K.minres_dr(Ap, eta[0].ravel(), 40, 20, 1e-13, max_cycles=400, eig_tol=1e-11, n_eig=8)
    th_o = np.sort(info["theta"][:6].real)
    th_g = np.sort(defl.ritz()[:6].real)
    assert np.abs(th_g - th_o).max() < 1e-9 * np.abs(th_o).max()


def test_gamma5_matches_oracle():
    require_gpu()
    dims = (4, 4, 2, 4)
    ctx, U = context(dims, 0.3, 31, 0.125)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3,) + ctx.shape) + 1j * rng.standard_normal((3,) + ctx.shape)
    y = to_host(ctx.gamma5(to_gpu(x)))
    assert np.array_equal(y, W.g5(x))
    xg = to_gpu(x)
    ctx.gamma5(xg, out=xg)  # in place
    assert np.array_equal(to_host(xg), W.g5(x))


def test_single_special_rhs_production():
    """Sec. 10's production setup: the hermitian modes of one MINRES-DR solve
    deflate every later solve of M' (GMRES-Proj on LQCD_OP_MG5, mixed
    precision), and x = g5 y solves M x = eta (compared with dense LU)."""
    require_gpu()
    dims, kappa = (4, 4, 2, 4), 0.125
    ctx, U = context(dims, 0.3, 31, kappa)
    eta0 = z4_noise(5, dims, 0, 1)
    say("production: MINRES-DR modes", dims)
    _, hdefl, _ = ctx.gmresdr_solve(to_gpu(eta0), op="MG5", m=40, k=20, tol=1e-12, tol_super=1e-13,
                                    eig_tol=1e-10, n_eig=10, max_cycles=300, method="minres-dr")
    eta = z4_noise(6, dims, 0, 4)
    say("production: deflated MG5 solves")
    y, _, st = ctx.gmresdr_solve(to_gpu(eta), op="MG5", m=40, k=20, tol=1e-11, defl=hdefl, inner="f32",
                                 inner_tol=1e-4, rhs_block=4)
    x = to_host(ctx.gamma5(y))
    xref, _ = _dense_solve(U, kappa, dims, eta)
    for r in range(4):
        assert rel_err(x[r], xref[r]) < 1e-9
        assert st[r]["true_resid"] < 1e-11


def test_minres_dr_rejects_non_hermitian_operator():
    require_gpu()
    from paper_1903_06986_amd.lqcd import LqcdError
    dims = (4, 4, 2, 4)
    ctx, U = context(dims, 0.3, 31, 0.125)
    eta = z4_noise(5, dims, 0, 1)
    with pytest.raises(LqcdError):
        ctx.gmresdr_solve(to_gpu(eta), op="schur", m=20, k=10, method="minres-dr")


@pytest.mark.parametrize("op,method", [("schur", "gmres-dr"), ("MG5", "gmres-dr"), ("MG5", "minres-dr")])
def test_first_rhs_cut_off_by_max_cycles_is_enoconv(op, method):
    """Two cycles of GMRES-DR(8,4) / MINRES-DR(8,4) cannot reach 1e-12 on
    a 4^4 lattice near kappa 0.13: the call must report ENOCONV (with the
    deflation space still handed back), not LQCD_OK."""
    require_gpu()
    import ctypes
    from paper_1903_06986_amd import lqcd
    dims = (4, 4, 4, 4)
    ctx, U = context(dims, 0.3, 33, 0.13)
    eta = to_gpu(z4_noise(6, dims, 0, 2))
    say("solve cut off", op, method)
    x = eta.clone()
    p = lqcd.SolveParams(8, 4, 2, 1e-12, 1e-12, 0.0, 0, lqcd.F64, 1e-5, 1, 0, lqcd._METHODS[method])
    st = (lqcd.SolveStats * 2)()
    h = ctypes.c_void_p(None)
    code = lqcd.lib().gmresdr_solve(ctx.handle, lqcd._OPS[op], ctypes.byref(p), lqcd._ptr(eta),
                                    lqcd._ptr(x), 2, ctypes.byref(h), st)
    assert code == 4, code                       # LQCD_ENOCONV
    assert h.value is not None                   # the deflation space is returned
    assert st[0].cycles == 2 and st[0].true_resid > 1e-12
    lqcd.lib().lqcd_defl_free(h)


@pytest.mark.parametrize("dims,kappa,nrhs,block", [((4, 4, 4, 4), 0.12, 5, 4), ((6, 4, 2, 8), 0.13, 5, 4),
                                                    ((4, 4, 4, 4), 0.12, 12, 12)])
def test_mixed_precision_solve(dims, kappa, nrhs, block):
    require_gpu()
    ctx, U = context(dims, 0.3, 1001, kappa)
    eta = z4_noise(2001, dims, 0, nrhs)
    say("solve mixed", dims, nrhs, block)
    x, defl, st = ctx.gmresdr_solve(to_gpu(eta), op="schur", m=20, k=10, tol=1e-11, tol_super=1e-13,
                                    inner="f32", inner_tol=1e-5, rhs_block=block)
    x = to_host(x)
    xref, _ = _dense_solve(U, kappa, dims, eta)
    for r in range(nrhs):
        assert rel_err(x[r], xref[r]) < 1e-9
        assert st[r]["true_resid"] < 1e-11
    assert all(s["refinements"] >= 1 for s in st[1:])


def test_full_size_true_residual_16x32():
    require_gpu()
    dims, kappa = (16, 16, 16, 32), 0.12
    ctx, U = context(dims, 0.25, 1002, kappa)
    eta = z4_noise(2002, dims, 0, 3)
    say("solve full size", dims)
    x, defl, st = ctx.gmresdr_solve(to_gpu(eta), op="schur", m=50, k=30, tol=1e-10, tol_super=1e-12,
                                    rhs_block=2)
    x = to_host(x)
    for r in range(3):
        res = np.linalg.norm(eta[r] - W.apply_M(U, kappa, x[r])) / np.linalg.norm(eta[r])
        assert res < 1.5e-10, (r, res)
        assert abs(res - st[r]["true_resid"]) < 1e-12


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_matrix_core_deflation_products(inner):
    """The deflation products V C with one shared basis (GMRES-Proj's
    x += V_k d and r -= V_{k+1} Hbar d for a block of right-hand sides, the
    Rayleigh-Ritz eigenvectors, the hermitian projections) run on the
    matrix cores; the FMA kernel is the reference.  Both give the LU
    solution to 1e-9 (their iterates differ by rounding only, so the two
    solutions agree to the solver tolerance), and the Rayleigh-Ritz
    eigenvalues of the same hermitian space agree to 1e-12."""
    require_gpu()
    dims, kappa = (6, 4, 2, 8), 0.13
    ctx, U = context(dims, 0.3, 1001, kappa)
    eta = z4_noise(2001, dims, 0, 13)
    xs = []
    for mfma in (0, 1):
        ctx.tune(gemm_mfma=mfma)
        say("solve gemm_mfma", mfma, inner)
        x, defl, st = ctx.gmresdr_solve(to_gpu(eta), op="schur", m=20, k=10, tol=1e-11, tol_super=1e-13,
                                        inner=inner, inner_tol=1e-5, rhs_block=13)
        assert max(s["true_resid"] for s in st) < 1e-11
        xs.append(to_host(x))
        _, hdefl, _ = ctx.gmresdr_solve(to_gpu(eta[:1]), op="MG5", m=30, k=18, tol=1e-12, tol_super=1e-13,
                                        eig_tol=1e-11, n_eig=12, max_cycles=400)
        lam, res = hdefl.eigpairs(12)
        if mfma == 0:
            lam0 = lam
        else:
            assert np.abs(lam - lam0).max() < 1e-10
    ctx.tune(gemm_mfma=1)
    xref, _ = _dense_solve(U, kappa, dims, eta)
    for x in xs:
        for r in range(13):
            assert rel_err(x[r], xref[r]) < 1e-9
    assert rel_err(xs[0], xs[1]) < 1e-9


@pytest.mark.parametrize("method,op", [("gmres-dr", "schur"), ("minres-dr", "MG5")])
def test_recombination_forms_agree(method, op):
    """The restart recombination V_{k+1} = V_{m+1} P in its two forms
    (outputs in registers with P in LDS, and the LDS-tiled form) gives the
    same first-right-hand-side solve: solutions and harmonic Ritz values
    agree to rounding, and the solution reaches LU."""
    require_gpu()
    dims, kappa = (6, 4, 2, 8), 0.13
    ctx, U = context(dims, 0.3, 31, kappa)
    eta = z4_noise(5, dims, 0, 1)
    out = {}
    try:
        for regs in (1, 0):
            ctx.tune(recombine_regs=regs)
            say("recombination form", regs, method)
            x, defl, st = ctx.gmresdr_solve(to_gpu(eta), op=op, m=16, k=8, tol=1e-12, tol_super=1e-13,
                                            max_cycles=400, method=method)
            assert st[0]["cycles"] > 2, st[0]  # several restarts ran
            out[regs] = (to_host(x), np.sort_complex(defl.ritz()[:10]), st[0]["matvecs"])
    finally:
        ctx.tune(recombine_regs=1)
    M = W.dense_M(U, kappa, dims)
    if op == "MG5":
        M = M @ W.dense_gamma(L.GAMMA5, L.volume(dims))
        xref = np.linalg.solve(M, eta.reshape(1, -1).T).T.reshape(eta.shape)
    else:
        xref = np.linalg.solve(M, eta.reshape(1, -1).T).T.reshape(eta.shape)
    assert rel_err(out[1][0], xref) < 1e-9
    assert rel_err(out[1][0], out[0][0]) < 1e-11
    assert np.abs(out[1][1] - out[0][1]).max() < 1e-9 * np.abs(out[0][1]).max()
    assert abs(out[1][2] - out[0][2]) <= 8
