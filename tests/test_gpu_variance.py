"""GPU variance harness against the oracle pipeline on the 4^4 configuration
(the same seeds, GMRES-DR(20,10), PS order 4, POLY degree 4, Q = 10): the
standard errors of the signal parts of the whole-lattice traces for all six
methods, to 1e-6 relative.  The GPU's hermitian modes come from MINRES-DR
(eigen-residual <= 1e-12 |lambda'|), the oracle's are the exact ones
(dense eigh of M' on 4^4)."""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, say
from synth import random_su3_links, get_config
from oracle import pipeline as opipe

pytestmark = pytest.mark.gpu


def test_config_errors_match_oracle():
    require_gpu()
    from paper_1903_06986_amd import Context
    from paper_1903_06986_amd import variance as Vh
    cfg = get_config("c1")
    dims, kappa = cfg["dims"], cfg["kappas"][0]
    U = random_su3_links(dims, cfg["eps"], cfg["link_seed"])
    ctx = Context(dims, U, kappa)
    eta = ctx.noise_z4(cfg["noise_seed"], 0, cfg["n_noise"])
    thetas = (0, 1, 2, 3, 4)
    p = dict(m=cfg["m"], k=cfg["k"], herm_m=cfg["herm_m"], herm_k=cfg["herm_k"], pert_order=cfg["pert_order"],
             poly_degree=cfg["poly_degree"], tol=1e-12, tol_super=1e-13, inner="f64", inner_tol=1e-5,
             rhs_block=4, max_cycles=2000, eig_tol=1e-12)
    say("variance harness c1")
    g = Vh.config_errors(ctx, eta, thetas, (0, 5, cfg["n_hermitian"]), p)
    say("oracle pipeline c1")
    from oracle import wilson as W, lattice as L, krylov as K
    Q = cfg["n_hermitian"]
    lam, Ev = K.hermitian_eigpairs_dense(W.dense_M(U, kappa, dims) @ W.dense_gamma(L.GAMMA5, L.volume(dims)), Q)
    o = opipe.run(U, dims, kappa, cfg["noise_seed"], cfg["n_noise"], cfg["m"], cfg["k"], cfg["pert_order"],
                  cfg["poly_degree"], Q, tol=1e-12, tol_super=1e-13,
                  modes=(lam, Ev.T.reshape((Q, dims[3], dims[2], dims[1], dims[0], 4, 3))))
    sig = [Vh.signal_part(t) for t in thetas]
    for meth in ("NS", "PS", "POLY", "HFES", "HFPS", "HFPOLY"):
        ref = np.array([o["methods"][meth]["err"][a, -1, sig[a]] for a in range(len(thetas))])
        got = g[meth] if meth in ("NS", "PS", "POLY") else g[(meth, cfg["n_hermitian"])]
        np.testing.assert_allclose(got, ref, rtol=1e-6, err_msg=meth)
    # Q = 0 reduces the hermitian-forced methods to NS, PS, POLY
    assert np.array_equal(g[("HFES", 0)], g["NS"])
    assert np.array_equal(g[("HFPOLY", 0)], g["POLY"])
