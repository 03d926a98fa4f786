"""End-to-end oracle run on the 4^4 configuration (CPU).

The full path (Sec. 7's procedure) on 4^4, eps = 0.3, kappa = 0.12 with 8
Z(4) noises: every solution meets its residual target, the estimates of
every method agree with the exact dense Tr(Theta M^{-1}) within their error
bars, and the subtraction reduces the error bar of the scalar (the
variance argument of Sec. 4).
"""
import numpy as np
import pytest

from synth import random_su3_links, get_config
from oracle import lattice as L
from oracle import wilson as W
from oracle import subtract as S
from oracle import pipeline


@pytest.fixture(scope="module")
def c1():
    cfg = get_config("c1")
    dims = cfg["dims"]
    U = random_su3_links(dims, cfg["eps"], cfg["link_seed"])
    kappa = cfg["kappas"][0]
    out = pipeline.run(U, dims, kappa, cfg["noise_seed"], cfg["n_noise"], cfg["m"], cfg["k"],
                       cfg["pert_order"], cfg["poly_degree"], cfg["n_hermitian"],
                       herm_m=cfg["herm_m"], herm_k=cfg["herm_k"])
    return cfg, U, kappa, out


def test_solutions(c1):
    cfg, U, kappa, out = c1
    r = out["eta"] - W.apply_M(U, kappa, out["x"])
    rel = np.linalg.norm(r.reshape(r.shape[0], -1), axis=1) / np.linalg.norm(out["eta"].reshape(r.shape[0], -1), axis=1)
    assert rel.max() < 1e-11
    assert out["mode_resid"].max() < 1e-8


def test_estimates_consistent_with_exact_trace(c1):
    cfg, U, kappa, out = c1
    dims = cfg["dims"]
    Minv = np.linalg.inv(W.dense_M(U, kappa, dims))
    exact = S.trace_correction_dense(Minv, dims, (0, 1, 2, 3, 4)).sum(axis=-1)
    for meth, res in out["methods"].items():
        est, err = res["est"][:, -1], res["err"][:, -1]
        # scalar signal in Re, vector signal in Im
        assert abs(est[0].real - exact[0].real) < 5 * err[0, 0] + 1e-9, meth
        for th in range(1, 5):
            assert abs(est[th].imag - exact[th].imag) < 5 * err[th, 1] + 1e-9, meth
    ns = out["methods"]["NS"]["err"][0, -1, 0]
    assert out["methods"]["HFPOLY"]["err"][0, -1, 0] < ns
    assert out["methods"]["PS"]["err"][0, -1, 0] < ns
