"""Pins for the workload helpers of the oracle: the plain-C hopping matrix
and the rightmost-eigenvalue search that fixes the near-critical kappa.

* hop_c equals the numpy stencil (two independent codings of Eq. (25));
* ARPACK's rightmost eigenvalues of P equal those of the dense matrix;
* on unit links the rightmost eigenvalue is the free-field value 8 (p = 0).
"""
import numpy as np
import pytest

from synth import random_su3_links, unit_links
from oracle import wilson as W
from oracle import critical_kappa as C
from oracle.chop import hop_c


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (4, 6, 2, 8)])
def test_c_hop_matches_numpy_hop(dims):
    U = random_su3_links(dims, 0.3, 5)
    rng = np.random.default_rng(1)
    shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = W.hop(U, v)
    assert np.abs(hop_c(U, v, threads=2) - ref).max() < 1e-13 * np.abs(ref).max()


def test_rightmost_eigenvalue_matches_dense():
    dims = (2, 2, 2, 4)
    U = random_su3_links(dims, 0.3, 1001)
    ev = np.linalg.eigvals(W.dense_P(U, dims))
    vals, vec, _ = C.rightmost_eig(U, dims, tol=1e-10, ncv=40)
    assert abs(vals[0].real - ev.real.max()) < 1e-9
    shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    v = vec.reshape(shape)
    assert np.linalg.norm(W.hop(U, v) - vals[0] * v) < 1e-8 * np.linalg.norm(v)


def test_rightmost_eigenvalue_free_field():
    dims = (4, 4, 2, 4)
    vals, _, _ = C.rightmost_eig(unit_links(dims), dims, tol=1e-10, ncv=40)
    assert abs(vals[0] - 8.0) < 1e-8


def test_rightmost_eigenvalue_through_even_odd_square():
    """The even/odd-square search finds the same rightmost eigenvalue (up to
    conjugation: both members of a pair have the same real part) and an
    eigenvector of P itself."""
    dims = (2, 2, 2, 4)
    U = random_su3_links(dims, 0.3, 1001)
    ev = np.linalg.eigvals(W.dense_P(U, dims))
    mu, _, v, _ = C.rightmost_eig_eo(U, dims, tol=1e-10, ncv=40)
    assert abs(mu.real - ev.real.max()) < 1e-9
    assert np.linalg.norm(W.hop(U, v) - mu * v) < 1e-8 * np.linalg.norm(v)


def test_c_hop_parity_blocks():
    dims = (4, 6, 2, 8)
    U = random_su3_links(dims, 0.3, 5)
    rng = np.random.default_rng(2)
    shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    full = W.hop(U, v)
    from oracle.lattice import parity
    par = parity(dims)[..., None, None]
    for p in (0, 1):
        out = hop_c(U, v, threads=2, parity=p)
        assert np.abs(out - np.where(par == p, full, 0)).max() < 1e-13 * np.abs(full).max()
