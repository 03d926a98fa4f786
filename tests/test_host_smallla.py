"""The library's host dense linear algebra against LAPACK (numpy), on CPU.

The solvers' projected problems (Hessenberg least squares, harmonic Ritz
eigenproblems, Rayleigh-Ritz) run in paper_1903_06986_amd/csrc/smallla.cpp;
this builds that file alone with g++ and compares it with numpy."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def la():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "libla.so")
    src = [os.path.join(ROOT, "tests", "native", "smallla_capi.cpp"),
           os.path.join(ROOT, "paper_1903_06986_amd", "csrc", "smallla.cpp")]
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", so] + src, check=True)
    return ctypes.CDLL(so)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cm(a):
    return np.asfortranarray(a.astype(np.complex128))


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("n", [1, 2, 5, 20, 80])
def test_eig_general(la, n):
    rng = np.random.default_rng(n)
    A = _cm(_rand(rng, n, n))
    w = np.zeros(n, complex)
    V = np.zeros((n, n), complex, order="F")
    assert la.la_eig(n, _p(A), _p(w), _p(V)) == 0
    assert np.abs(A @ V - V * w).max() < 1e-11 * np.abs(A).max() * n
    ref = np.linalg.eigvals(A)
    for x in w:
        assert np.min(np.abs(ref - x)) < 1e-10 * np.abs(ref).max()


def test_eig_hessenberg_like_gmres(la):
    """Harmonic-Ritz-type matrix: Hessenberg plus a rank-one last column."""
    rng = np.random.default_rng(7)
    m = 40
    H = np.triu(_rand(rng, m, m), -1)
    f = _rand(rng, m)
    G = _cm(H + np.outer(f, np.eye(m)[-1]))
    w = np.zeros(m, complex)
    V = np.zeros((m, m), complex, order="F")
    assert la.la_eig(m, _p(G), _p(w), _p(V)) == 0
    assert np.abs(G @ V - V * w).max() < 1e-10 * np.abs(G).max()


@pytest.mark.parametrize("n", [1, 3, 30])
def test_eigh(la, n):
    rng = np.random.default_rng(10 + n)
    B = _rand(rng, n, n)
    A = _cm(B + B.conj().T)
    w = np.zeros(n)
    V = np.zeros((n, n), complex, order="F")
    la.la_eigh(n, _p(A), _p(w), _p(V))
    assert np.abs(w - np.linalg.eigvalsh(A)).max() < 1e-12 * np.abs(w).max()
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-13
    assert np.abs(A @ V - V * w).max() < 1e-12 * np.abs(A).max()


def test_lstsq_and_solve(la):
    rng = np.random.default_rng(3)
    for r, c in ((21, 20), (41, 40), (9, 3)):
        A = _cm(np.triu(_rand(rng, r, c), -1))
        b = _rand(rng, r)
        x = np.zeros(c, complex)
        la.la_lstsq(r, c, _p(A), _p(b), _p(x))
        ref = np.linalg.lstsq(A, b, rcond=None)[0]
        assert np.abs(x - ref).max() < 1e-11 * np.abs(ref).max()
    A = _cm(_rand(rng, 15, 15))
    b = _rand(rng, 15)
    x = np.zeros(15, complex)
    la.la_solve(15, _p(A), _p(b), _p(x))
    assert np.abs(A @ x - b).max() < 1e-12


def test_thin_q(la):
    rng = np.random.default_rng(4)
    A = _cm(_rand(rng, 30, 11))
    Q = np.zeros((30, 11), complex, order="F")
    la.la_thin_q(30, 11, _p(A), _p(Q))
    assert np.abs(Q.conj().T @ Q - np.eye(11)).max() < 1e-14
    # same column space
    P = Q @ Q.conj().T
    assert np.abs(P @ A - A).max() < 1e-12


@pytest.mark.parametrize("n", [1, 4, 40])
def test_cholesky_inverse(la, n):
    """Li = L^{-1} of the Cholesky factor: lower triangular, L = numpy's
    factor, and Li A Li^H = I; a matrix that is not positive definite is
    refused."""
    rng = np.random.default_rng(20 + n)
    B = _rand(rng, n + 3, n)
    A = _cm(B.conj().T @ B)
    Li = np.zeros((n, n), complex, order="F")
    assert la.la_cholesky_inv(n, _p(A), _p(Li)) == 0
    assert np.abs(np.triu(Li, 1)).max(initial=0) == 0
    assert np.abs(np.linalg.inv(Li) - np.linalg.cholesky(A)).max() < 1e-10 * np.abs(A).max()
    assert np.abs(Li @ A @ Li.conj().T - np.eye(n)).max() < 1e-10
    C = _cm(-A)
    assert la.la_cholesky_inv(n, _p(C), _p(Li)) == 1
