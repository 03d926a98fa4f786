"""Synthetic SU(3) gauge fields.

The paper measures on quenched Wilson ensembles at beta = 6.0 and on MILC
dynamical lattices; neither is available here.  Stand-in links have the same
shapes and are drawn as U = exp(i eps H) with H a random traceless hermitian
3x3 matrix (independent Gaussian real and imaginary entries), eps setting how
far the field is from the free (unit-link) case.

Layout (the library's external layout): complex128 array of shape
``(Lt, Lz, Ly, Lx, 4, 3, 3)``, i.e. ``[t][z][y][x][mu][row][col]`` with
mu = 0..3 the x, y, z, t directions.
"""
import numpy as np


def unit_links(dims):
    """Free field: every link is the 3x3 identity.  dims = (Lx, Ly, Lz, Lt)."""
    Lx, Ly, Lz, Lt = dims
    U = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def random_su3_links(dims, eps, seed):
    """U = exp(i eps H), H traceless hermitian with Gaussian entries.

    A has iid N(0,1) real and imaginary parts (drawn from a PCG64 stream with
    the given seed, all real parts of the whole field first, then all
    imaginary parts, each in [t][z][y][x][mu][row][col] order);
    H = (A + A^dagger)/2 - tr(.)/3; the exponential uses the FP64 eigh of H,
    so U is unitary with det U = 1 to rounding.
    """
    Lx, Ly, Lz, Lt = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (Lt, Lz, Ly, Lx, 4, 3, 3)
    A = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[..., None, None] * np.eye(3)
    w, v = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    U = np.einsum("...ak,...k,...bk->...ab", v, ph, np.conj(v))
    return np.ascontiguousarray(U)
