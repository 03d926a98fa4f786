"""Lattice conventions (oracle; test infrastructure only).

The paper (Sec. 2) indexes vectors in "space-time-color-Dirac space" without
fixing a gamma basis or an ordering; the choices below are the readings this
project fixes for both sides.  Pinned by tests/test_oracle_lattice.py
(Clifford algebra, gamma5 = g1 g2 g3 g4, parity/checkerboard bijections).

* Euclidean hermitian gammas in the chiral basis
  g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0, 1], [1, 0]],
  g_5 = g_1 g_2 g_3 g_4 = diag(1, 1, -1, -1).
* mu = 0..3 are the x, y, z, t directions; extents dims = (Lx, Ly, Lz, Lt).
* Lexicographic site s = x + Lx (y + Ly (z + Lz t)); vector index
  (s * 4 + spin) * 3 + colour.  Fields are arrays of shape
  (Lt, Lz, Ly, Lx, 4, 3) (numpy C order reproduces that index).
* Parity (x + y + z + t) mod 2; checkerboard index s >> 1 (a bijection from
  each parity onto 0..V/2-1 because Lx is even).
* Periodic boundaries in all four directions (Sec. 7 states periodic
  fermion boundary conditions).
"""
import numpy as np

SIGMA = np.array([[[0, 1], [1, 0]],
                  [[0, -1j], [1j, 0]],
                  [[1, 0], [0, -1]]], dtype=np.complex128)


def gammas():
    """Return (g[0..3], g5) as complex128 4x4 arrays; g[mu] for mu = x,y,z,t."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    z2 = np.zeros((2, 2))
    for k in range(3):
        g[k] = np.block([[z2, -1j * SIGMA[k]], [1j * SIGMA[k], z2]])
    g[3] = np.block([[z2, np.eye(2)], [np.eye(2), z2]])
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


GAMMA, GAMMA5 = gammas()


def volume(dims):
    Lx, Ly, Lz, Lt = dims
    return Lx * Ly * Lz * Lt


def check_dims(dims):
    if len(dims) != 4 or any(int(L) < 2 or int(L) % 2 for L in dims):
        raise ValueError("every extent must be even and >= 2: %r" % (dims,))


def coords(dims):
    """Integer coordinate arrays (x, y, z, t), each of shape (Lt, Lz, Ly, Lx)."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly),
                             np.arange(Lx), indexing="ij")
    return x, y, z, t


def parity(dims):
    x, y, z, t = coords(dims)
    return (x + y + z + t) % 2


def lex_site(dims):
    x, y, z, t = coords(dims)
    Lx, Ly, Lz, _ = dims
    return x + Lx * (y + Ly * (z + Lz * t))


def eo_tables(dims):
    """Checkerboard tables.

    Returns (even_sites, odd_sites): for each parity p an int64 array whose
    entry cb is the lexicographic site s with parity p and s >> 1 == cb.
    """
    check_dims(dims)
    V = volume(dims)
    s = lex_site(dims).ravel()
    p = parity(dims).ravel()
    tabs = []
    for par in (0, 1):
        tab = np.full(V // 2, -1, dtype=np.int64)
        sel = s[p == par]
        tab[sel >> 1] = sel
        assert (tab >= 0).all()
        tabs.append(tab)
    return tabs[0], tabs[1]


def to_eo(dims, field):
    """Split a lexicographic field (..., Lt, Lz, Ly, Lx, 4, 3) into
    (even, odd) checkerboard arrays of shape (..., V/2, 4, 3)."""
    ev, od = eo_tables(dims)
    V = volume(dims)
    lead = field.shape[:-6]
    f = field.reshape(lead + (V, 4, 3))
    return f[..., ev, :, :], f[..., od, :, :]


def from_eo(dims, even, odd):
    ev, od = eo_tables(dims)
    V = volume(dims)
    lead = even.shape[:-3]
    f = np.zeros(lead + (V, 4, 3), dtype=np.result_type(even, odd))
    f[..., ev, :, :] = even
    f[..., od, :, :] = odd
    Lx, Ly, Lz, Lt = dims
    return f.reshape(lead + (Lt, Lz, Ly, Lx, 4, 3))


def timeslice_of_site(dims):
    """t coordinate of every lexicographic site (length V)."""
    Lx, Ly, Lz, Lt = dims
    return np.arange(volume(dims)) // (Lx * Ly * Lz)
