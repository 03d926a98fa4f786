"""Plain-C form of the hopping matrix P (Sec. 5.1 Eqs. (24)-(25)) for large
lattices (oracle; test and workload infrastructure only).

`hop_c(U, psi)` computes the same P psi as `oracle.wilson.hop`, site by site
in C (oracle/c/hop.c, OpenMP), with the spin projectors taken from
`oracle.lattice.GAMMA`.  The shared object is built by `build()` (gcc) into
oracle/c/liboraclehop.so.
"""
import ctypes
import os
import subprocess

import numpy as np

from .lattice import GAMMA

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "c", "hop.c")
LIB = os.path.join(_HERE, "c", "liboraclehop.so")
_ONE = np.eye(4, dtype=np.complex128)
_PM = np.ascontiguousarray(np.array([_ONE - GAMMA[mu] for mu in range(4)]))
_PP = np.ascontiguousarray(np.array([_ONE + GAMMA[mu] for mu in range(4)]))
_lib = None


def build():
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", SRC, "-o", LIB])


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.oracle_hop.argtypes = [ctypes.c_void_p] * 6 + [ctypes.c_int]
        L.oracle_hop.restype = None
        L.oracle_hop_parity.argtypes = [ctypes.c_void_p] * 6 + [ctypes.c_int, ctypes.c_int]
        L.oracle_hop_parity.restype = None
        _lib = L
    return _lib


def hop_c(U, psi, threads=None, parity=None):
    """P psi for one field of shape (Lt, Lz, Ly, Lx, 4, 3); with parity 0
    or 1 only the output sites of that parity (the rest zero)."""
    Lt, Lz, Ly, Lx = psi.shape[:4]
    dims = np.array([Lx, Ly, Lz, Lt], dtype=np.int32)
    U = np.ascontiguousarray(U, dtype=np.complex128)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty_like(psi)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    nt = int(threads or os.cpu_count() or 1)
    if parity is None:
        _load().oracle_hop(p(dims), p(U), p(_PM), p(_PP), p(psi), p(out), nt)
    else:
        _load().oracle_hop_parity(p(dims), p(U), p(_PM), p(_PP), p(psi), p(out), int(parity), nt)
    return out
