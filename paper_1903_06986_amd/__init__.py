"""MI355X (gfx950) library for disconnected-loop noise estimation with
deflated GMRES solves and perturbative / polynomial / hermitian-forced
subtraction (Baral, Whyte, Wilcox, Morgan, arXiv:1903.06986).

The compute path is the C ABI of ``include/lqcd.h`` implemented in HIP
(``csrc/``, built into ``liblqcd.so``); ``lqcd`` is its ctypes binding.
"""
from . import lqcd  # noqa: F401
from .lqcd import Batch, Context, Deflation, LqcdError, lib  # noqa: F401
