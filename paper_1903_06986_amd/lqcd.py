"""Python binding of the gfx950 C ABI in ``include/lqcd.h`` (ctypes).

Argument marshalling only: every computation runs in ``liblqcd.so``.  Field
arguments are torch tensors on the GPU (complex128, lexicographic layout
[rhs][t][z][y][x][spin][colour] unless stated otherwise); torch supplies the
device memory and the stream, nothing else.  The library must have been
built (``paper_1903_06986_amd.build``); there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblqcd.so")

F64, F32, F16, BF16 = 0, 1, 2, 3
OP_M, OP_MDAG, OP_MG5, OP_HOP, OP_SCHUR = 0, 1, 2, 3, 4
LAYOUT_LEX, LAYOUT_EO = 0, 1
NS, PS, POLY, HFES, HFPS, HFPOLY = 0, 1, 2, 3, 4, 5
DEFL_HFES, DEFL_EIGPOLY, DEFL_ES = 0, 1, 2
_PREC = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16}
_OPS = {"M": OP_M, "Mdag": OP_MDAG, "MG5": OP_MG5, "hop": OP_HOP, "schur": OP_SCHUR}

STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOCONV", 5: "EBREAKDOWN", 6: "ENAN"}


class LqcdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class SolveParams(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("k", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("tol", ctypes.c_double), ("tol_super", ctypes.c_double),
                ("eig_tol", ctypes.c_double), ("n_eig", ctypes.c_int),
                ("inner", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("rhs_block", ctypes.c_int), ("proj_m", ctypes.c_int), ("method", ctypes.c_int)]


_METHODS = {"gmres-dr": 0, "minres-dr": 1}


class SolveStats(ctypes.Structure):
    _fields_ = [("matvecs", ctypes.c_int), ("cycles", ctypes.c_int),
                ("refinements", ctypes.c_int), ("reorth", ctypes.c_int), ("true_resid", ctypes.c_double)]


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "lqcd_create": [ctypes.POINTER(ctypes.c_int), _P, _D, _P, ctypes.POINTER(_P)],
    "lqcd_set_kappa": [_P, _D],
    "lqcd_set_stream": [_P, _P],
    "lqcd_destroy": [_P],
    "lqcd_noise_z4": [_P, ctypes.c_uint64, ctypes.c_int64, _I, _P, _P],
    "lqcd_pack_eo": [_P, _I, _P, _P, _I],
    "lqcd_unpack_eo": [_P, _I, _P, _P, _I],
    "lqcd_gamma5": [_P, _P, _P, _I],
    "wilson_apply": [_P, _I, _I, _I, _P, _P, _I],
    "gmresdr_solve": [_P, _I, ctypes.POINTER(SolveParams), _P, _P, _I, ctypes.POINTER(_P),
                      ctypes.POINTER(SolveStats)],
    "lqcd_defl_eigpairs": [_P, _P, _I, _P, _P],
    "lqcd_defl_ritz": [_P, _P, ctypes.POINTER(ctypes.c_int)],
    "deflate_project": [_P, _P, _I, _I, _P, _I, _P, _I, _P, _P, _I, _P, _P],
    "deflate_project_multi": [_P, _P, _I, _I, _P, _P, _P, _P, _I, _P, _P, _I, _P],
    "pert_subtract": [_P, _I, _P, _I, _P, _P, _I, _P],
    "poly_subtract": [_P, _I, _P, _P, _P, _P, _I, _P, _P, _I, _P],
    "poly_subtract_multi": [_P, _I, _I, _P, _P, _P, _I],
    "loop_estimate": [_P, _P, _I, _P, _P, _P, _I, _P, _P, _P, _P],
    "loop_estimate_noalloc": [_P, _P, _I, _P, _P, _P, _I, _P, _P, _P, _P],
    "loop_estimate_multi": [_P, _P, _I, _P, _P, _P, _I, _I, _P, _P, _P, _P],
    "loop_gradient": [_P, _P, _P, _I, ctypes.POINTER(SolveParams), ctypes.POINTER(_P), _P, _P, _I,
                      _P, _P, ctypes.POINTER(SolveStats)],
    "lqcd_batch_create": [_P, _I, ctypes.POINTER(_P)],
    "lqcd_batch_destroy": [_P],
    "lqcd_batch_set_grid": [_P, _I],
    "lqcd_batch_set_tile": [_P, _I],
    "batch_solve": [_P, ctypes.POINTER(SolveParams), _P, _P, _P, _P, _I, ctypes.POINTER(SolveStats)],
    "batch_autotune": [_P, ctypes.POINTER(SolveParams), _P, _P, _P, ctypes.POINTER(_I), ctypes.POINTER(_I), _P],
    "batch_wilson_apply": [_P, _P, _P, _P],
    "lqcd_timer_enable": [_P, _I],
    "lqcd_timer_read": [_P, _I, _P, _P, _P],
    "lqcd_tune_set": [_P, _I, _I],
}


def lib():
    """Load liblqcd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblqcd.so is not built (%s); run paper_1903_06986_amd.build.build()"
                           % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.lqcd_defl_free.argtypes = [_P]
    L.lqcd_defl_free.restype = None
    L.lqcd_last_error.argtypes = []
    L.lqcd_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(code):
    if code != 0:
        raise LqcdError(code, lib().lqcd_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("field tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("field tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _field(t, nrhs, per_rhs, what, dtype=None):
    """Check a device field before its pointer goes to the library: a
    contiguous GPU tensor of `dtype` (complex128 unless given) holding
    nrhs * per_rhs elements.  A wrong size or type would make the kernels
    read or write past the allocation."""
    import torch
    dtype = torch.complex128 if dtype is None else dtype
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s: expected a torch tensor" % what)
    if t.dtype != dtype:
        raise ValueError("%s: dtype %s, expected %s" % (what, t.dtype, dtype))
    if t.numel() != nrhs * per_rhs:
        raise ValueError("%s: %d elements, expected %d right-hand sides of %d"
                         % (what, t.numel(), nrhs, per_rhs))
    return _ptr(t)


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _thetas(thetas):
    t = np.ascontiguousarray(np.asarray(thetas, dtype=np.int32))
    return t, t.ctypes.data_as(ctypes.c_void_p), len(t)


class Deflation:
    """Owns an lqcd_defl handle (deflation space of one operator)."""

    def __init__(self, handle, ctx):
        self.handle = handle
        self.ctx = ctx

    def eigpairs(self, Q):
        lam = np.zeros(Q)
        res = np.zeros(Q)
        _check(lib().lqcd_defl_eigpairs(self.ctx.handle, self.handle, Q,
                                        lam.ctypes.data_as(_P), res.ctypes.data_as(_P)))
        return lam, res

    def ritz(self):
        k = ctypes.c_int(0)
        buf = np.zeros(1024, dtype=np.complex128)
        _check(lib().lqcd_defl_ritz(self.handle, buf.ctypes.data_as(_P), ctypes.byref(k)))
        return buf[:k.value].copy()

    def free(self):
        if self.handle:
            lib().lqcd_defl_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """A lattice, its links on the GPU and a hopping parameter."""

    def __init__(self, dims, links, kappa, stream=None):
        import torch
        self.dims = tuple(int(d) for d in dims)
        Lx, Ly, Lz, Lt = self.dims
        self.V = Lx * Ly * Lz * Lt
        self.shape = (Lt, Lz, Ly, Lx, 4, 3)
        self.kappa = float(kappa)
        U, Up = _host(links, np.complex128)
        if U.size != self.V * 36:
            raise ValueError("links must hold V*4*3*3 complex numbers")
        d = (ctypes.c_int * 4)(*self.dims)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _P()
        _check(lib().lqcd_create(d, Up, self.kappa, _P(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().lqcd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    KERNEL_CLASSES = ("hop64", "hop32", "dot", "axpy", "gemm", "force")

    def tune(self, hop_nb64=None, hop_nb32=None, hop_tile64=None, hop_tile32=None, hop_order=None,
             hop_tblock64=None, hop_tblock32=None, hop_tsites32=None, hop_rgroup=None, hop_tsites64=None,
             gemm_mfma=None, hop_rnest=None, cycle_reorth=None, kept_period=None,
             arnoldi_steps=None, sstep_z16=None, recombine_regs=None):
        """Set launch-shape parameters (see lqcd_tune_set)."""
        for code, v in ((0, hop_nb64), (1, hop_nb32), (2, hop_tile64), (3, hop_tile32), (4, hop_order),
                        (5, hop_tblock64), (6, hop_tblock32), (7, hop_tsites32), (8, hop_rgroup),
                        (9, hop_tsites64), (10, gemm_mfma), (11, hop_rnest), (12, cycle_reorth), (13, kept_period),
                        (14, arnoldi_steps), (15, sstep_z16), (16, recombine_regs)):
            if v is not None:
                _check(lib().lqcd_tune_set(self.handle, code, int(v)))

    def timer(self, on):
        """Enable (and reset) or disable per-kernel-class event timing."""
        _check(lib().lqcd_timer_enable(self.handle, 1 if on else 0))

    def timer_read(self):
        """{class: (milliseconds, algorithmic bytes, launches)} since enabling."""
        out = {}
        for k, name in enumerate(self.KERNEL_CLASSES):
            ms, by, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
            _check(lib().lqcd_timer_read(self.handle, k, ctypes.byref(ms), ctypes.byref(by), ctypes.byref(n)))
            out[name] = (ms.value, by.value, n.value)
        return out

    def set_kappa(self, kappa):
        self.kappa = float(kappa)
        _check(lib().lqcd_set_kappa(self.handle, self.kappa))

    # ------------------------------------------------------------ fields
    def empty(self, nrhs):
        import torch
        return torch.empty((nrhs,) + self.shape, dtype=torch.complex128, device="cuda")

    def noise_z4(self, seed, first, nrhs, codes=False):
        import torch
        eta = self.empty(nrhs)
        cd = torch.empty((nrhs,) + self.shape, dtype=torch.uint8, device="cuda") if codes else None
        _check(lib().lqcd_noise_z4(self.handle, ctypes.c_uint64(seed), first, nrhs, _ptr(eta),
                                   _field(cd, nrhs, 12 * self.V, "codes", torch.uint8) if codes else None))
        return (eta, cd) if codes else eta

    def pack_eo(self, x, prec="f64"):
        import torch
        dt = torch.complex128 if prec == "f64" else torch.complex64
        out = torch.empty((x.shape[0], 2, 12, self.V // 2), dtype=dt, device="cuda")
        _check(lib().lqcd_pack_eo(self.handle, _PREC[prec], _field(x, x.shape[0], 12 * self.V, "x"),
                                  _ptr(out), x.shape[0]))
        return out

    def unpack_eo(self, eo, prec="f64"):
        import torch
        out = self.empty(eo.shape[0])
        dt = torch.complex128 if prec == "f64" else torch.complex64
        _check(lib().lqcd_unpack_eo(self.handle, _PREC[prec], _field(eo, eo.shape[0], 12 * self.V, "eo", dt),
                                    _ptr(out), eo.shape[0]))
        return out

    def gamma5(self, x, out=None):
        """g5 x for LEX complex128 fields (in place when out is x)."""
        import torch
        if x.numel() != x.shape[0] * 12 * self.V or x.dtype != torch.complex128:
            raise ValueError("gamma5 needs LEX complex128 fields of this lattice")
        out = torch.empty_like(x) if out is None else out
        n = x.shape[0]
        _check(lib().lqcd_gamma5(self.handle, _field(x, n, 12 * self.V, "x"),
                                 _field(out, n, 12 * self.V, "out"), n))
        return out

    def wilson_apply(self, op, x, prec="f64", layout="lex", out=None):
        import torch
        if x.numel() != x.shape[0] * 12 * self.V:
            raise ValueError("field size does not match the lattice")
        if out is None:
            out = torch.empty_like(x)
        lay = LAYOUT_LEX if layout == "lex" else LAYOUT_EO
        dt = torch.complex128 if (lay == LAYOUT_LEX or prec == "f64") else torch.complex64
        n = x.shape[0]
        _check(lib().wilson_apply(self.handle, _OPS[op], _PREC[prec], lay, _field(x, n, 12 * self.V, "x", dt),
                                  _field(out, n, 12 * self.V, "out", dt), n))
        return out

    # ----------------------------------------------------------- solvers
    def gmresdr_solve(self, b, op="schur", m=20, k=10, tol=1e-10, tol_super=1e-13, eig_tol=0.0,
                      n_eig=0, max_cycles=1000, inner="f64", inner_tol=1e-5, rhs_block=1,
                      defl=None, proj_m=0, method="gmres-dr"):
        """method: "gmres-dr" or "minres-dr" (hermitian op "MG5" only) for the
        first right-hand side when no deflation data is given."""
        import torch
        x = torch.empty_like(b)
        nrhs = b.shape[0]
        p = SolveParams(m, k, max_cycles, tol, tol_super, eig_tol, n_eig, _PREC[inner], inner_tol,
                        rhs_block, proj_m, _METHODS[method])
        stats = (SolveStats * max(nrhs, 1))()
        h = _P(defl.handle.value if defl is not None else None)
        code = lib().gmresdr_solve(self.handle, _OPS[op], ctypes.byref(p), _field(b, nrhs, 12 * self.V, "b"),
                                   _field(x, nrhs, 12 * self.V, "x"), nrhs, ctypes.byref(h), stats)
        newdefl = Deflation(_P(h.value), self) if (defl is None and h.value) else defl
        _check(code)
        st = [dict(matvecs=s.matvecs, cycles=s.cycles, refinements=s.refinements, reorth=s.reorth,
                   true_resid=s.true_resid) for s in stats[:nrhs]]
        return x, newdefl, st

    # --------------------------------------------------------- subtraction
    def pert_subtract(self, order, eta, thetas=(0, 1, 2, 3, 4), want_corr=True):
        import torch
        xt = torch.empty_like(eta)
        th, thp, nth = _thetas(thetas)
        corr = np.zeros((nth, self.dims[3]), dtype=np.complex128)
        n = eta.shape[0]
        _check(lib().pert_subtract(self.handle, order, thp, nth, _field(eta, n, 12 * self.V, "eta"),
                                   _field(xt, n, 12 * self.V, "xt"), n,
                                   corr.ctypes.data_as(_P) if want_corr else None))
        return xt, corr

    def poly_subtract(self, degree, eta, b=None, coeffs=None, thetas=(0, 1, 2, 3, 4), want_corr=True):
        import torch
        xt = torch.empty_like(eta)
        th, thp, nth = _thetas(thetas)
        c = np.zeros(degree + 1, dtype=np.complex128) if coeffs is None else \
            np.ascontiguousarray(coeffs, dtype=np.complex128).copy()
        a = np.zeros(degree + 1, dtype=np.complex128)
        corr = np.zeros((nth, self.dims[3]), dtype=np.complex128)
        n = eta.shape[0]
        bp = None if b is None else _field(b, 1, 12 * self.V, "b")
        _check(lib().poly_subtract(self.handle, degree, bp, c.ctypes.data_as(_P),
                                   a.ctypes.data_as(_P), thp, nth, _field(eta, n, 12 * self.V, "eta"),
                                   _field(xt, n, 12 * self.V, "xt"), n,
                                   corr.ctypes.data_as(_P) if want_corr else None))
        return xt, corr, c, a

    def deflate_project(self, defl, Q, eta, xt=None, corr=None, mode=DEFL_HFES, coeffs=None,
                        thetas=(0, 1, 2, 3, 4)):
        import torch
        th, thp, nth = _thetas(thetas)
        if xt is None:
            xt = torch.zeros_like(eta)
        corr = np.zeros((nth, self.dims[3]), dtype=np.complex128) if corr is None else \
            np.ascontiguousarray(corr, dtype=np.complex128).copy()
        cf, cfp = (None, None) if coeffs is None else _host(coeffs, np.complex128)
        xi = np.zeros(Q, dtype=np.complex128)
        n = eta.shape[0]
        _check(lib().deflate_project(self.handle, defl.handle, Q, mode, cfp,
                                     0 if coeffs is None else len(cf), thp, nth,
                                     _field(eta, n, 12 * self.V, "eta"), _field(xt, n, 12 * self.V, "xt"),
                                     n, corr.ctypes.data_as(_P), xi.ctypes.data_as(_P)))
        return xt, corr, xi

    def deflate_project_multi(self, defl, Q, eta, variants, thetas=(0, 1, 2, 3, 4)):
        """deflate_project for several (mode, coeffs, xt, corr) variants of
        one noise at once (modes HFES / EIGPOLY; xt updated in place, None:
        a new zero field; corr None: zeros).  Returns [(xt, corr)]."""
        import torch
        th, thp, nth = _thetas(thetas)
        n = eta.shape[0]
        nv = len(variants)
        keep, xts, corrs = [], [], []
        modes = np.array([m for m, _, _, _ in variants], dtype=np.int32)
        cps, ncs = [], []
        for mode, coeffs, xt, corr in variants:
            xts.append(torch.zeros_like(eta) if xt is None else xt)
            cr = np.zeros((nth, self.dims[3]), dtype=np.complex128) if corr is None else \
                np.ascontiguousarray(corr, dtype=np.complex128).copy()
            corrs.append(cr)
            if coeffs is None:
                cps.append(None)
                ncs.append(0)
            else:
                cf = np.ascontiguousarray(coeffs, dtype=np.complex128)
                keep.append(cf)
                cps.append(cf.ctypes.data_as(_P))
                ncs.append(len(cf))
        nc = np.array(ncs, dtype=np.int32)
        _check(lib().deflate_project_multi(self.handle, defl.handle, Q, nv, modes.ctypes.data_as(_P),
                                           (_P * nv)(*cps), nc.ctypes.data_as(_P), thp, nth,
                                           _field(eta, n, 12 * self.V, "eta"),
                                           (_P * nv)(*[_field(x, n, 12 * self.V, "xt") for x in xts]), n,
                                           (_P * nv)(*[c.ctypes.data_as(_P) for c in corrs])))
        del keep
        return list(zip(xts, corrs))

    def poly_subtract_multi(self, eta, coeffs_list):
        """p_a(kappa P) eta for each coefficient list (complex, lowest power
        first; shorter lists pad with zeros) from one chain of powers.
        Returns one new device field per polynomial."""
        import torch
        degree = max(len(c) for c in coeffs_list) - 1
        cf = np.zeros((len(coeffs_list), degree + 1), dtype=np.complex128)
        for a, c in enumerate(coeffs_list):
            cf[a, :len(c)] = c
        n = eta.shape[0]
        outs = [torch.empty_like(eta) for _ in coeffs_list]
        ptrs = (_P * len(outs))(*[_field(o, n, 12 * self.V, "xt") for o in outs])
        _check(lib().poly_subtract_multi(self.handle, len(outs), degree, cf.ctypes.data_as(_P),
                                         _field(eta, n, 12 * self.V, "eta"), ptrs, n))
        return outs

    def loop_estimate(self, eta, x, xt=None, corr=None, thetas=(0, 1, 2, 3, 4), samples=False, noalloc=False):
        """noalloc: call loop_estimate_noalloc (partial sums in the library's
        fixed device scratch instead of a context workspace)."""
        th, thp, nth = _thetas(thetas)
        Lt = self.dims[3]
        nrhs = eta.shape[0]
        est = np.zeros((nth, Lt + 1), dtype=np.complex128)
        err = np.zeros((nth, Lt + 1, 2))
        smp = np.zeros((nrhs, nth, Lt + 1), dtype=np.complex128) if samples else None
        cp = None
        if corr is not None:
            corr = np.ascontiguousarray(corr, dtype=np.complex128)
            cp = corr.ctypes.data_as(_P)
        fv = 12 * self.V
        fn = lib().loop_estimate_noalloc if noalloc else lib().loop_estimate
        _check(fn(self.handle, thp, nth, _field(eta, nrhs, fv, "eta"), _field(x, nrhs, fv, "x"),
                                   None if xt is None else _field(xt, nrhs, fv, "xt"), nrhs, cp,
                                   est.ctypes.data_as(_P), err.ctypes.data_as(_P),
                                   smp.ctypes.data_as(_P) if samples else None))
        return (est, err, smp) if samples else (est, err)

    def loop_estimate_multi(self, eta, x, xts, corrs=None, thetas=(0, 1, 2, 3, 4), samples=False):
        """loop_estimate for several subtracted vectors of one solve at once
        (xts: list of device fields or None; corrs: matching list of trace
        corrections or None).  Returns one (est, err[, samples]) per entry,
        each equal bit for bit to loop_estimate's."""
        th, thp, nth = _thetas(thetas)
        Lt = self.dims[3]
        nrhs = eta.shape[0]
        nv = len(xts)
        fv = 12 * self.V
        ptrs = (_P * nv)(*[None if t is None else _field(t, nrhs, fv, "xt") for t in xts])
        keep = []
        cptrs = None
        if corrs is not None:
            assert len(corrs) == nv, "one trace correction (or None) per subtracted vector"
            cl = []
            for cr in corrs:
                if cr is None:
                    cl.append(None)
                else:
                    a = np.ascontiguousarray(cr, dtype=np.complex128)
                    keep.append(a)
                    cl.append(a.ctypes.data_as(_P))
            cptrs = (_P * nv)(*cl)
        est = np.zeros((nv, nth, Lt + 1), dtype=np.complex128)
        err = np.zeros((nv, nth, Lt + 1, 2))
        smp = np.zeros((nv, nrhs, nth, Lt + 1), dtype=np.complex128) if samples else None
        _check(lib().loop_estimate_multi(self.handle, thp, nth, _field(eta, nrhs, fv, "eta"),
                                         _field(x, nrhs, fv, "x"), ptrs, nv, nrhs, cptrs,
                                         est.ctypes.data_as(_P), err.ctypes.data_as(_P),
                                         smp.ctypes.data_as(_P) if samples else None))
        del keep
        if samples:
            return [(est[v], err[v], smp[v]) for v in range(nv)]
        return [(est[v], err[v]) for v in range(nv)]

    # ------------------------------------------------------ differentiation
    def loop_gradient(self, eta, x=None, thetas=(0,), weights=None, defl=None, links=True, m=20, k=10,
                      tol=1e-10, tol_super=1e-13, eig_tol=0.0, n_eig=0, max_cycles=1000, inner="f64",
                      inner_tol=1e-5, rhs_block=1, proj_m=0):
        """Derivatives of T = (1/N) sum_n eta_n^+ Theta_w M^{-1} eta_n (see
        loop_gradient in lqcd.h).  weights: complex [ntheta][Lt] or None.
        Returns (dT/dkappa complex, dT/dw complex tensor [Lt,Lz,Ly,Lx,4,8] or
        None, deflation space, adjoint-solve statistics)."""
        import torch
        th, thp, nth = _thetas(thetas)
        wp = None
        if weights is not None:
            w = np.ascontiguousarray(np.broadcast_to(np.asarray(weights, dtype=np.complex128),
                                                     (nth, self.dims[3])))
            wp = w.ctypes.data_as(_P)
        nrhs = eta.shape[0]
        p = SolveParams(m, k, max_cycles, tol, tol_super, eig_tol, n_eig, _PREC[inner], inner_tol,
                        rhs_block, proj_m)
        stats = (SolveStats * max(nrhs, 1))()
        dk = np.zeros(1, dtype=np.complex128)
        dl = torch.empty(self.shape[:4] + (4, 8), dtype=torch.complex128, device="cuda") if links else None
        h = _P(defl.handle.value if defl is not None else None)
        fv = 12 * self.V
        code = lib().loop_gradient(self.handle, thp, wp, nth, ctypes.byref(p), ctypes.byref(h),
                                   _field(eta, nrhs, fv, "eta"), None if x is None else _field(x, nrhs, fv, "x"),
                                   nrhs, dk.ctypes.data_as(_P),
                                   None if dl is None else _field(dl, 1, self.V * 32, "dlinks"), stats)
        newdefl = Deflation(_P(h.value), self) if (defl is None and h.value) else defl
        _check(code)
        st = [dict(matvecs=s.matvecs, cycles=s.cycles, refinements=s.refinements, reorth=s.reorth,
                   true_resid=s.true_resid) for s in stats[:nrhs]]
        return complex(dk[0]), dl, newdefl, st


class Batch:
    """Several contexts (lattices) solved together (see batch_solve in lqcd.h)."""

    def __init__(self, contexts):
        self.contexts = list(contexts)
        arr = (_P * len(self.contexts))(*[c.handle.value for c in self.contexts])
        h = _P()
        _check(lib().lqcd_batch_create(arr, len(self.contexts), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().lqcd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, fields):
        """Device pointers of one LEX complex128 field list entry per lattice,
        each checked against its lattice's volume."""
        if len(fields) != len(self.contexts):
            raise ValueError("one field list entry per lattice")
        ptrs = []
        for f, c in zip(fields, self.contexts):
            if f is None or f.numel() == 0:
                ptrs.append(None)
            else:
                ptrs.append(_field(f, f.shape[0], 12 * c.V, "field of lattice %s" % (c.dims,)).value)
        return (_P * len(fields))(*ptrs)

    def set_grid(self, workgroups):
        _check(lib().lqcd_batch_set_grid(self.handle, int(workgroups)))

    def set_tile(self, tile_sites):
        """Batched stencil form: 0 = persistent slot-table launch, 16/32/64 =
        link tiles of that many sites per lattice group."""
        _check(lib().lqcd_batch_set_tile(self.handle, int(tile_sites)))

    def wilson_apply(self, xs):
        """Mhat (FP32) of every field list entry, one launch over all lattices."""
        import torch
        outs = [torch.empty_like(x) for x in xs]
        nr = (_I * len(xs))(*[x.shape[0] for x in xs])
        _check(lib().batch_wilson_apply(self.handle, self._ptrs(xs), self._ptrs(outs), nr))
        return outs

    @staticmethod
    def _params(m, k, tol, max_cycles, inner_tol, rhs_block, proj_m):
        return SolveParams(m, k, max_cycles, tol, tol, 0.0, 0, F32, inner_tol, rhs_block, proj_m)

    def solve(self, bs, defls, m=20, k=10, tol=1e-10, max_cycles=1000, inner_tol=1e-4, rhs_block=8,
              proj_m=0, graph=True):
        """Solve M x = b for every lattice's fields bs[l] ([nrhs_l, ...] LEX
        complex128) with deflation spaces defls[l]; returns (xs, stats)."""
        import torch
        xs = [torch.empty_like(b) for b in bs]
        nr = (_I * len(bs))(*[b.shape[0] for b in bs])
        total = sum(b.shape[0] for b in bs)
        stats = (SolveStats * max(total, 1))()
        p = self._params(m, k, tol, max_cycles, inner_tol, rhs_block, proj_m)
        dp = (_P * len(defls))(*[d.handle.value for d in defls])
        _check(lib().batch_solve(self.handle, ctypes.byref(p), self._ptrs(bs), self._ptrs(xs), nr, dp,
                                 1 if graph else 0, stats))
        st = [dict(matvecs=s.matvecs, cycles=s.cycles, refinements=s.refinements, reorth=s.reorth,
                   true_resid=s.true_resid) for s in stats[:total]]
        return xs, st

    TUNE_BLOCKS = (4, 8, 16, 32)
    TUNE_TILES = (0, 16, 32, 64)

    def autotune(self, bs, defls, m=20, k=10, tol=1e-10, max_cycles=1000, inner_tol=1e-4, proj_m=0):
        """Returns (best rhs_block, best tile, {(rhs_block, tile): rhs/s});
        tile 0 is the persistent slot-table stencil."""
        nr = (_I * len(bs))(*[b.shape[0] for b in bs])
        p = self._params(m, k, tol, max_cycles, inner_tol, 8, proj_m)
        dp = (_P * len(defls))(*[d.handle.value for d in defls])
        bb, bt = _I(0), _I(0)
        nt = len(self.TUNE_TILES)
        rates = np.zeros(len(self.TUNE_BLOCKS) * nt)
        _check(lib().batch_autotune(self.handle, ctypes.byref(p), self._ptrs(bs), nr, dp, ctypes.byref(bb),
                                    ctypes.byref(bt), rates.ctypes.data_as(_P)))
        table = {}
        for i, blk in enumerate(self.TUNE_BLOCKS):
            for j, t in enumerate(self.TUNE_TILES):
                table[(blk, t)] = float(rates[nt * i + j])
        return bb.value, bt.value, table
