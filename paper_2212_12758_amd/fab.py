"""ctypes binding of libfab (include/fab.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libfab.so; this module
only converts Python arguments to the C ABI.  torch supplies device memory
(the arena tensor, b and out) and the stream.  Loading fails loudly when the
built library is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfab.so")

OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, EBUSY, ENOTFOUND, ESCRATCH = range(8)
NOALLOC_SCRATCH_BYTES = 64 << 20
F_EXP, F_POW, F_POLY, F_SIGN = 1, 2, 3, 4
SKETCH_SRHT, SKETCH_SPARSE_SIGN = 1, 2
PREC_FP32, PREC_FP64, PREC_AUTO = 1, 2, 3
LS_AUTO, LS_SKETCH, LS_NONE, LS_LSQR, LS_GRAM = 0, 1, 2, 3, 4
BASIS_TRUNCATED, BASIS_SKETCHED_GS, BASIS_SKETCHED_GS2, BASIS_WHITENED = 0, 1, 2, 3


class fab_func(C.Structure):
    _fields_ = [("kind", C.c_int), ("alpha", C.c_double), ("sigma", C.c_double), ("p", C.c_double),
                ("coef", C.POINTER(C.c_double)), ("ncoef", C.c_int)]


class fab_params(C.Structure):
    _fields_ = [("m", C.c_int), ("k", C.c_int), ("s", C.c_int), ("sketch", C.c_int), ("zeta", C.c_int),
                ("seed", C.c_uint64), ("prec", C.c_int), ("ls_mode", C.c_int), ("tol", C.c_double),
                ("basis", C.c_int), ("ls_maxit", C.c_int)]


class fab_info(C.Structure):
    _fields_ = [("err_est", C.c_double), ("ls_gate", C.c_double), ("round_est", C.c_double),
                ("conv_est", C.c_double), ("kappa_R", C.c_double), ("h_last", C.c_double),
                ("beta", C.c_double), ("m_used", C.c_int), ("breakdown", C.c_int), ("fell_back", C.c_int),
                ("ls_iters", C.c_int), ("prec_used", C.c_int), ("whitened_at", C.c_int),
                ("ls_limit", C.c_int), ("block_rhs", C.c_int), ("latency_us", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class fab_diag(C.Structure):
    _fields_ = [("hbar", C.POINTER(C.c_double)), ("sv", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("c", C.POINTER(C.c_double)), ("eta", C.POINTER(C.c_double))]


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libfab.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2212_12758_amd.build` "
                          "(there is no non-HIP fallback)")
    lib = C.CDLL(path)
    vp, i, u64, sz = C.c_void_p, C.c_int, C.c_uint64, C.c_size_t
    lib.fab_init.argtypes = [C.POINTER(vp), i, vp, sz, vp]
    lib.fab_create_matrix_stencil.argtypes = [vp, i, i, i, i, C.POINTER(C.c_double), C.POINTER(vp)]
    lib.fab_create_matrix_csr.argtypes = [vp, C.c_int64, C.c_int64, vp, vp, vp, i, C.POINTER(vp)]
    lib.fab_destroy_matrix.argtypes = [vp]
    lib.fab_solve.argtypes = [vp, vp, vp, i, fab_func, C.POINTER(fab_params), vp, C.POINTER(fab_info)]
    lib.fab_solve_diag.argtypes = [vp, vp, vp, i, fab_func, C.POINTER(fab_params), vp, C.POINTER(fab_info),
                                   C.POINTER(fab_diag)]
    lib.fab_solve_noalloc.argtypes = [vp, vp, vp, i, fab_func, C.POINTER(fab_params), vp, C.POINTER(fab_info)]
    lib.fab_submit.argtypes = [vp, vp, vp, i, fab_func, C.POINTER(fab_params), vp, C.POINTER(u64)]
    lib.fab_poll.argtypes = [vp, u64, C.POINTER(i), C.POINTER(fab_info)]
    lib.fab_wait.argtypes = [vp, u64, C.POINTER(fab_info)]
    lib.fab_finalize.argtypes = [vp]
    lib.fab_set_block_limit.argtypes = [vp, i]
    lib.fab_hold.argtypes = [vp, i]
    lib.fab_profile_enable.argtypes = [vp, i]
    lib.fab_profile_read.argtypes = [vp, i, C.POINTER(C.c_longlong), C.POINTER(C.c_double), i]
    lib.fab_strerror.argtypes = [i]
    lib.fab_strerror.restype = C.c_char_p
    lib.fab_version.restype = C.c_char_p
    _lib = lib
    return lib


class FabError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        lib = load_library()
        super().__init__(f"{what}: {lib.fab_strerror(code).decode()} (status {code})")


def _check(code: int, what: str):
    if code != OK:
        raise FabError(code, what)


def make_func(f) -> tuple:
    """Duck-typed f (kind 'exp' | 'pow' | 'poly' | 'sign', alpha, sigma, p, coef) -> (fab_func, keepalive)."""
    kind = {"exp": F_EXP, "pow": F_POW, "poly": F_POLY, "sign": F_SIGN}[f.kind]
    coef = tuple(getattr(f, "coef", ()) or ())
    arr = (C.c_double * max(1, len(coef)))(*coef) if coef else None
    ff = fab_func(kind, float(getattr(f, "alpha", 0.0)), float(getattr(f, "sigma", 0.0)),
                  float(getattr(f, "p", 0.0)), C.cast(arr, C.POINTER(C.c_double)) if arr else None, len(coef))
    return ff, arr


def make_params(m, k, s, sketch="srht", zeta=8, seed=0, prec="fp32", ls_mode="sketch", tol=1e-6,
                basis="truncated", ls_maxit=0) -> fab_params:
    sk = {"srht": SKETCH_SRHT, "sparse_sign": SKETCH_SPARSE_SIGN}[sketch] if isinstance(sketch, str) else sketch
    pr = {"fp32": PREC_FP32, "fp64": PREC_FP64, "auto": PREC_AUTO}[prec] if isinstance(prec, str) else prec
    ls = {"auto": LS_AUTO, "sketch": LS_SKETCH, "none": LS_NONE, "lsqr": LS_LSQR, "gram": LS_GRAM}[ls_mode] \
        if isinstance(ls_mode, str) else ls_mode
    bs = {"truncated": BASIS_TRUNCATED, "sketched_gs": BASIS_SKETCHED_GS,
          "sketched_gs2": BASIS_SKETCHED_GS2, "whitened": BASIS_WHITENED}[basis] \
        if isinstance(basis, str) else basis
    return fab_params(int(m), int(k), int(s), sk, int(zeta), int(seed) & ((1 << 64) - 1), pr, ls, float(tol),
                      int(bs), int(ls_maxit))


class Matrix:
    def __init__(self, ctx: "Context", handle, n: int, keep=None):
        self.ctx, self.handle, self.n, self._keep = ctx, handle, n, keep

    def destroy(self):
        if self.handle:
            _check(load_library().fab_destroy_matrix(self.handle), "fab_destroy_matrix")
            self.handle = None


class Context:
    """One libfab context on a CUDA(HIP) device; the arena is a torch uint8 tensor."""

    def __init__(self, device: int = 0, arena_bytes: int = 1 << 30, stream=None):
        import torch

        self.lib = load_library()
        self.device = device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        st = stream if stream is not None else torch.cuda.current_stream(device)
        self._stream = st
        h = C.c_void_p()
        _check(self.lib.fab_init(C.byref(h), device, C.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                 C.c_void_p(st.cuda_stream)), "fab_init")
        self.handle = h

    # ---------------------------------------------------------------- operators
    def stencil(self, st) -> Matrix:
        """A Stencil-like object (dim, nx, ny, nz, coeff[7])."""
        coeff = (C.c_double * 7)(*[float(c) for c in st.coeff])
        h = C.c_void_p()
        _check(self.lib.fab_create_matrix_stencil(self.handle, int(st.dim), int(st.nx), int(st.ny), int(st.nz),
                                                  coeff, C.byref(h)), "fab_create_matrix_stencil")
        return Matrix(self, h, int(st.nx) * int(st.ny) * int(st.nz))

    def csr(self, rowptr, col, val) -> Matrix:
        import numpy as np

        rp = np.ascontiguousarray(rowptr, dtype=np.int32)
        ci = np.ascontiguousarray(col, dtype=np.int32)
        va = np.ascontiguousarray(val, dtype=np.float32)
        h = C.c_void_p()
        n = len(rp) - 1
        _check(self.lib.fab_create_matrix_csr(self.handle, n, len(ci), rp.ctypes.data, ci.ctypes.data,
                                              va.ctypes.data, 0, C.byref(h)), "fab_create_matrix_csr")
        return Matrix(self, h, n)

    def matrix(self, op) -> Matrix:
        return self.stencil(op) if hasattr(op, "coeff") else self.csr(*op)

    # ---------------------------------------------------------------- solves
    @staticmethod
    def _shape(b):
        if b.dim() == 1:
            return 1
        return int(b.shape[1])

    def solve(self, A: Matrix, b, f, params: fab_params, out=None, diag: bool = False):
        """Blocking solve.  b: float64 CUDA tensor [n] or [n, nrhs] (contiguous).
        Returns (out, [info dict per rhs]) or (out, infos, diag dict) with diag=True."""
        import numpy as np
        import torch

        assert b.dtype == torch.float64 and b.is_cuda and b.is_contiguous()
        nrhs = self._shape(b)
        if out is None:
            out = torch.empty_like(b)
        ff, keep = make_func(f)
        infos = (fab_info * nrhs)()
        if not diag:
            rc = self.lib.fab_solve(self.handle, A.handle, C.c_void_p(b.data_ptr()), nrhs, ff, C.byref(params),
                                    C.c_void_p(out.data_ptr()), infos)
            _check(rc, "fab_solve")
            return out, [i.as_dict() for i in infos]
        m, s = params.m, params.s
        bufs = {"hbar": np.zeros((nrhs, m, m + 1)), "sv": np.zeros((nrhs, m + 1, s)), "y": np.zeros((nrhs, m)),
                "c": np.zeros((nrhs, m)), "eta": np.zeros((nrhs, m + 1))}
        dg = fab_diag(*[bufs[k].ctypes.data_as(C.POINTER(C.c_double)) for k in ("hbar", "sv", "y", "c", "eta")])
        rc = self.lib.fab_solve_diag(self.handle, A.handle, C.c_void_p(b.data_ptr()), nrhs, ff, C.byref(params),
                                     C.c_void_p(out.data_ptr()), infos, C.byref(dg))
        _check(rc, "fab_solve_diag")
        d = {"hbar": bufs["hbar"].transpose(0, 2, 1), "sv": bufs["sv"].transpose(0, 2, 1), "y": bufs["y"],
             "c": bufs["c"], "eta": bufs["eta"]}
        if nrhs == 1:
            d = {k: v[0] for k, v in d.items()}
        return out, [i.as_dict() for i in infos], d

    def solve_noalloc(self, A: Matrix, b, f, params: fab_params, out):
        """fab_solve_noalloc: the blocking solve in the library's static device
        scratch (no allocation).  out must be given.  Returns [info dict per rhs]."""
        import torch

        assert b.dtype == torch.float64 and b.is_cuda and b.is_contiguous()
        assert out.dtype == torch.float64 and out.is_cuda and out.shape == b.shape
        nrhs = self._shape(b)
        ff, keep = make_func(f)
        infos = (fab_info * nrhs)()
        rc = self.lib.fab_solve_noalloc(self.handle, A.handle, C.c_void_p(b.data_ptr()), nrhs, ff, C.byref(params),
                                        C.c_void_p(out.data_ptr()), infos)
        _check(rc, "fab_solve_noalloc")
        return [i.as_dict() for i in infos]

    def submit(self, A: Matrix, b, f, params: fab_params, out):
        """Non-blocking; the request runs on a library stream, so pending torch
        work producing b is completed first."""
        self._stream.synchronize()
        ff, keep = make_func(f)
        req = C.c_uint64()
        _check(self.lib.fab_submit(self.handle, A.handle, C.c_void_p(b.data_ptr()), self._shape(b), ff,
                                   C.byref(params), C.c_void_p(out.data_ptr()), C.byref(req)), "fab_submit")
        return Request(self, req.value, self._shape(b), (b, out, keep))

    def set_block_limit(self, max_rhs: int):
        """Largest block of merged single-rhs served requests (1 disables merging)."""
        _check(self.lib.fab_set_block_limit(self.handle, int(max_rhs)), "fab_set_block_limit")

    def hold(self, on: bool = True):
        """Hold (or release) admission of queued served requests."""
        _check(self.lib.fab_hold(self.handle, 1 if on else 0), "fab_hold")

    # ---------------------------------------------------------------- measurement
    K_DOTS, K_UPDATE, K_COMBINE, K_DENSE, K_OTHER = range(5)

    def profile(self, classes=()):
        """Record HIP events around launches of the given kernel classes (blocking solves)."""
        mask = 0
        for c in classes:
            mask |= 1 << c
        _check(self.lib.fab_profile_enable(self.handle, mask), "fab_profile_enable")

    def profile_read(self, cls: int, reset: bool = True):
        """(launches, total_ms) for one kernel class since the last reset."""
        n, t = C.c_longlong(), C.c_double()
        _check(self.lib.fab_profile_read(self.handle, cls, C.byref(n), C.byref(t), int(reset)), "fab_profile_read")
        return n.value, t.value

    def close(self):
        if getattr(self, "handle", None):
            _check(self.lib.fab_finalize(self.handle), "fab_finalize")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Request:
    def __init__(self, ctx: Context, rid: int, nrhs: int, keep):
        self.ctx, self.id, self.nrhs, self._keep = ctx, rid, nrhs, keep
        self.done = False
        self.status = None
        self.info = None

    def poll(self) -> bool:
        if self.done:
            return True
        d = C.c_int(0)
        infos = (fab_info * self.nrhs)()
        rc = self.ctx.lib.fab_poll(self.ctx.handle, self.id, C.byref(d), infos)
        if d.value:
            self.done, self.status, self.info = True, rc, [i.as_dict() for i in infos]
        elif rc != OK:
            raise FabError(rc, "fab_poll")
        return self.done

    def wait(self):
        if not self.done:
            infos = (fab_info * self.nrhs)()
            rc = self.ctx.lib.fab_wait(self.ctx.handle, self.id, infos)
            self.done, self.status, self.info = True, rc, [i.as_dict() for i in infos]
        _check(self.status, "request")
        return self.info
