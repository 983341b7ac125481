"""Python binding of the C-ABI in ``include/tucker.h``.

Argument marshalling only: every step of the computation runs in the HIP
library ``libtucker.so``.  torch supplies device memory (outputs and
workspaces) and the stream (the current torch stream of the tensor's device).

Tensors use the paper's layout: logical shape ``(I_1, ..., I_N)`` with mode 1
fastest in memory (Fortran strides), e.g.
``torch.empty(I_N, ..., I_1, device="cuda").permute(N-1, ..., 0)``.
Factor matrices are FP64 ``I_n x R_n`` tensors with column-major strides.

Importing this module does not need a GPU; calling the compute functions
does.  A missing library raises immediately: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtucker.so")

MAX_NDIM = 8
F64, F32 = 0, 1
GRAM_PRECISIONS = {"fp64": 0, "split_bf16": 1, "qr": 2}
TTM_PRECISIONS = {"fp64": 0, "bf16": 1, "bf16x3": 2}
_TTM_NAMES = {v: k for k, v in TTM_PRECISIONS.items()}
STATUS = {0: "TK_OK", -1: "TK_ERR_INVALID_ARG", -2: "TK_ERR_UNSUPPORTED",
          -3: "TK_ERR_WORKSPACE", -4: "TK_ERR_HIP", -5: "TK_ERR_NONFINITE",
          -6: "TK_ERR_EIG_NO_CONVERGENCE", -7: "TK_ERR_CAPACITY"}

EXPORTS = ("gram_mode_n", "gram_workspace_bytes", "gram_mode_n_noalloc",
           "gram_noalloc_scratch_bytes", "qr_r_mode_n", "qr_workspace_bytes",
           "ttm_mode_n", "sthosvd_compress",
           "sthosvd_workspace_bytes", "tucker_reconstruct", "reconstruct_workspace_bytes",
           "tucker_error_metrics", "error_metrics_workspace_bytes",
           "sthosvd_batch_workspace_bytes", "sthosvd_batch_create", "sthosvd_batch_run",
           "sthosvd_batch_finish", "sthosvd_batch_destroy", "sthosvd_mode_order",
           "tucker_hooi_workspace_bytes", "tucker_hooi", "tk_status_string", "tk_last_error")


class TuckerError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("dims", ctypes.c_int64 * MAX_NDIM)]


class Options(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("mode_order", ctypes.POINTER(ctypes.c_int32)),
                ("fixed_ranks", ctypes.POINTER(ctypes.c_int64)),
                ("max_ranks", ctypes.POINTER(ctypes.c_int64)),
                ("gram_precision", ctypes.c_int32), ("ttm_precision", ctypes.c_int32),
                ("time_first_gram", ctypes.c_int32)]


class Tucker(ctypes.Structure):
    _fields_ = [("core_dev", ctypes.c_void_p), ("core_capacity", ctypes.c_int64),
                ("factors_dev", ctypes.c_void_p * MAX_NDIM), ("eigvals_dev", ctypes.c_void_p),
                ("ranks", ctypes.c_int64 * MAX_NDIM), ("discarded", ctypes.c_double * MAX_NDIM),
                ("norm2", ctypes.c_double), ("fp64_modes", ctypes.c_uint32),
                ("ttm_precision_used", ctypes.c_int32),
                ("tail_error_bound", ctypes.c_double * MAX_NDIM),
                ("first_gram_ms", ctypes.c_double)]


class BatchOutputs(ctypes.Structure):
    _fields_ = [("core_dev", ctypes.POINTER(ctypes.c_void_p)),
                ("core_capacity", ctypes.POINTER(ctypes.c_int64)),
                ("factors_dev", ctypes.POINTER(ctypes.c_void_p)),
                ("ranks_dev", ctypes.c_void_p), ("discarded_dev", ctypes.c_void_p),
                ("norm2_dev", ctypes.c_void_p), ("status_dev", ctypes.c_void_p),
                ("tail_bound_dev", ctypes.c_void_p)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("gram_tiles_per_wg", ctypes.c_int32 * MAX_NDIM),
                ("ttm_blocks_per_wg", ctypes.c_int32 * MAX_NDIM)]


_lib = None
_vp, _sz, _i64, _int = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int
_pshape = ctypes.POINTER(Shape)


def library() -> ctypes.CDLL:
    """Load ``libtucker.so`` (built by ``python -m paper_1510_06689_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1510_06689_amd.build` (no fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "gram_mode_n": (_int, [_pshape, _vp, _int, _int, _vp, _vp, _vp, _sz, _vp]),
        "gram_workspace_bytes": (_sz, [_pshape, _int, _int]),
        "gram_mode_n_noalloc": (_int, [_pshape, _vp, _int, _int, _vp, _vp, _vp]),
        "gram_noalloc_scratch_bytes": (_sz, []),
        "qr_r_mode_n": (_int, [_pshape, _vp, _int, _vp, _vp, _vp, _sz, _vp]),
        "qr_workspace_bytes": (_sz, [_pshape, _int]),
        "ttm_mode_n": (_int, [_pshape, _vp, _int, _vp, _i64, _i64, _int, _int, _vp, _vp]),
        "sthosvd_compress": (_int, [_pshape, _vp, ctypes.POINTER(Options),
                                    ctypes.POINTER(Tucker), _vp, _sz, _vp]),
        "sthosvd_workspace_bytes": (_sz, [_pshape, ctypes.POINTER(Options)]),
        "tucker_reconstruct": (_int, [_pshape, _vp, ctypes.POINTER(_vp),
                                      ctypes.POINTER(_i64), ctypes.POINTER(_i64), _int, _vp,
                                      _vp, _sz, _vp]),
        "reconstruct_workspace_bytes": (_sz, [_pshape, ctypes.POINTER(_i64)]),
        "tucker_error_metrics": (_int, [_pshape, _vp, _vp, ctypes.POINTER(ctypes.c_double),
                                        _vp, _sz, _vp]),
        "error_metrics_workspace_bytes": (_sz, [_pshape]),
        "sthosvd_batch_workspace_bytes": (_sz, [_int, _pshape, ctypes.POINTER(Options),
                                                ctypes.POINTER(BatchTuning)]),
        "sthosvd_batch_create": (_int, [_int, _pshape, ctypes.POINTER(_vp), ctypes.POINTER(Options),
                                        ctypes.POINTER(BatchTuning), ctypes.POINTER(BatchOutputs),
                                        _vp, _sz, _vp, ctypes.POINTER(_vp)]),
        "sthosvd_batch_run": (_int, [_vp, _vp]),
        "sthosvd_batch_finish": (_int, [_vp, _vp]),
        "sthosvd_batch_destroy": (None, [_vp]),
        "tucker_hooi_workspace_bytes": (_sz, [ctypes.POINTER(Shape), ctypes.POINTER(Options)]),
        "tucker_hooi": (_int, [ctypes.POINTER(Shape), _vp, ctypes.POINTER(Options), _int,
                               ctypes.c_double, ctypes.POINTER(Tucker),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), _vp,
                               _sz, _vp]),
        "sthosvd_mode_order": (_int, [_int, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64), _int, _int,
                                      ctypes.POINTER(ctypes.c_int)]),
        "tk_status_string": (ctypes.c_char_p, [_int]),
        "tk_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = library().tk_last_error().decode(errors="replace")
        raise TuckerError(status, msg)


# ------------------------------------------------------------ marshalling

def is_fortran(x: torch.Tensor) -> bool:
    expect = 1
    for d, s in zip(x.shape, x.stride()):
        if d != 1 and s != expect:
            return False
        expect *= d
    return True


def empty_fortran(dims: Sequence[int], dtype, device) -> torch.Tensor:
    n = len(dims)
    return torch.empty(tuple(reversed(list(dims))), dtype=dtype, device=device).permute(
        *reversed(range(n)))


def empty_colmajor(rows: int, cols: int, device, dtype=torch.float64) -> torch.Tensor:
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}; use float64 or float32")


def shape_of(x: torch.Tensor, dims: Optional[Sequence[int]] = None,
             dtype: Optional[int] = None) -> Shape:
    s = Shape()
    dims = list(x.shape) if dims is None else list(dims)
    if not 1 <= len(dims) <= MAX_NDIM:
        raise ValueError(f"ndim must be in [1, {MAX_NDIM}]")
    s.ndim = len(dims)
    s.dtype = _dtype_code(x) if dtype is None else dtype
    for k, d in enumerate(dims):
        s.dims[k] = int(d)
    return s


def _require_device(*ts: torch.Tensor):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("tensors must live on a GPU device")
        if not is_fortran(t):
            raise ValueError("tensors must be densely packed with mode 1 fastest "
                             "(Fortran strides)")


def _stream(dev) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _workspace(nbytes: int, dev) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=dev)
    return ws


def _aligned(ws: torch.Tensor) -> int:
    p = ws.data_ptr()
    return (p + 255) & ~255


# ------------------------------------------------------------------- API

def gram(y: torch.Tensor, mode: int, precision: str = "fp64"):
    """``S = Y_(n) Y_(n)^T`` (FP64, J x J) and ``||Y||^2`` (FP64 scalar tensor)."""
    _require_device(y)
    lib = library()
    sh = shape_of(y)
    prec = GRAM_PRECISIONS[precision]
    need = lib.gram_workspace_bytes(ctypes.byref(sh), mode, prec)
    if need == 0:
        _check(lib.gram_mode_n(ctypes.byref(sh), y.data_ptr(), mode, prec, None, None, None, 0,
                               None))
    j = y.shape[mode]
    s = torch.empty((j, j), dtype=torch.float64, device=y.device)
    sumsq = torch.empty((), dtype=torch.float64, device=y.device)
    ws = _workspace(need, y.device)
    _check(lib.gram_mode_n(ctypes.byref(sh), y.data_ptr(), mode, prec, s.data_ptr(),
                           sumsq.data_ptr(), _aligned(ws), need, _stream(y.device)))
    return s, sumsq


def gram_noalloc(y: torch.Tensor, mode: int, precision: str = "fp64", out=None, sumsq=None):
    """``gram`` through the allocation-free entry point: the library's static
    per-device scratch instead of a workspace.  ``out`` (J x J FP64) and
    ``sumsq`` (FP64 scalar) may be given, so that nothing is allocated here
    either; ``sumsq`` is then only written when given."""
    _require_device(y)
    j = y.shape[mode]
    s = torch.empty((j, j), dtype=torch.float64, device=y.device) if out is None else out
    if out is None and sumsq is None:
        sumsq = torch.empty((), dtype=torch.float64, device=y.device)
    _check(library().gram_mode_n_noalloc(ctypes.byref(shape_of(y)), y.data_ptr(), mode,
                                         GRAM_PRECISIONS[precision], s.data_ptr(),
                                         None if sumsq is None else sumsq.data_ptr(),
                                         _stream(y.device)))
    return s, sumsq


def qr_r(y: torch.Tensor, mode: int):
    """R factor (FP64 J x J, column-major, upper triangular, diagonal >= 0) of
    a Householder QR of ``Y_(n)^T`` (Sec. IX) and ``||Y||^2``."""
    _require_device(y)
    lib = library()
    sh = shape_of(y)
    need = lib.qr_workspace_bytes(ctypes.byref(sh), mode)
    if need == 0:
        _check(lib.qr_r_mode_n(ctypes.byref(sh), y.data_ptr(), mode, None, None, None, 0, None))
    j = y.shape[mode]
    r = empty_colmajor(j, j, y.device)
    sumsq = torch.empty((), dtype=torch.float64, device=y.device)
    ws = _workspace(need, y.device)
    _check(lib.qr_r_mode_n(ctypes.byref(sh), y.data_ptr(), mode, r.data_ptr(), sumsq.data_ptr(),
                           _aligned(ws), need, _stream(y.device)))
    return r, sumsq


def ttm(y: torch.Tensor, mode: int, m: torch.Tensor, transpose: bool = True,
        precision: str = "fp64") -> torch.Tensor:
    """``Z = Y x_n op(M)``; ``op(M) = M^T`` when ``transpose`` (M is J_n x K),
    else ``M`` (K x J_n).  M is FP64 and column-major."""
    _require_device(y)
    if m.dtype != torch.float64 or m.dim() != 2 or not is_fortran(m):
        raise ValueError("M must be a column-major FP64 matrix")
    lib = library()
    sh = shape_of(y)
    rows, cols = m.shape
    k = cols if transpose else rows
    zd = list(y.shape)
    zd[mode] = k
    z = empty_fortran(zd, y.dtype, y.device)
    _check(lib.ttm_mode_n(ctypes.byref(sh), y.data_ptr(), mode, m.data_ptr(), rows, cols,
                          int(transpose), TTM_PRECISIONS[precision], z.data_ptr(),
                          _stream(y.device)))
    return z


@dataclass
class TuckerTensor:
    core: torch.Tensor            # dims = ranks, same dtype as the input
    factors: list                 # U_n: FP64 I_n x R_n, column-major
    ranks: tuple
    eigvals: list                 # per-mode Gram spectra (FP64, descending)
    discarded: tuple              # discarded eigenvalue mass per mode
    norm2: float                  # ||X||^2
    fp64_modes: tuple = ()        # modes whose split-bf16 Gram was redone in FP64
    ttm_precision: str = "fp64"   # arithmetic the TTMs actually ran in
    tail_error_bound: tuple = ()  # per mode: bound on |discarded - exact tail sum|

    @property
    def full_dims(self):
        return tuple(int(u.shape[0]) for u in self.factors)


def _options(ndim, eps, order, ranks, max_ranks, gram_precision, ttm_precision, keep):
    opt = Options()
    opt.eps = float(eps)
    if order is not None:
        a = (ctypes.c_int32 * ndim)(*[int(v) for v in order])
        keep.append(a)
        opt.mode_order = ctypes.cast(a, ctypes.POINTER(ctypes.c_int32))
    if ranks is not None:
        a = (ctypes.c_int64 * ndim)(*[int(v) for v in ranks])
        keep.append(a)
        opt.fixed_ranks = ctypes.cast(a, ctypes.POINTER(ctypes.c_int64))
    if max_ranks is not None:
        a = (ctypes.c_int64 * ndim)(*[int(v) for v in max_ranks])
        keep.append(a)
        opt.max_ranks = ctypes.cast(a, ctypes.POINTER(ctypes.c_int64))
    opt.gram_precision = GRAM_PRECISIONS[gram_precision]
    opt.ttm_precision = TTM_PRECISIONS[ttm_precision]
    return opt


class Compressor:
    """ST-HOSVD (Alg. 1) with preallocated outputs and workspace, reusable
    across calls on tensors of the same shape (the benchmark's timed step)."""

    def __init__(self, dims: Sequence[int], dtype, device, eps: float, order=None, ranks=None,
                 max_ranks=None, gram_precision: str = "fp64", ttm_precision: str = "fp64"):
        self.dims = tuple(int(d) for d in dims)
        self.dtype = dtype
        self.device = torch.device(device)
        n = len(self.dims)
        self._keep = []
        self.opt = _options(n, eps, order, ranks, max_ranks, gram_precision, ttm_precision,
                            self._keep)
        probe = torch.empty(0, dtype=dtype)
        self.shape = shape_of(probe, self.dims, _dtype_code(probe))
        lib = library()
        need = lib.sthosvd_workspace_bytes(ctypes.byref(self.shape), ctypes.byref(self.opt))
        if need == 0:  # invalid arguments: let the entry point report why
            _check(lib.sthosvd_compress(ctypes.byref(self.shape), None, ctypes.byref(self.opt),
                                        None, None, 0, None))
        self.ws_bytes = need
        self.ws = _workspace(need, self.device)
        caps = [min(d, int(max_ranks[k])) if max_ranks is not None else d
                for k, d in enumerate(self.dims)]
        if ranks is not None:
            caps = [int(r) for r in ranks]
        self.core_capacity = math.prod(caps)
        self.core_buf = torch.empty(self.core_capacity, dtype=dtype, device=self.device)
        self.factor_bufs = [torch.empty(d * d, dtype=torch.float64, device=self.device)
                            for d in self.dims]
        self.eig_buf = torch.empty(sum(self.dims), dtype=torch.float64, device=self.device)
        self.out = Tucker()
        self.out.core_dev = self.core_buf.data_ptr()
        self.out.core_capacity = self.core_capacity
        for k, f in enumerate(self.factor_bufs):
            self.out.factors_dev[k] = f.data_ptr()
        self.out.eigvals_dev = self.eig_buf.data_ptr()

    def run(self, x: torch.Tensor, time_first_gram: bool = False) -> float:
        """One ST-HOSVD of ``x``; synchronises the current stream.  With
        ``time_first_gram`` returns the duration (ms) of the first processed
        mode's partial-Gram kernel, timed with HIP events inside the call;
        else 0."""
        if tuple(x.shape) != self.dims or x.dtype != self.dtype:
            raise ValueError("tensor does not match the compressor's shape/dtype")
        _require_device(x)
        self.opt.time_first_gram = 1 if time_first_gram else 0
        _check(library().sthosvd_compress(ctypes.byref(self.shape), x.data_ptr(),
                                          ctypes.byref(self.opt), ctypes.byref(self.out),
                                          _aligned(self.ws), self.ws_bytes,
                                          _stream(self.device)))
        return float(self.out.first_gram_ms)

    def run_hooi(self, x: torch.Tensor, max_sweeps: int = 20, tol: float = 0.0) -> list:
        """Alg. 2 (HOOI) of ``x`` from this compressor's ST-HOSVD settings;
        returns the fits ||X||^2 - ||G||^2 after the ST-HOSVD and after each
        sweep (``result()`` then holds the HOOI core and factors)."""
        if tuple(x.shape) != self.dims or x.dtype != self.dtype:
            raise ValueError("tensor does not match the compressor's shape/dtype")
        _require_device(x)
        lib = library()
        need = lib.tucker_hooi_workspace_bytes(ctypes.byref(self.shape), ctypes.byref(self.opt))
        fits = (ctypes.c_double * (max_sweeps + 1))()
        done = ctypes.c_int(0)
        if need == 0:  # unsupported options: let the entry point report why
            _check(lib.tucker_hooi(ctypes.byref(self.shape), x.data_ptr(), ctypes.byref(self.opt),
                                   int(max_sweeps), float(tol), ctypes.byref(self.out), fits,
                                   ctypes.byref(done), None, 0, _stream(self.device)))
        if getattr(self, "hooi_ws_bytes", 0) < need:
            self.hooi_ws = _workspace(need, self.device)
            self.hooi_ws_bytes = need
        _check(lib.tucker_hooi(ctypes.byref(self.shape), x.data_ptr(), ctypes.byref(self.opt),
                               int(max_sweeps), float(tol), ctypes.byref(self.out), fits,
                               ctypes.byref(done), _aligned(self.hooi_ws), self.hooi_ws_bytes,
                               _stream(self.device)))
        return [float(fits[k]) for k in range(done.value + 1)]

    def result(self, copy: bool = False) -> TuckerTensor:
        """The last run's outputs: views into this compressor's buffers (valid
        until its next run, and keeping those buffers alive), or with ``copy``
        compact copies that hold only the ``prod R_n`` core elements."""
        if copy:
            r = self.result()
            return TuckerTensor(_fortran_copy(r.core), [_fortran_copy(f) for f in r.factors],
                                r.ranks, [e.clone() for e in r.eigvals], r.discarded, r.norm2,
                                r.fp64_modes, r.ttm_precision, r.tail_error_bound)
        n = len(self.dims)
        ranks = tuple(int(self.out.ranks[k]) for k in range(n))
        core = self.core_buf[:math.prod(ranks)].view(tuple(reversed(ranks))).permute(
            *reversed(range(n)))
        factors = [self.factor_bufs[k][:self.dims[k] * ranks[k]].view(ranks[k], self.dims[k]).t()
                   for k in range(n)]
        eig, off = [], 0
        for d in self.dims:
            eig.append(self.eig_buf[off:off + d])
            off += d
        return TuckerTensor(core, factors, ranks, eig,
                            tuple(float(self.out.discarded[k]) for k in range(n)),
                            float(self.out.norm2),
                            tuple(k for k in range(n) if self.out.fp64_modes >> k & 1),
                            _TTM_NAMES[int(self.out.ttm_precision_used)],
                            tuple(float(self.out.tail_error_bound[k]) for k in range(n)))


def sthosvd(x: torch.Tensor, eps: float, order=None, ranks=None, max_ranks=None,
            gram_precision: str = "fp64", ttm_precision: str = "fp64") -> TuckerTensor:
    """Alg. 1 (ST-HOSVD) of ``x`` on its GPU.  Returns copies of the outputs."""
    c = Compressor(x.shape, x.dtype, x.device, eps, order, ranks, max_ranks, gram_precision,
                   ttm_precision)
    c.run(x)
    return c.result(copy=True)


def hooi(x: torch.Tensor, eps: float, order=None, ranks=None, max_ranks=None,
         max_sweeps: int = 20, tol: float = 0.0, gram_precision: str = "fp64",
         ttm_precision: str = "fp64"):
    """Alg. 2 (HOOI) of ``x`` on its GPU, starting from ST-HOSVD.  Returns
    ``(TuckerTensor, fits)`` with copies of the outputs; ``fits[0]`` is the
    ST-HOSVD's ||X||^2 - ||G||^2 and ``fits[k]`` that after sweep k."""
    c = Compressor(x.shape, x.dtype, x.device, eps, order, ranks, max_ranks, gram_precision,
                   ttm_precision)
    fits = c.run_hooi(x, max_sweeps, tol)
    return c.result(copy=True), fits


def _fortran_copy(t: torch.Tensor) -> torch.Tensor:
    out = empty_fortran(t.shape, t.dtype, t.device)
    out.copy_(t)
    return out


def reconstruct(core: torch.Tensor, factors: Sequence[torch.Tensor], full_dims=None,
                precision: str = "fp64") -> torch.Tensor:
    """``X~ = G x_1 U_1 ... x_N U_N`` (Sec. II-C).  A factor may be a row
    subset (any FP64 column-major view), which yields the matching subtensor."""
    _require_device(core)
    n = core.dim()
    if len(factors) != n:
        raise ValueError("one factor per mode")
    lds = []
    for k, u in enumerate(factors):
        if u.dtype != torch.float64 or u.dim() != 2 or u.stride(0) != 1 or u.shape[1] != \
                core.shape[k]:
            raise ValueError(f"factor {k} must be a column-major FP64 I_n x R_n matrix")
        lds.append(max(u.stride(1), u.shape[0]) if u.shape[1] > 1 else u.shape[0])
    full = [int(u.shape[0]) for u in factors] if full_dims is None else list(full_dims)
    lib = library()
    sh = shape_of(core)
    fd = (ctypes.c_int64 * n)(*full)
    ld = (ctypes.c_int64 * n)(*lds)
    ptrs = (ctypes.c_void_p * n)(*[u.data_ptr() for u in factors])
    need = lib.reconstruct_workspace_bytes(ctypes.byref(sh), fd)
    ws = _workspace(need, core.device)
    out = empty_fortran(full, core.dtype, core.device)
    _check(lib.tucker_reconstruct(ctypes.byref(sh), core.data_ptr(), ptrs, ld, fd,
                                  TTM_PRECISIONS[precision], out.data_ptr(), _aligned(ws), need,
                                  _stream(core.device)))
    return out


def error_metrics(x: torch.Tensor, xhat: torch.Tensor):
    """``(||X - X~||^2, max|X - X~|, ||X||^2)`` accumulated in FP64."""
    _require_device(x, xhat)
    if x.shape != xhat.shape or x.dtype != xhat.dtype:
        raise ValueError("x and xhat must match in shape and dtype")
    lib = library()
    sh = shape_of(x)
    need = lib.error_metrics_workspace_bytes(ctypes.byref(sh))
    ws = _workspace(need, x.device)
    out = (ctypes.c_double * 3)()
    _check(lib.tucker_error_metrics(ctypes.byref(sh), x.data_ptr(), xhat.data_ptr(), out,
                                    _aligned(ws), need, _stream(x.device)))
    return float(out[0]), float(out[1]), float(out[2])


ORDER_RULES = {"flops": 0, "ratio": 1, "bytes": 2}


def mode_order(dims, ranks, rule: str = "bytes", elem_bytes: int = 4) -> tuple:
    """A mode order for Alg. 1 from the extents and (expected) ranks: the
    greedy least-flops heuristic (``"flops"``), the greedy largest I_n/R_n
    heuristic (``"ratio"``), both named in Sec. VIII-C's mode-order
    experiment, or the order with the least algorithmic HBM traffic of this
    library (``"bytes"``, exhaustive).  Host-only; no GPU needed."""
    n = len(dims)
    d = (ctypes.c_int64 * n)(*[int(v) for v in dims])
    r = (ctypes.c_int64 * n)(*[int(v) for v in ranks])
    out = (ctypes.c_int * n)()
    _check(library().sthosvd_mode_order(n, d, r, ORDER_RULES[rule], int(elem_bytes), out))
    return tuple(int(v) for v in out)


class BatchCompressor:
    """ST-HOSVD of many independent FP32 tensors in one launch sequence per
    mode step (the batched C-ABI).  ``run()`` only enqueues work and may be
    captured into a HIP graph (``capture()``); ranks the split Gram cannot
    certify are recomputed in FP64 within the run.  ``finish()`` synchronises
    and raises on capacity or non-finite errors."""

    def __init__(self, xs, eps: float, order=None, ranks=None, max_ranks=None,
                 ttm_precision: str = "bf16x3", tuning=None):
        lib = library()
        self.xs = list(xs)
        if not self.xs:
            raise ValueError("empty batch")
        for x in self.xs:
            _require_device(x)
        dev = self.xs[0].device
        self.device = dev
        b = len(self.xs)
        n = self.xs[0].dim()
        self.ndim = n
        self._keep = []
        self.opt = _options(n, eps, order, ranks, max_ranks, "split_bf16", ttm_precision,
                            self._keep)
        self.shapes = (Shape * b)()
        for i, x in enumerate(self.xs):
            self.shapes[i] = shape_of(x)
        self.tuning = BatchTuning()
        if tuning is not None:
            g, t = tuning
            for k in range(min(len(g), MAX_NDIM)):
                self.tuning.gram_tiles_per_wg[k] = int(g[k])
            for k in range(min(len(t), MAX_NDIM)):
                self.tuning.ttm_blocks_per_wg[k] = int(t[k])
        need = lib.sthosvd_batch_workspace_bytes(b, self.shapes, ctypes.byref(self.opt),
                                                 ctypes.byref(self.tuning))
        if need == 0:
            h = _vp()
            _check(lib.sthosvd_batch_create(b, self.shapes, None, ctypes.byref(self.opt), None,
                                            None, None, 0, None, ctypes.byref(h)))
        self.dims = [tuple(int(d) for d in x.shape) for x in self.xs]
        caps = []
        for d in self.dims:
            c = list(d)
            if max_ranks is not None:
                c = [min(ci, int(m)) for ci, m in zip(c, max_ranks)]
            if ranks is not None:
                c = [min(ci, int(r)) for ci, r in zip(c, ranks)]
            caps.append(c)
        self.core_bufs = [torch.empty(math.prod(c), dtype=torch.float32, device=dev) for c in caps]
        self.factor_bufs = [[torch.empty(di * di, dtype=torch.float64, device=dev) for di in d]
                            for d in self.dims]
        self.ranks_dev = torch.zeros(b * n, dtype=torch.int64, device=dev)
        self.disc_dev = torch.zeros(b * n, dtype=torch.float64, device=dev)
        self.norm2_dev = torch.zeros(b, dtype=torch.float64, device=dev)
        self.status_dev = torch.zeros(2 * b, dtype=torch.int32, device=dev)
        self.bound_dev = torch.zeros(b * n, dtype=torch.float64, device=dev)
        self._cores = (_vp * b)(*[t.data_ptr() for t in self.core_bufs])
        self._caps = (_i64 * b)(*[t.numel() for t in self.core_bufs])
        facs = (_vp * (b * MAX_NDIM))()
        for i, fl in enumerate(self.factor_bufs):
            for k, f in enumerate(fl):
                facs[i * MAX_NDIM + k] = f.data_ptr()
        self._facs = facs
        self.outs = BatchOutputs(self._cores, self._caps, self._facs, self.ranks_dev.data_ptr(),
                                 self.disc_dev.data_ptr(), self.norm2_dev.data_ptr(),
                                 self.status_dev.data_ptr(), self.bound_dev.data_ptr())
        self.ws = _workspace(need, dev)
        xp = (_vp * b)(*[x.data_ptr() for x in self.xs])
        self._xp = xp
        h = _vp()
        _check(lib.sthosvd_batch_create(b, self.shapes, xp, ctypes.byref(self.opt),
                                        ctypes.byref(self.tuning), ctypes.byref(self.outs),
                                        _aligned(self.ws), need, _stream(dev), ctypes.byref(h)))
        self.handle = h
        self.graph = None

    def run(self, stream=None) -> None:
        s = _stream(self.device) if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(library().sthosvd_batch_run(self.handle, s))

    def capture(self):
        """Capture one run() into a HIP graph (torch.cuda.CUDAGraph) for replay()."""
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self.run(stream=s)          # warm-up outside the capture
        torch.cuda.current_stream(self.device).wait_stream(s)
        torch.cuda.synchronize(self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.run(stream=s)
        self.graph = g
        return g

    def replay(self) -> None:
        self.graph.replay()

    def finish(self) -> None:
        _check(library().sthosvd_batch_finish(self.handle, _stream(self.device)))

    def results(self):
        n = self.ndim
        ranks = self.ranks_dev.view(-1, n).cpu().tolist()
        disc = self.disc_dev.view(-1, n).cpu().tolist()
        norm2 = self.norm2_dev.cpu().tolist()
        status = self.status_dev.view(-1, 2).cpu().tolist()
        bounds = self.bound_dev.view(-1, n).cpu().tolist()
        out = []
        for i, d in enumerate(self.dims):
            r = tuple(int(v) for v in ranks[i])
            core = self.core_bufs[i][:math.prod(r)].view(tuple(reversed(r))).permute(
                *reversed(range(n)))
            facs = [self.factor_bufs[i][k][:d[k] * r[k]].view(r[k], d[k]).t() for k in range(n)]
            out.append(TuckerTensor(core, facs, r, [], tuple(disc[i]), float(norm2[i]),
                                    tuple(k for k in range(n) if status[i][1] >> k & 1),
                                    _TTM_NAMES[int(self.opt.ttm_precision)],
                                    tuple(bounds[i])))
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                library().sthosvd_batch_destroy(h)
            except Exception:
                pass
            self.handle = None


_lib_id = None


def _library_id() -> str:
    """sha256 of the library file: tunings are kept per build."""
    global _lib_id
    if _lib_id is None:
        try:
            with open(LIB_PATH, "rb") as f:
                _lib_id = hashlib.sha256(f.read()).hexdigest()
        except OSError:
            _lib_id = "missing"
    return _lib_id


def batch_tuning_key(shapes, dtype, eps, options, candidates_gram, candidates_ttm,
                     device_name, library_id) -> str:
    """Cache key of a batch tuning: everything the search depends on."""
    blob = json.dumps({"shapes": [list(map(int, sh)) for sh in shapes], "dtype": str(dtype),
                       "eps": float(eps), "options": options,
                       "candidates": [list(candidates_gram), list(candidates_ttm)],
                       "device": device_name, "library": library_id}, sort_keys=True)
    return hashlib.sha256(blob.encode()).hexdigest()


def load_batch_tuning(path: str, key: str):
    """(gram_tiles_per_wg, ttm_blocks_per_wg, ms) stored under key, or None."""
    try:
        with open(path) as f:
            rec = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    return list(rec["gram"]), list(rec["ttm"]), float(rec["ms"])


def store_batch_tuning(path: str, key: str, gram, ttm, ms: float) -> None:
    """Adds key -> tuning to the JSON file at path (written whole, then renamed)."""
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        table = {}
    table[key] = {"gram": [int(v) for v in gram], "ttm": [int(v) for v in ttm], "ms": float(ms)}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune_batch(xs, eps, candidates_gram=(8, 16, 32, 64), candidates_ttm=(16, 64, 256),
                   reps: int = 5, cache: Optional[str] = None, info: Optional[dict] = None,
                   **kw):
    """Project autotuner for the batched path: per mode step, picks the Gram
    tiles-per-workgroup and TTM blocks-per-workgroup that minimise the time of
    a whole batch run (coordinate search, graph replays timed with events).
    Returns (gram_tiles_per_wg, ttm_blocks_per_wg, ms) for BatchCompressor.
    ``cache``: a JSON file of earlier results, keyed by the problems' shapes,
    dtype, eps, options, candidate sets, device and library build; a hit
    returns the stored tuning without timing anything.  ``info`` (a dict), if
    given, receives ``cache_hit`` and ``key``."""
    n = xs[0].dim()
    key = None
    if cache is not None:
        dev = xs[0].device
        name = torch.cuda.get_device_name(dev) if dev.type == "cuda" else str(dev)
        options = {k: (list(v) if isinstance(v, (list, tuple)) else v) for k, v in kw.items()}
        key = batch_tuning_key([x.shape for x in xs], xs[0].dtype, eps, options,
                               candidates_gram, candidates_ttm, name, _library_id())
        hit = load_batch_tuning(cache, key)
        if info is not None:
            info.update(cache_hit=hit is not None, key=key)
        if hit is not None:
            return hit
    g = [16] * n
    t = [64] * n

    def timed(gv, tv):
        c = BatchCompressor(xs, eps, tuning=(gv, tv), **kw)
        c.capture()
        c.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            c.replay()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    best = timed(g, t)
    for s in range(n):
        for cand in candidates_gram:
            if cand == g[s]:
                continue
            trial = list(g)
            trial[s] = cand
            ms = timed(trial, t)
            if ms < best:
                best, g = ms, trial
        for cand in candidates_ttm:
            if cand == t[s]:
                continue
            trial = list(t)
            trial[s] = cand
            ms = timed(g, trial)
            if ms < best:
                best, t = ms, trial
    if cache is not None:
        store_batch_tuning(cache, key, g, t, best)
    return g, t, best
