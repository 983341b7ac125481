"""FP64 CPU oracle for ST-HOSVD -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product library never calls it
and the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, FP64, no BLAS).  This module
only marshals numpy arrays across ``ctypes``.  Tensors are numpy arrays of
logical shape ``(I_1..I_N)`` stored with mode 1 fastest (Fortran order), the
layout of Sec. IV-A; matrices are ordinary 2-D numpy arrays.

Readings of the paper that the oracle adopts (where it is silent or garbled):

* unfolding column index uses prefix products of the other modes (Sec. II-A
  formula read through the unfolding figure of Sec. IV-C);
* TTM multiplies by a ``K x I_n`` matrix, ``Y_(n) = V X_(n)`` (Sec. II-A);
* the rank threshold ``eps^2 ||X||^2 / N`` uses the original tensor's norm and
  the full mode count for every mode (Alg. 1);
* ``R_n >= 1`` always; negative rounding eigenvalues count as 0 in tail sums;
  tail sums run from the smallest eigenvalue up; eigenvalue ties keep index
  order; each eigenvector's largest-magnitude entry is positive.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (plain -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"],
                       check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_norm2.restype = ctypes.c_double
        lib.orc_norm2.argtypes = [_d, ctypes.c_int64]
        for name in ("orc_unfold", "orc_fold"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [_d, ctypes.c_int, _i64, ctypes.c_int, _d]
        lib.orc_ttm.restype = ctypes.c_int
        lib.orc_ttm.argtypes = [_d, ctypes.c_int, _i64, ctypes.c_int, _d, ctypes.c_int64, _d]
        lib.orc_gram.restype = ctypes.c_int
        lib.orc_gram.argtypes = [_d, ctypes.c_int, _i64, ctypes.c_int, _d]
        lib.orc_gram_matrix.restype = ctypes.c_int
        lib.orc_gram_matrix.argtypes = [_d, ctypes.c_int64, ctypes.c_int64, _d]
        lib.orc_gram_entry.restype = ctypes.c_double
        lib.orc_gram_entry.argtypes = [_d, ctypes.c_int, _i64, ctypes.c_int, ctypes.c_int64,
                                       ctypes.c_int64]
        lib.orc_ttm_entry.restype = ctypes.c_double
        lib.orc_ttm_entry.argtypes = [_d, ctypes.c_int, _i64, ctypes.c_int, _d, _i64]
        lib.orc_sym_eig.restype = ctypes.c_int
        lib.orc_sym_eig.argtypes = [_d, ctypes.c_int64, _d, _d, ctypes.c_int]
        lib.orc_qr_r.restype = ctypes.c_int
        lib.orc_qr_r.argtypes = [_d, ctypes.c_int64, ctypes.c_int64, _d]
        lib.orc_svd_jacobi.restype = ctypes.c_int
        lib.orc_svd_jacobi.argtypes = [_d, ctypes.c_int64, _d, _d, ctypes.c_int]
        lib.orc_truncate.restype = ctypes.c_int
        lib.orc_truncate.argtypes = [_d, ctypes.c_int64, ctypes.c_double, ctypes.c_int64, _i64,
                                     _d]
        lib.orc_sthosvd.restype = ctypes.c_int
        lib.orc_sthosvd.argtypes = [_d, ctypes.c_int, _i64, ctypes.c_double, _i32, _i64, _d,
                                    _i64, _d, _d, _d, _d, _i32]
        lib.orc_reconstruct.restype = ctypes.c_int
        lib.orc_reconstruct.argtypes = [_d, ctypes.c_int, _i64, _d, _i64, _d]
        lib.orc_error_metrics.restype = ctypes.c_int
        lib.orc_error_metrics.argtypes = [_d, _d, ctypes.c_int64, _d]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_d)


def _f64_fortran(x) -> np.ndarray:
    return np.asfortranarray(np.asarray(x, dtype=np.float64))


def _flat(x: np.ndarray) -> np.ndarray:
    """Memory-order (mode-1-fastest) 1-D view of a Fortran-ordered array."""
    return x.reshape(-1, order="F")


def _dims(x: np.ndarray):
    return (ctypes.c_int64 * x.ndim)(*x.shape)


def _check(rc: int, what: str):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")
    return rc


def norm2(x) -> float:
    """||X||^2, pairwise summed in FP64."""
    x = _f64_fortran(x)
    f = _flat(x)
    return _load().orc_norm2(_p(f), f.size)


def unfold(x, n: int) -> np.ndarray:
    """Explicit mode-n unfolding (0-based ``n``), an ``I_n x (I/I_n)`` matrix."""
    x = _f64_fortran(x)
    m = np.empty((x.shape[n], x.size // x.shape[n]), dtype=np.float64)
    _check(_load().orc_unfold(_p(_flat(x)), x.ndim, _dims(x), n, _p(m)), "unfold")
    return m


def fold(m, n: int, dims) -> np.ndarray:
    """Inverse of :func:`unfold`."""
    m = np.ascontiguousarray(m, dtype=np.float64)
    dims = tuple(int(d) for d in dims)
    out = np.empty(int(np.prod(dims)), dtype=np.float64)
    cd = (ctypes.c_int64 * len(dims))(*dims)
    _check(_load().orc_fold(_p(m), len(dims), cd, n, _p(out)), "fold")
    return out.reshape(dims, order="F")


def ttm(y, n: int, v) -> np.ndarray:
    """``Y x_n V`` for a ``K x I_n`` matrix ``V`` (Sec. II-A)."""
    y = _f64_fortran(y)
    v = np.ascontiguousarray(v, dtype=np.float64)
    k = v.shape[0]
    if v.shape[1] != y.shape[n]:
        raise ValueError("V must be K x I_n")
    zd = list(y.shape)
    zd[n] = k
    z = np.empty(int(np.prod(zd)), dtype=np.float64)
    _check(_load().orc_ttm(_p(_flat(y)), y.ndim, _dims(y), n, _p(v), k, _p(z)), "ttm")
    return z.reshape(zd, order="F")


def gram(y, n: int) -> np.ndarray:
    """``S = Y_(n) Y_(n)^T`` via the explicit unfolding, pairwise sums."""
    y = _f64_fortran(y)
    s = np.empty((y.shape[n], y.shape[n]), dtype=np.float64)
    _check(_load().orc_gram(_p(_flat(y)), y.ndim, _dims(y), n, _p(s)), "gram")
    return s


def gram_of_matrix(m) -> np.ndarray:
    m = np.ascontiguousarray(m, dtype=np.float64)
    s = np.empty((m.shape[0], m.shape[0]), dtype=np.float64)
    _check(_load().orc_gram_matrix(_p(m), m.shape[0], m.shape[1], _p(s)), "gram_matrix")
    return s


def gram_entry(y, n: int, a: int, b: int) -> float:
    """One entry ``S[a, b]`` of the mode-n Gram, straight from the definition."""
    y = _f64_fortran(y)
    return _load().orc_gram_entry(_p(_flat(y)), y.ndim, _dims(y), n, a, b)


def ttm_entry(y, n: int, v, out_idx) -> float:
    """One entry of ``Y x_n V`` at multi-index ``out_idx`` (0-based)."""
    y = _f64_fortran(y)
    v = np.ascontiguousarray(v, dtype=np.float64)
    idx = (ctypes.c_int64 * y.ndim)(*[int(i) for i in out_idx])
    return _load().orc_ttm_entry(_p(_flat(y)), y.ndim, _dims(y), n, _p(v), idx)


def sym_eig(s, max_sweeps: int = 50):
    """Jacobi eigendecomposition: ``(lam_desc, V, sweeps)``; columns of V are
    eigenvectors, sign-normalised (largest |entry| positive)."""
    a = np.array(s, dtype=np.float64, order="C", copy=True)
    j = a.shape[0]
    lam = np.empty(j)
    v = np.empty((j, j))
    sw = _load().orc_sym_eig(_p(a), j, _p(lam), _p(v), max_sweeps)
    _check(sw, "sym_eig")
    return lam, v, sw


def qr_r(a) -> np.ndarray:
    """R factor (``j x j``, diagonal >= 0, strict lower part zero) of a
    Householder QR of the ``m x j`` matrix ``a`` (Sec. IX)."""
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    m, j = a.shape
    r = np.empty((j, j))
    _check(_load().orc_qr_r(_p(a), m, j, _p(r)), "qr_r")
    return r


def svd_jacobi(b, max_sweeps: int = 60):
    """One-sided Jacobi SVD of a square matrix: ``(sigma_desc, V, sweeps)``;
    the columns of V are right singular vectors, sign-normalised (largest
    |entry| positive)."""
    b = np.array(b, dtype=np.float64, order="C", copy=True)
    j = b.shape[0]
    sig = np.empty(j)
    v = np.empty((j, j))
    sw = _load().orc_svd_jacobi(_p(b), j, _p(sig), _p(v), max_sweeps)
    _check(sw, "svd_jacobi")
    return sig, v, sw


def mode_svd_qr(y, n: int):
    """Leading left singular pairs of ``Y_(n)`` through the QR of
    ``Y_(n)^T`` (Sec. IX): ``(lambda_desc, U, sweeps)`` with
    ``lambda_r = sigma_r^2`` and U the right singular vectors of R."""
    a = np.ascontiguousarray(unfold(y, n).T)
    sig, v, sw = svd_jacobi(qr_r(a))
    return sig * sig, v, sw


def truncate(lam, tau: float, fixed_rank: int = 0):
    """Rank rule of Alg. 1 -> ``(R, discarded_tail_sum)``."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    r = ctypes.c_int64()
    t = ctypes.c_double()
    _check(_load().orc_truncate(_p(lam), lam.size, tau, fixed_rank, ctypes.byref(r),
                                ctypes.byref(t)), "truncate")
    return int(r.value), float(t.value)


@dataclass
class TuckerResult:
    core: np.ndarray            # Fortran order, shape = ranks
    factors: list               # U_n, I_n x R_n
    ranks: tuple
    eigvals: list               # per-mode spectra, descending
    discarded: np.ndarray       # tail sum dropped at each mode
    norm2: float                # ||X||^2
    sweeps: list                # Jacobi sweeps per mode


def sthosvd(x, eps: float, order=None, ranks=None) -> TuckerResult:
    """Alg. 1 (ST-HOSVD) on the CPU in FP64."""
    x = _f64_fortran(x)
    nd = x.ndim
    dims = x.shape
    core = np.empty(x.size)
    rk = (ctypes.c_int64 * nd)()
    fac = np.empty(sum(d * d for d in dims))
    eig = np.empty(sum(dims))
    disc = np.empty(nd)
    nrm = np.empty(1)
    sw = (ctypes.c_int * nd)()
    ordp = (ctypes.c_int * nd)(*order) if order is not None else None
    fixp = (ctypes.c_int64 * nd)(*ranks) if ranks is not None else None
    _check(_load().orc_sthosvd(_p(_flat(x)), nd, _dims(x), eps, ordp, fixp, _p(core), rk,
                               _p(fac), _p(eig), _p(disc), _p(nrm), sw), "sthosvd")
    ranks_t = tuple(int(r) for r in rk)
    factors, spectra = [], []
    fo = eo = 0
    for k in range(nd):
        u = fac[fo:fo + dims[k] * ranks_t[k]].reshape(dims[k], ranks_t[k]).copy()
        factors.append(u)
        spectra.append(eig[eo:eo + dims[k]].copy())
        fo += dims[k] * dims[k]
        eo += dims[k]
    g = core[:int(np.prod(ranks_t))].reshape(ranks_t, order="F").copy()
    return TuckerResult(g, factors, ranks_t, spectra, disc, float(nrm[0]), list(sw))


def sthosvd_qr(x, eps: float, order=None, ranks=None) -> TuckerResult:
    """Alg. 1 with the SVD of each ``Y_(n)`` taken through the QR of
    ``Y_(n)^T`` instead of the Gram (the stable variant Sec. IX proposes for
    eps near sqrt(u)): per mode, R of a Householder QR, one-sided Jacobi SVD
    of R, eigenvalues ``sigma^2``, the same rank rule, U_n = leading right
    singular vectors of R, ``Y <- Y x_n U_n^T``.  ``sweeps`` counts Jacobi
    sweeps."""
    x = _f64_fortran(x)
    nd = x.ndim
    order = list(range(nd)) if order is None else [int(k) for k in order]
    if sorted(order) != list(range(nd)):
        raise ValueError("order must be a permutation of the modes")
    nu = norm2(x)
    tau = eps * eps * nu / nd
    y = x
    factors, spectra = [None] * nd, [None] * nd
    rk, disc, sweeps = [0] * nd, np.zeros(nd), [0] * nd
    for n in order:
        lam, v, sw = mode_svd_qr(y, n)
        r, d = truncate(lam, tau, int(ranks[n]) if ranks is not None else 0)
        factors[n] = v[:, :r].copy()
        spectra[n] = lam
        rk[n], disc[n], sweeps[n] = r, d, sw
        y = ttm(y, n, factors[n].T)
    return TuckerResult(y, factors, tuple(rk), spectra, disc, nu, sweeps)


@dataclass
class HooiResult:
    core: np.ndarray            # Fortran order, shape = ranks
    factors: list               # U_n, I_n x R_n
    ranks: tuple
    fits: list                  # ||X||^2 - ||G||^2 after ST-HOSVD, then after each sweep
    norm2: float                # ||X||^2
    sweeps: int                 # sweeps run


def hooi(x, eps: float, ranks=None, order=None, max_sweeps: int = 50,
         tol: float = 0.0) -> HooiResult:
    """Alg. 2 (HOOI) on the CPU in FP64.  Starts from ST-HOSVD (Alg. 1, with
    ``eps`` or fixed ``ranks``); each sweep visits modes 1..N, forms
    Y = X x_m U_m^T over every m != n (ascending m), takes the leading R_n
    eigenvectors of Y_(n) Y_(n)^T as the new U_n, and after mode N forms the
    core G = Y x_N U_N^T.  Stops when the fit ||X||^2 - ||G||^2 (the model
    error, Sec. II-B) decreases by at most ``tol * ||X||^2`` in a sweep, or
    after ``max_sweeps`` sweeps; ``tol < 0`` runs exactly ``max_sweeps``."""
    x = _f64_fortran(x)
    init = sthosvd(x, eps, order=order, ranks=ranks)
    nd = x.ndim
    rk = init.ranks
    u = [f.copy() for f in init.factors]
    nu = init.norm2
    g = init.core
    fits = [nu - float(np.sum(g * g))]
    sweeps = 0
    for _ in range(max_sweeps):
        y = x
        for n in range(nd):
            y = x
            for m in range(nd):
                if m != n:
                    y = ttm(y, m, u[m].T)
            _, v, _ = sym_eig(gram(y, n))
            u[n] = v[:, :rk[n]].copy()
        g = ttm(y, nd - 1, u[nd - 1].T)
        fits.append(nu - float(np.sum(g * g)))
        sweeps += 1
        if tol >= 0.0 and fits[-2] - fits[-1] <= tol * nu:
            break
    return HooiResult(g, u, rk, fits, nu, sweeps)


def reconstruct(core, factors, full_dims=None) -> np.ndarray:
    """``X~ = G x_1 U_1 ... x_N U_N`` (Sec. II-C)."""
    core = _f64_fortran(core)
    nd = core.ndim
    full = tuple(int(u.shape[0]) for u in factors) if full_dims is None else tuple(full_dims)
    packed = np.concatenate([np.ascontiguousarray(u, dtype=np.float64).ravel() for u in factors])
    out = np.empty(int(np.prod(full)))
    _check(_load().orc_reconstruct(_p(_flat(core)), nd, _dims(core), _p(packed),
                                   (ctypes.c_int64 * nd)(*full), _p(out)), "reconstruct")
    return out.reshape(full, order="F")


def error_metrics(x, xhat):
    """``(||X - X~||^2, max|X - X~|, ||X||^2)``."""
    x = _f64_fortran(x)
    xh = _f64_fortran(xhat)
    out = np.empty(3)
    _check(_load().orc_error_metrics(_p(_flat(x)), _p(_flat(xh)), x.size, _p(out)), "metrics")
    return float(out[0]), float(out[1]), float(out[2])


def compression_ratio(dims, ranks) -> float:
    """``C = prod I_n / (prod R_n + sum I_n R_n)`` (Sec. VII-B)."""
    return float(np.prod(dims, dtype=np.float64) /
                 (np.prod(ranks, dtype=np.float64) + sum(i * r for i, r in zip(dims, ranks))))
