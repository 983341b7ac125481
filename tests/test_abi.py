"""Host-side checks of the C-ABI (no GPU needed): the library loads, exports
every function the header declares, and rejects invalid arguments before
touching the device."""
import ctypes
import os
import re

import pytest

from paper_1510_06689_amd import tucker as tk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "tucker.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_exports_match_library():
    names = header_functions()
    assert "sthosvd_compress" in names and "gram_mode_n" in names
    lib = tk.library()
    for n in names:
        assert hasattr(lib, n), f"{n} declared in tucker.h but not exported"
    assert set(names) == set(tk.EXPORTS)


def test_library_is_gfx950_build():
    with open(tk.LIB_PATH, "rb") as f:
        blob = f.read()
    assert b"gfx950" in blob


def shape(dims, dtype=tk.F64):
    s = tk.Shape()
    s.ndim = len(dims)
    s.dtype = dtype
    for k, d in enumerate(dims):
        s.dims[k] = d
    return s


def last_error():
    return tk.library().tk_last_error().decode()


FAKE = 0x1000  # never dereferenced: validation fails first


def test_gram_validation():
    lib = tk.library()
    s = shape([4, 5, 6])
    assert lib.gram_mode_n(None, FAKE, 0, 0, FAKE, None, None, 0, None) == -1
    assert lib.gram_mode_n(ctypes.byref(s), FAKE, 3, 0, FAKE, None, None, 0, None) == -1
    assert "mode" in last_error()
    assert lib.gram_mode_n(ctypes.byref(s), FAKE, -1, 0, FAKE, None, None, 0, None) == -1
    assert lib.gram_mode_n(ctypes.byref(s), FAKE, 0, 7, FAKE, None, None, 0, None) == -1
    # split-bf16 needs FP32 storage
    assert lib.gram_mode_n(ctypes.byref(s), FAKE, 0, 1, FAKE, None, None, 0, None) == -2
    # workspace too small / misaligned
    need = lib.gram_workspace_bytes(ctypes.byref(s), 0, 0)
    assert need > 0
    assert lib.gram_mode_n(ctypes.byref(s), FAKE, 0, 0, FAKE, None, FAKE, need - 1, None) == -3
    assert lib.gram_mode_n(ctypes.byref(s), FAKE, 0, 0, FAKE, None, FAKE + 8, need, None) == -3
    bad = shape([4, 0, 6])
    assert lib.gram_mode_n(ctypes.byref(bad), FAKE, 0, 0, FAKE, None, None, 0, None) == -1
    big = shape([513, 2])
    assert lib.gram_mode_n(ctypes.byref(big), FAKE, 0, 0, FAKE, None, None, 0, None) == -2
    nd = shape([2] * 8)
    nd.ndim = 9
    assert lib.gram_mode_n(ctypes.byref(nd), FAKE, 0, 0, FAKE, None, None, 0, None) == -1
    wrong_dtype = shape([4, 5], dtype=7)
    assert lib.gram_mode_n(ctypes.byref(wrong_dtype), FAKE, 0, 0, FAKE, None, None, 0, None) == -1


def test_qr_validation():
    lib = tk.library()
    s = shape([4, 5, 6])
    assert lib.qr_r_mode_n(None, FAKE, 0, FAKE, None, None, 0, None) == -1
    assert lib.qr_r_mode_n(ctypes.byref(s), FAKE, 3, FAKE, None, None, 0, None) == -1
    assert "mode" in last_error()
    assert lib.qr_r_mode_n(ctypes.byref(s), None, 0, FAKE, None, None, 0, None) == -1
    assert lib.qr_r_mode_n(ctypes.byref(s), FAKE, 0, None, None, None, 0, None) == -1
    need = lib.qr_workspace_bytes(ctypes.byref(s), 0)
    assert need > 0
    assert lib.qr_r_mode_n(ctypes.byref(s), FAKE, 0, FAKE, None, FAKE, need - 1, None) == -3
    assert lib.qr_r_mode_n(ctypes.byref(s), FAKE, 0, FAKE, None, FAKE + 8, need, None) == -3
    wide = shape([129, 2])
    assert lib.qr_workspace_bytes(ctypes.byref(wide), 0) == 0
    assert lib.qr_r_mode_n(ctypes.byref(wide), FAKE, 0, FAKE, None, None, 0, None) == -2
    assert lib.qr_workspace_bytes(ctypes.byref(wide), 1) > 0  # the narrow mode is fine


def test_qr_option_validation():
    lib = tk.library()
    keep = []
    o = tk._options(3, 1e-7, None, None, None, "qr", "fp64", keep)
    s = shape([4, 5, 6])
    assert lib.sthosvd_workspace_bytes(ctypes.byref(s), ctypes.byref(o)) > 0
    s32 = shape([4, 5, 6], dtype=tk.F32)
    assert lib.sthosvd_workspace_bytes(ctypes.byref(s32), ctypes.byref(o)) > 0
    wide = shape([4, 129, 6])
    assert lib.sthosvd_workspace_bytes(ctypes.byref(wide), ctypes.byref(o)) == 0
    out = tk.Tucker()
    assert lib.sthosvd_compress(ctypes.byref(wide), FAKE, ctypes.byref(o), ctypes.byref(out),
                                None, 0, None) == -2
    # HOOI runs its sweeps on Grams: the QR option is rejected there
    assert lib.tucker_hooi_workspace_bytes(ctypes.byref(s), ctypes.byref(o)) == 0
    fits = (ctypes.c_double * 2)()
    done = ctypes.c_int(0)
    assert lib.tucker_hooi(ctypes.byref(s), FAKE, ctypes.byref(o), 1, 0.0, ctypes.byref(out),
                           fits, ctypes.byref(done), None, 0, None) == -2


def test_ttm_validation():
    lib = tk.library()
    s = shape([4, 5, 6])
    # op(M) must be K x J_n
    assert lib.ttm_mode_n(ctypes.byref(s), FAKE, 1, FAKE, 4, 3, 1, 0, 0x9000000, None) == -1
    assert lib.ttm_mode_n(ctypes.byref(s), FAKE, 1, FAKE, 3, 4, 0, 0, 0x9000000, None) == -1
    assert lib.ttm_mode_n(ctypes.byref(s), FAKE, 1, FAKE, 5, 3, 2, 0, 0x9000000, None) == -1
    # bf16 variants need FP32 storage
    assert lib.ttm_mode_n(ctypes.byref(s), FAKE, 1, FAKE, 5, 3, 1, 1, 0x9000000, None) == -2
    # overlapping output
    assert lib.ttm_mode_n(ctypes.byref(s), FAKE, 1, FAKE, 5, 3, 1, 0, FAKE + 8, None) == -1
    assert "overlap" in last_error()
    assert lib.ttm_mode_n(ctypes.byref(s), None, 1, FAKE, 5, 3, 1, 0, 0x9000000, None) == -1


def opts(eps=1e-3, order=None, ranks=None, max_ranks=None, gp=0, tp=0, keep=None):
    keep = [] if keep is None else keep
    return tk._options(3, eps, order, ranks, max_ranks, {0: "fp64", 1: "split_bf16"}[gp],
                       {0: "fp64", 1: "bf16", 2: "bf16x3"}[tp], keep), keep


def test_sthosvd_validation():
    lib = tk.library()
    s = shape([4, 5, 6])
    out = tk.Tucker()
    out.core_dev = FAKE
    out.core_capacity = 120
    for k in range(3):
        out.factors_dev[k] = FAKE
    cases = [
        (dict(eps=-1.0), -1), (dict(eps=float("nan")), -1), (dict(eps=float("inf")), -1),
        (dict(order=(0, 0, 1)), -1), (dict(order=(0, 1, 3)), -1),
        (dict(ranks=(0, 1, 1)), -1), (dict(ranks=(5, 1, 1)), -1),
        (dict(max_ranks=(0, 2, 2)), -1), (dict(ranks=(3, 3, 3), max_ranks=(2, 5, 6)), -7),
        (dict(gp=1), -2), (dict(tp=2), -2),
    ]
    for kw, code in cases:
        o, keep = opts(**kw)
        assert lib.sthosvd_workspace_bytes(ctypes.byref(s), ctypes.byref(o)) == 0, kw
        rc = lib.sthosvd_compress(ctypes.byref(s), FAKE, ctypes.byref(o), ctypes.byref(out),
                                  None, 0, None)
        assert rc == code, (kw, rc, last_error())
    o, keep = opts()
    need = lib.sthosvd_workspace_bytes(ctypes.byref(s), ctypes.byref(o))
    assert need > 0
    assert lib.sthosvd_compress(ctypes.byref(s), FAKE, ctypes.byref(o), ctypes.byref(out),
                                FAKE, need - 1, None) == -3
    assert lib.sthosvd_compress(ctypes.byref(s), FAKE, ctypes.byref(o), None, FAKE, need,
                                None) == -1
    out.factors_dev[2] = None
    assert lib.sthosvd_compress(ctypes.byref(s), FAKE, ctypes.byref(o), ctypes.byref(out),
                                FAKE, need, None) == -1
    # a rank capacity shrinks the workspace
    o2, keep2 = opts(max_ranks=(2, 2, 2))
    assert lib.sthosvd_workspace_bytes(ctypes.byref(s), ctypes.byref(o2)) < need


def test_reconstruct_and_metrics_validation():
    lib = tk.library()
    core = shape([2, 3])
    full = (ctypes.c_int64 * 2)(5, 0)
    ptrs = (ctypes.c_void_p * 2)(FAKE, FAKE)
    assert lib.reconstruct_workspace_bytes(ctypes.byref(core), full) == 0
    assert lib.tucker_reconstruct(ctypes.byref(core), FAKE, ptrs, None, full, 0, FAKE, None, 0,
                                  None) == -1
    full = (ctypes.c_int64 * 2)(5, 7)
    need = lib.reconstruct_workspace_bytes(ctypes.byref(core), full)
    assert need > 0
    ld = (ctypes.c_int64 * 2)(4, 7)
    assert lib.tucker_reconstruct(ctypes.byref(core), FAKE, ptrs, ld, full, 0, FAKE, FAKE, need,
                                  None) == -1
    assert lib.tucker_reconstruct(ctypes.byref(core), FAKE, ptrs, None, full, 1, FAKE, FAKE,
                                  need, None) == -2
    assert lib.tucker_error_metrics(None, FAKE, FAKE, None, None, 0, None) == -1


def test_batch_ttm_precision_floor():
    """Under the eps rule a batch refuses a TTM precision whose output error
    would reach the rank threshold (it has no output to report a raised
    precision in): bf16 needs eps^2/N >= 2^-13, split-bf16 eps^2/N >= 2^-31."""
    lib = tk.library()
    shapes = (tk.Shape * 2)(shape([8, 8, 8, 4], tk.F32), shape([6, 8, 8, 4], tk.F32))

    def need(eps, ttm, ranks=None):
        keep = []
        opt = tk._options(4, eps, None, ranks, None, "split_bf16", ttm, keep)
        return lib.sthosvd_batch_workspace_bytes(2, shapes, ctypes.byref(opt), None)

    floor_bf16 = (4 * 2.0 ** -13) ** 0.5      # eps with eps^2 / 4 = 2^-13
    floor_x3 = (4 * 2.0 ** -31) ** 0.5
    assert need(1.01 * floor_bf16, "bf16") > 0
    assert need(0.99 * floor_bf16, "bf16") == 0
    assert "bf16" in last_error() and "TK_TTM_BF16X3" in last_error()
    assert need(0.99 * floor_bf16, "bf16x3") > 0
    assert need(1.01 * floor_x3, "bf16x3") > 0
    assert need(0.99 * floor_x3, "bf16x3") == 0
    # fixed ranks: no rank decision depends on the TTM, any precision goes
    assert need(0.0, "bf16", ranks=(2, 2, 2, 2)) > 0
    h = ctypes.c_void_p()
    keep = []
    opt = tk._options(4, 1e-4, None, None, None, "split_bf16", "bf16", keep)
    assert lib.sthosvd_batch_create(2, shapes, None, ctypes.byref(opt), None, None, None, 0,
                                    None, ctypes.byref(h)) == -2


def test_status_strings():
    lib = tk.library()
    for code in range(0, -8, -1):
        assert lib.tk_status_string(code).decode() != "unknown status"
    assert lib.tk_status_string(-99).decode() == "unknown status"


def test_binding_rejects_host_tensors():
    import torch
    x = torch.zeros(3, 4, dtype=torch.float64)
    with pytest.raises(ValueError):
        tk.gram(x, 0)
