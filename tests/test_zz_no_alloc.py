"""The allocation-free Gram entry point (gram_mode_n_noalloc, its scratch a
static per-device array) against gram_mode_n with a caller's workspace: the
same kernels and the same plan, so the results agree bit for bit.  Two calls
in a row, the second on a smaller input, so that the second reuses scratch
the first left behind; both precisions, the largest plan (J = 256, L = 1),
a pair-group shape (J = 256, L > 1) and a narrow mode."""
import ctypes

import pytest
import torch

import synth
from paper_1510_06689_amd import tucker
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    # (dims, mode, precision, dtype): the second of each precision is smaller
    ((256, 40, 30), 0, "split_bf16", torch.float32),   # the largest plan (68.0 MiB)
    ((128, 96, 200), 0, "split_bf16", torch.float32),
    ((100, 30, 7), 0, "split_bf16", torch.float32),
    ((40, 256, 30), 1, "split_bf16", torch.float32),
    ((17, 140, 9), 1, "split_bf16", torch.float32),
    ((96, 80, 300), 2, "fp64", torch.float64),
    ((50, 33, 20), 1, "fp64", torch.float64),
    ((128, 64, 24), 2, "fp64", torch.float32),   # narrow mode (J = 24, runs of 8192)
    ((64, 16, 5), 2, "fp64", torch.float32),
]


def _ws_gram(y, mode, precision):
    lib = tucker.library()
    sh = tucker.shape_of(y)
    prec = tucker.GRAM_PRECISIONS[precision]
    need = lib.gram_workspace_bytes(ctypes.byref(sh), mode, prec)
    ws = tucker._workspace(need, y.device)
    j = y.shape[mode]
    s = torch.empty((j, j), dtype=torch.float64, device=y.device)
    q = torch.empty((), dtype=torch.float64, device=y.device)
    tucker._check(lib.gram_mode_n(ctypes.byref(sh), y.data_ptr(), mode, prec, s.data_ptr(),
                                  q.data_ptr(), tucker._aligned(ws), need,
                                  tucker._stream(y.device)))
    return s, q, need


def test_noalloc_equals_gram_mode_n_on_consecutive_calls():
    lib = tucker.library()
    limit = lib.gram_noalloc_scratch_bytes()
    assert limit == 72 << 20
    for i, (dims, mode, prec, dtype) in enumerate(CASES):
        say(f"noalloc case {i}: dims {dims} mode {mode} {prec} {dtype}")
        y = to_dev(synth.random_tensor(dims, seed=100 + i, dtype=dtype))
        ref, qref, need = _ws_gram(y, mode, prec)
        assert 0 < need <= limit
        j = dims[mode]
        out = torch.full((j, j), float("nan"), dtype=torch.float64, device=y.device)
        q = torch.full((), float("nan"), dtype=torch.float64, device=y.device)
        s, q = tucker.gram_noalloc(y, mode, prec, out=out, sumsq=q)
        torch.cuda.synchronize()
        assert s.data_ptr() == out.data_ptr()
        assert torch.equal(s, ref), (i, (s - ref).abs().max().item())
        assert torch.equal(q, qref)


def test_noalloc_rejects_bad_arguments_before_the_device():
    lib = tucker.library()
    sh = tucker.Shape()
    sh.ndim, sh.dtype = 2, tucker.F32
    sh.dims[0], sh.dims[1] = 8, 8
    assert lib.gram_mode_n_noalloc(ctypes.byref(sh), 0x1000, 2, 0, 0x1000, None, None) == -1
    assert lib.gram_mode_n_noalloc(ctypes.byref(sh), None, 0, 0, 0x1000, None, None) == -1
    sh.dtype = tucker.F64
    assert lib.gram_mode_n_noalloc(ctypes.byref(sh), 0x1000, 0, 1, 0x1000, None, None) == -2
