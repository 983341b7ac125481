"""Parity at the largest single-GPU workload, combustion256 (256x256x256x64x16
stored FP32: 2^34 elements, 68.7 GB), on the mixed path in both mode orders
(1..5 and 5..1, Sec. VIII-C on the order's cost) and on the FP64-arithmetic path
over the same FP32 data.

The oracle checks what it can compute one by one: mode-1 Gram entries (J = 256,
the split kernel's three pair groups) from two-row slices of the unfolding.
The runs are checked against properties that hold at any size: the planted
ranks, ||X||^2 - ||G||^2 = sum of discarded eigenvalues (= ||X - X~||^2,
checked by a reconstruction for order 1..5), orthonormal factors, and per
order the mixed path's discarded sums and error within the bounds derived from
the split Gram's reported representation error and the TTMs' arithmetic
(gpu_util.carried_errors) of the FP64-arithmetic path's in the same order."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1510_06689_amd import tucker
from gpu_util import U32, U64, check_against_oracle, mode1_rows, say, split_gram_bound

pytestmark = pytest.mark.gpu

W = synth.WORKLOADS["combustion256"]
PAIRS = [(0, 0), (7, 200), (255, 255), (128, 129), (31, 32)]


@pytest.fixture(scope="module")
def x32():
    say(f"generating {W.name} {W.dims} FP32 ({W.numel * 4 / 1e9:.1f} GB)")
    x = W.make(dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    yield x
    del x
    torch.cuda.empty_cache()


@pytest.mark.timeout(400)
def test_combustion256_mode1_split_gram_entries(x32):
    s, _ = tucker.gram(x32, 0, precision="split_bf16")
    torch.cuda.synchronize()
    s = s.cpu().numpy()
    k = x32.numel() // x32.shape[0]
    for i, j in PAIRS:
        sub = mode1_rows(x32, i, j)
        ref = oracle.gram(sub, 0)
        d = np.sqrt(np.diag(ref))
        tol = (k + 2) * U64 * np.outer(d, d) + split_gram_bound(sub)
        got = np.array([[s[i, i], s[i, j]], [s[j, i], s[j, j]]])
        say(f"S[{i},{j}] = {got[0, 1]:.12e} oracle {ref[0, 1]:.12e}")
        assert np.all(np.abs(got - ref) <= tol), (i, j, got - ref, tol)


def _identity(res):
    nu = res.norm2
    g2 = float((res.core.double() ** 2).sum().item())
    return nu, g2, float(sum(res.discarded))


def _orthonormal(res):
    for u in res.factors:
        ut = u.cpu().numpy()
        assert np.abs(ut.T @ ut - np.eye(ut.shape[1])).max() <= 1e-12


@pytest.mark.timeout(400)
def test_combustion256_both_orders_and_fp64(x32):
    eps = W.eps
    for name, order in (("1..5", None), ("5..1", (4, 3, 2, 1, 0))):
        r64 = tucker.sthosvd(x32, eps, order=order, gram_precision="fp64", ttm_precision="fp64")
        torch.cuda.empty_cache()
        nu, g2, disc = _identity(r64)
        assert r64.ranks == W.ranks
        # FP64 arithmetic, FP32 storage: rounding a stored TTM output changes its
        # squared norm by at most 2 u32 of it, once per mode
        assert abs((nu - g2) - disc) <= 2 * len(W.dims) * U32 * nu
        _orthonormal(r64)
        rel64 = math.sqrt(disc / nu)
        r = tucker.sthosvd(x32, eps, order=order, gram_precision="split_bf16",
                           ttm_precision="bf16x3")
        torch.cuda.empty_cache()
        nu, g2, disc = _identity(r)
        say(f"order {name}: ranks {r.ranks}, modes redone in FP64 {r.fp64_modes}, "
            f"discarded/||X||^2 {disc / nu:.4e}, bounds/tau "
            f"{[round(b / (eps * eps * nu / 5), 4) for b in r.tail_error_bound]}")
        assert r.ranks == W.ranks
        # FP32 storage and split products: the identity holds to ~2^-17 of ||X||^2
        assert abs((nu - g2) - disc) <= 1e-6 * nu
        _orthonormal(r)
        rel = math.sqrt(disc / nu)
        if order is None:
            xh = tucker.reconstruct(r.core, r.factors)
            e2, _, n2 = tucker.error_metrics(x32, xh)
            del xh
            torch.cuda.empty_cache()
            assert math.isclose(n2, nu, rel_tol=1e-6)
            assert abs(e2 - disc) <= 1e-6 * nu
            assert math.sqrt(e2 / nu) <= eps
        say(f"  relerr mixed {rel:.6e} fp64 {rel64:.6e}")
        check_against_oracle(r, r64, W.dims, order, r.ttm_precision, rel, rel64,
                             storage_u=U32 * math.sqrt(2))
        del r, r64
        torch.cuda.empty_cache()
