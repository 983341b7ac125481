"""GPU parity of the mixed-precision path against the FP64 CPU oracle run on
the same FP32-stored values (widened exactly to FP64).

Tolerances are worst-case bounds of the split arithmetic, not fitted:

* split-bf16 Gram: per tile and row, x 2^(7-E) = hi + lo + d with hi an
  integer, lo its bf16 residual and |d| <= 2^-10, where max|x| < 2^E <=
  2 max|x|; so every element is represented to 2^-16 m_i (m_i the row's
  largest magnitude).  With all four products formed, hi*hi summed exactly
  and the rest (<= 2^7 units per product) accumulated in FP32 over at most
  24 steps per tile:
      |dS_ij| <= 2^-16 (m_i |x_j|_1 + m_j |x_i|_1) + 2^-24 K m_i m_j.
  Exact rank agreement on planted tensors is the sharper check: dropping
  lo*lo or rounding the hi*hi sums in FP32 changes the ranks there.
* split-bf16 TTM: x = hi + lo + d with |d| <= 2^-16 |x| on both operands,
  three products; plain bf16 TTM: |a_h y_h - a y| <= (2^-7 + 2^-16) |a y|;
  plus FP32 accumulation and the final FP32 rounding of the output.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1510_06689_amd import tucker
from gpu_util import U32, U64, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def split_gram_tolerance(xh, n, ref):
    """Elementwise bound of the split-bf16 Gram of mode n (see module doc)."""
    m = oracle.unfold(xh, n)
    rowmax = np.abs(m).max(axis=1)
    l1 = np.abs(m).sum(axis=1)
    k = m.shape[1]
    d = np.sqrt(np.abs(np.diag(ref)))
    return (2.0**-16 * (np.outer(rowmax, l1) + np.outer(l1, rowmax))
            + 2.0**-24 * k * np.outer(rowmax, rowmax)
            + (k + 2) * U64 * np.outer(d, d) + 1e-300)


GRAM_CASES = [
    ((32, 32, 32), None),
    ((5, 7, 3), None),
    ((128, 64, 16), None),
    ((40, 33, 37, 6), None),
    ((3, 16, 100), None),
    ((2, 200, 5), None),
    ((16, 300, 3), (1,)),
    ((1, 20, 1), None),
    ((7,), None),
    ((512, 3), (0,)),
    ((130, 2, 2, 9), None),
    ((256, 24, 8), (0, 1)),
    ((24, 256, 3), (1,)),
    ((47, 23, 32, 16), (2, 3)),
    ((47, 23, 1, 16), (3,)),
    ((100, 9, 13), (0,)),       # J % 4 == 0 with L == 1: 16-byte column pieces, J class 128
    ((132, 5, 7), (0,)),        # the same for J class 256 (three pair groups)
    ((128, 1000), (0,)),        # several tiles per workgroup and a ragged last tile
]


@pytest.mark.parametrize("dims,modes", GRAM_CASES)
def test_split_gram_matches_oracle(dims, modes):
    x = synth.random_tensor(dims, seed=7 * sum(dims), dtype=torch.float32)
    xh = x.double().numpy()
    xd = to_dev(x)
    for n in (range(len(dims)) if modes is None else modes):
        say(f"split gram dims={dims} mode={n}")
        s, sumsq = tucker.gram(xd, n, precision="split_bf16")
        torch.cuda.synchronize()
        s = s.cpu().numpy()
        ref = oracle.gram(xh, n)
        tol = split_gram_tolerance(xh, n, ref)
        err = np.abs(s - ref)
        assert np.all(err <= tol), f"max err/tol {np.max(err / tol)}"
        assert np.array_equal(s, s.T)
        assert math.isclose(float(sumsq.item()), float(np.trace(s)),
                            rel_tol=(dims[n] + 2) * U64)


def test_split_gram_diagonal_is_unbiased():
    """Dropping lo*lo would bias every diagonal entry by -sum(lo^2), about
    -1e-4 relative for Gaussian data (lo is up to half a unit of 2^(E-7));
    with it the relative errors are random, a few 1e-7 per row, and their
    mean over 128 rows is smaller still."""
    x = synth.random_tensor((128, 4096), seed=11, dtype=torch.float32)
    xh = x.double().numpy()
    s, _ = tucker.gram(to_dev(x), 0, precision="split_bf16")
    torch.cuda.synchronize()
    ref = oracle.gram(xh, 0)
    rel = (np.diag(s.cpu().numpy()) - np.diag(ref)) / np.diag(ref)
    assert abs(rel.mean()) < 5e-7, rel.mean()
    assert np.abs(rel).max() < 1e-5


def test_split_gram_is_deterministic():
    x = to_dev(synth.random_tensor((96, 40, 50), seed=5, dtype=torch.float32))
    for n in range(3):
        a, _ = tucker.gram(x, n, precision="split_bf16")
        b, _ = tucker.gram(x, n, precision="split_bf16")
        torch.cuda.synchronize()
        assert torch.equal(a, b)


TTM_CASES = [
    ((32, 32, 32), 0, 4), ((32, 32, 32), 1, 5), ((32, 32, 32), 2, 6),
    ((5, 7, 3), 1, 2), ((128, 64, 16), 0, 16), ((128, 64, 16), 1, 17),
    ((128, 64, 16), 2, 40), ((40, 33, 37, 6), 0, 3), ((40, 33, 37, 6), 1, 64),
    ((40, 33, 37, 6), 2, 100), ((40, 33, 37, 6), 3, 6), ((3, 16, 100), 1, 1),
    ((2, 200, 5), 1, 300), ((16, 300, 3), 1, 33), ((7,), 0, 3), ((512, 3), 0, 20),
    ((20, 30, 2), 2, 300), ((64, 9, 18), 0, 64), ((256, 40, 3), 0, 32),
    ((47, 32, 32, 16), 1, 23), ((47, 23, 32, 16), 2, 17),
]


@pytest.mark.parametrize("precision", ["bf16x3", "bf16"])
@pytest.mark.parametrize("transpose", [True, False])
@pytest.mark.parametrize("dims,n,k", TTM_CASES)
def test_mixed_ttm_matches_oracle(dims, n, k, transpose, precision):
    say(f"mixed ttm dims={dims} mode={n} K={k} transpose={transpose} {precision}")
    x = synth.random_tensor(dims, seed=5 * sum(dims) + k, dtype=torch.float32)
    xh = x.double().numpy()
    rng = np.random.default_rng(k + 1)
    v = rng.standard_normal((k, dims[n]))
    m = v.T if transpose else v
    md = tucker.empty_colmajor(m.shape[0], m.shape[1], "cuda:0").copy_(
        torch.as_tensor(np.asfortranarray(m)).to("cuda:0"))
    z = tucker.ttm(to_dev(x), n, md, transpose=transpose, precision=precision)
    torch.cuda.synchronize()
    ref = oracle.ttm(xh, n, v)
    absprod = oracle.ttm(np.abs(xh), n, np.abs(v))
    nks = (dims[n] + 31) // 32
    if precision == "bf16x3":
        c = 4 * 2.0**-16 + (3 * nks + 4) * 2.0**-24
    else:
        c = 2.0**-7 + 2.0**-14 + (nks + 4) * 2.0**-24
    tol = c * absprod + U32 * np.abs(ref) + 1e-300
    err = np.abs(to_host(z).astype(np.float64) - ref)
    assert err.shape == ref.shape
    assert np.all(err <= tol), f"max err/tol {np.max(err / tol)}"


MIXED_STHOSVD = [
    # dims, ranks, rho, eps, order
    ((32, 32, 32), (4, 5, 6), 1.0, 1e-4, None),
    ((48, 40, 36, 12), (6, 5, 4, 3), 0.7, 1e-4, None),
    ((48, 40, 36, 12), (6, 5, 4, 3), 0.7, 1e-3, (3, 2, 1, 0)),
    ((130, 20, 9), (8, 4, 3), 0.8, 1e-4, (1, 0, 2)),
]


@pytest.mark.parametrize("dims,ranks,rho,eps,order", MIXED_STHOSVD)
def test_mixed_sthosvd_ranks_and_error(dims, ranks, rho, eps, order):
    """Mixed ST-HOSVD on FP32 storage against the FP64 oracle on the same
    values: identical ranks, relative error within 1e-4 of the oracle's (and
    within eps), spectra within the split Gram's perturbation."""
    say(f"mixed sthosvd dims={dims} eps={eps} order={order}")
    x = synth.planted_tucker(dims, ranks, rho=rho, noise=1e-5, seed=3 + sum(dims),
                             dtype=torch.float32)
    xh = x.double().numpy()
    xd = to_dev(x)
    res = tucker.sthosvd(xd, eps, order=order, gram_precision="split_bf16",
                         ttm_precision="bf16x3")
    ref = oracle.sthosvd(xh, eps, order=order)
    assert res.ranks == ref.ranks
    nu = ref.norm2
    first = (order or range(len(dims)))[0]
    lam = res.eigvals[first].cpu().numpy()
    g1 = oracle.gram(xh, first)
    bound = np.linalg.norm(split_gram_tolerance(xh, first, g1))  # |dlam| <= |dS|_2 <= |dS|_F
    assert np.all(np.abs(lam - ref.eigvals[first]) <= bound)
    xg = tucker.reconstruct(res.core, res.factors)
    e2, _, _ = tucker.error_metrics(xd, xg)
    rel = math.sqrt(e2 / nu)
    xr = oracle.reconstruct(ref.core, ref.factors)
    rel_ref = math.sqrt(float(np.sum((xh - xr) ** 2)) / nu)
    assert rel <= eps
    assert abs(rel - rel_ref) <= 1e-4
    say(f"  relerr mixed {rel:.3e} oracle {rel_ref:.3e}")


def test_mixed_reconstruct_matches_fp64():
    x = synth.planted_tucker((30, 20, 10), (4, 3, 2), rho=0.8, noise=1e-3, seed=9).numpy()
    ref = oracle.sthosvd(x, 1e-2)
    core = to_dev(ref.core, dtype=torch.float32)
    facs = [tucker.empty_colmajor(u.shape[0], u.shape[1], "cuda:0").copy_(torch.as_tensor(u))
            for u in ref.factors]
    xm = to_host(tucker.reconstruct(core, facs, precision="bf16x3")).astype(np.float64)
    x64 = to_host(tucker.reconstruct(core, facs, precision="fp64")).astype(np.float64)
    scale = np.abs(x64).max()
    assert np.abs(xm - x64).max() <= 64 * 2.0**-16 * scale


def test_mixed_guard_recomputes_uncertain_modes_in_fp64():
    """At eps = 1e-5 the threshold falls inside the noise eigenvalues, where
    the split Gram cannot certify the rank: the guard must redo those modes
    in FP64 (and the TTMs run in FP64, the split TTM's error being of the
    threshold's order), after which every rank equals the oracle's.  At
    eps = 1e-3 the margin is wide and no mode is redone."""
    x = synth.planted_tucker((64, 32, 32, 16), (8, 8, 8, 4), rho=0.7, factor_kind="cosine",
                             noise=1e-5, noise_mode="sigma", seed=21, dtype=torch.float32)
    xh = x.double().numpy()
    xd = to_dev(x)
    for eps, expect_fallback in ((1e-5, True), (1e-3, False)):
        say(f"guard eps={eps}")
        res = tucker.sthosvd(xd, eps, gram_precision="split_bf16", ttm_precision="bf16x3")
        ref = oracle.sthosvd(xh, eps)
        assert res.ranks == ref.ranks, (res.ranks, ref.ranks, res.fp64_modes)
        assert (len(res.fp64_modes) > 0) == expect_fallback, res.fp64_modes
        assert res.ttm_precision == ("fp64" if expect_fallback else "bf16x3")
