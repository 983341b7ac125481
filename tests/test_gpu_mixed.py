"""GPU parity of the mixed-precision path against the FP64 CPU oracle run on
the same FP32-stored values (widened exactly to FP64).

Tolerances are worst-case bounds of the split arithmetic, not fitted:

* split Gram: per tile and row, q = x 2^(15-E) is rounded to an integer
  and split into 8-bit halves, x = x~ + d with |d| <= 2^(E-16), where E is
  the exponent of 1.004 max|x| rounded up (so that |q| < 32640 fits the two
  int8 halves): 2^E <= 2 * 1.004 max|x|, and every element is represented
  to c 2^-15 m_i with c = 1.004 (m_i the row's largest magnitude).  The
  products of the halves are exact and sum_k d_ik^2 is subtracted from the
  diagonal, so S~ - S = -(X D^T + D X^T) + offdiag(D D^T):
      |dS_ij| <= c 2^-15 (m_i |x_j|_1 + m_j |x_i|_1) + c^2 2^-30 K m_i m_j.
  Exact rank agreement on planted tensors is the sharper check.
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
from gpu_util import SPLIT_STEP, U32, U64, check_against_oracle, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def split_gram_tolerance(xh, n, ref):
    """Elementwise bound of the split-bf16 Gram of mode n (see module doc)."""
    m = oracle.unfold(xh, n)
    rowmax = np.abs(m).max(axis=1)
    l1 = np.abs(m).sum(axis=1)
    k = m.shape[1]
    d = np.sqrt(np.abs(np.diag(ref)))
    c = SPLIT_STEP
    return (c * 2.0**-15 * (np.outer(rowmax, l1) + np.outer(l1, rowmax))
            + c * c * 2.0**-30 * k * np.outer(rowmax, rowmax)
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
    # J == 128 with L % 8 == 0: two register tiles where tile widths divide
    ((8, 128, 700), (1,)),      # 16 b-blocks per tile, ragged last tile
    ((16, 128, 45), (1,)),      # 8 b-blocks per tile, ragged last tile
    ((256, 128, 5), (1,)),      # each b-block cut into two full tiles
    ((24, 128, 20), (1,)),      # 128 % 24 != 0: one register tile
    ((200, 128, 3), (1,)),      # 200 % 128 != 0: one register tile
    # L % 4 == 0, L % 8 != 0: the two 4-column halves at their own offsets
    ((12, 40, 30), (1,)),       # packed tiles (10 b-blocks), class 64
    ((20, 100, 9), (1,)),       # packed tiles (6 b-blocks, ragged), class 128
    ((36, 128, 5), (1,)),       # J == 128: one register tile (two need L % 8 == 0)
    ((132, 24, 7), (1,)),       # cut tiles (132 > 128 columns per run)
    ((7, 200, 9), (1,)),        # J class 256, strided loader (L = 7), pair groups
    ((32, 256, 40), (1,)),      # J = 256, contiguous loader (L = 32), pair groups
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
    # L == 1 with J % 8 != 0 and K % 4 != 0: 16-byte accesses at 4-byte alignment
    ((37, 20, 11), 0, 5), ((100, 30, 7), 0, 12), ((93, 17, 5), 0, 33),
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
    values: identical ranks, every discarded sum within the library's
    reported split-Gram bound plus the carried TTM errors, the relative error
    within eps and within what those imply of the oracle's, spectra within the
    split Gram's perturbation."""
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
    tol = check_against_oracle(res, ref, dims, order, res.ttm_precision, rel, rel_ref)
    tau = eps * eps / len(dims)
    say(f"  relerr mixed {rel:.6e} oracle {rel_ref:.6e}; bounds {res.tail_error_bound}; "
        f"sum of tolerances {tol / tau:.3f} tau")
    assert tol <= len(dims) * tau   # each mode's bound stays below its threshold


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
    for eps in (1e-5, 1e-3):
        say(f"guard eps={eps}")
        res = tucker.sthosvd(xd, eps, gram_precision="split_bf16", ttm_precision="bf16x3")
        ref = oracle.sthosvd(xh, eps)
        say(f"  ranks {res.ranks} oracle {ref.ranks}, redone {res.fp64_modes}")
        assert res.ranks == ref.ranks, (res.ranks, ref.ranks, res.fp64_modes)
        if eps == 1e-3:
            assert not res.fp64_modes          # cuts far from tau: certified
        assert res.ttm_precision == ("fp64" if eps == 1e-5 else "bf16x3")


def _first_mode_tie_case():
    """The late-mode tensor processed in the order (2, 1, 3, 4), with eps set
    so that the first-processed mode (J = 128, the same data on the GPU and
    the oracle) is cut at t_R = (1 - 1e-4) tau: no split-Gram bound is that
    small, while FP64 Grams agree far more closely (the other modes' cuts are
    far from tau)."""
    dims, ranks = (24, 128, 24, 12), (6, 24, 6, 4)
    x = synth.planted_tucker(dims, ranks, rho=0.64, factor_kind="cosine", noise=1e-7,
                             noise_mode="sigma", seed=77, dtype=torch.float32)
    xh = x.double().numpy()
    order = (1, 0, 2, 3)
    eps = 1e-4
    for _ in range(10):
        probe = oracle.sthosvd(xh, eps, order=order)
        lam = np.maximum(probe.eigvals[1], 0.0)
        t_r = float(lam[probe.ranks[1]:].sum())
        nxt = math.sqrt(t_r / (1.0 - 1e-4) * len(dims) / probe.norm2)
        if abs(nxt / eps - 1.0) < 1e-13:
            break
        eps = nxt
    return x, xh, eps, order


def test_mixed_guard_redoes_a_near_tie_in_fp64():
    x, xh, eps, order = _first_mode_tie_case()
    ref = oracle.sthosvd(xh, eps, order=order)
    res = tucker.sthosvd(to_dev(x), eps, order=order, gram_precision="split_bf16",
                         ttm_precision="bf16x3")
    say(f"near tie eps={eps:.6e}: ranks {res.ranks} oracle {ref.ranks}, redone {res.fp64_modes}")
    assert 1 in res.fp64_modes
    assert res.ranks == ref.ranks


def _late_mode_case(frac=0.7):
    """A 4-way tensor whose second mode (J = 128, processed after the first
    mode's truncation) is cut where the oracle's tail sum is frac tau (by
    default the threshold sits 0.3 tau above it), at eps near 1e-4 (tau about 2.7e-9 ||X||^2): between
    the error a split Gram's tail sums can carry in a late mode (about tau/3)
    and a quarter of tau.  The core decays slowly (rho = 0.64, mode-2 rank
    24) so that signal eigenvalues reach that level; eps is the fixed point
    of tau = t_R / frac over the oracle's own mode-2 tail sums (frac = 0.7:
    t_{R-1} = 1.26 tau at R = 21; the other modes' cuts are far from tau)."""
    dims, ranks = (24, 128, 24, 12), (6, 24, 6, 4)
    x = synth.planted_tucker(dims, ranks, rho=0.64, factor_kind="cosine", noise=1e-7,
                             noise_mode="sigma", seed=77, dtype=torch.float32)
    xh = x.double().numpy()
    eps = 1e-4
    for _ in range(8):
        probe = oracle.sthosvd(xh, eps)
        lam = np.maximum(probe.eigvals[1], 0.0)
        t_r = float(lam[probe.ranks[1]:].sum())
        nxt = math.sqrt(t_r / frac * len(dims) / probe.norm2)
        if abs(nxt / eps - 1.0) < 1e-12:
            break
        eps = nxt
    return x, xh, eps


def test_mixed_guard_late_mode_near_threshold():
    """Whatever the guard decides on the late mode near its threshold, the
    ranks equal the oracle's, and where the split rank was accepted the
    discarded sum lies within the reported bound."""
    x, xh, eps = _late_mode_case()
    ref = oracle.sthosvd(xh, eps)
    tau = eps * eps * ref.norm2 / 4
    say(f"late-mode case eps={eps:.4e}, oracle ranks {ref.ranks}, mode-2 tail "
        f"{ref.discarded[1] / tau:.3f} tau")
    res = tucker.sthosvd(to_dev(x), eps, gram_precision="split_bf16", ttm_precision="bf16x3")
    say(f"  gpu ranks {res.ranks}, redone in FP64 {res.fp64_modes}, bounds "
        f"{[b / tau for b in res.tail_error_bound]} tau")
    xg = tucker.reconstruct(res.core, res.factors)
    e2, _, _ = tucker.error_metrics(to_dev(x), xg)
    xr = oracle.reconstruct(ref.core, ref.factors)
    rel_ref = math.sqrt(float(np.sum((xh - xr) ** 2)) / ref.norm2)
    check_against_oracle(res, ref, x.shape, None, res.ttm_precision,
                         math.sqrt(e2 / ref.norm2), rel_ref)
    for n, b in enumerate(res.tail_error_bound):
        if n not in res.fp64_modes and b > 0:
            assert b <= tau - res.discarded[n]     # an accepted cut clears its bound


@pytest.mark.parametrize("eps,expect", [(3e-2, "bf16"), (1e-3, "bf16x3"), (1e-5, "fp64")])
def test_mixed_bf16_ttm_raised_under_eps_rule(eps, expect):
    """A requested bf16 TTM (relative error ~2^-8) runs as requested only
    when eps^2 / N >= 2^-13; below that it is raised to split-bf16, and below
    2^-31 to FP64 arithmetic; the ranks equal the oracle's either way."""
    x = synth.planted_tucker((64, 32, 32, 16), (8, 8, 8, 4), rho=0.7, factor_kind="cosine",
                             noise=1e-5, noise_mode="sigma", seed=21, dtype=torch.float32)
    xh = x.double().numpy()
    res = tucker.sthosvd(to_dev(x), eps, gram_precision="split_bf16", ttm_precision="bf16")
    ref = oracle.sthosvd(xh, eps)
    say(f"bf16 ttm requested at eps={eps}: ran {res.ttm_precision}, ranks {res.ranks} "
        f"oracle {ref.ranks}")
    assert res.ttm_precision == expect
    assert res.ranks == ref.ranks
    fixed = tucker.sthosvd(to_dev(x), 0.0, ranks=ref.ranks, gram_precision="split_bf16",
                           ttm_precision="bf16")
    assert fixed.ttm_precision == "bf16"        # fixed ranks keep the request


def test_first_gram_timing_leaves_results_unchanged():
    """tk_options.time_first_gram: the call reports a positive duration for
    the first mode's partial-Gram kernel (HIP events inside the call) and
    otherwise computes exactly what the untimed call computes."""
    x = synth.planted_tucker((96, 40, 36, 8), (8, 6, 6, 3), rho=0.7, factor_kind="cosine",
                             noise=1e-5, noise_mode="sigma", seed=81, dtype=torch.float32)
    xd = to_dev(x)
    for gp, tp in (("split_bf16", "bf16x3"), ("fp64", "fp64")):
        c = tucker.Compressor(x.shape, x.dtype, xd.device, 1e-4, gram_precision=gp,
                              ttm_precision=tp)
        assert c.run(xd) == 0.0
        r0 = c.result(copy=True)
        t = c.run(xd, time_first_gram=True)
        r1 = c.result(copy=True)
        say(f"{gp}/{tp}: first-mode partial Gram {t:.4f} ms, ranks {r1.ranks}")
        assert 0.0 < t < 1e3
        assert r0.ranks == r1.ranks
        assert torch.equal(r0.core, r1.core)
        assert all(torch.equal(a, b) for a, b in zip(r0.factors, r1.factors))
        assert c.run(xd) == 0.0  # the flag is per call
