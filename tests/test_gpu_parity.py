"""GPU parity: every entry point of the C-ABI against the FP64 CPU oracle on
the same seeded inputs, element by element.  Shapes cover every tile regime
of the kernels (mode 1 with contiguous columns, short packed rows, long
strided rows), several tiles per workgroup and ragged tails (extents that are
not multiples of the 16-row blocks or 32-column tiles), extents 1 and the
largest supported extent, FP64 and FP32 storage."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1510_06689_amd import tucker
from gpu_util import U32, U64, gram_tolerance, say, to_dev, to_host, ttm_tolerance

pytestmark = pytest.mark.gpu

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
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dims,modes", GRAM_CASES)
def test_gram_matches_oracle(dims, modes, dtype):
    x = synth.random_tensor(dims, seed=sum(dims), dtype=dtype)
    xh = x.double().numpy()
    xd = to_dev(x)
    nu = oracle.norm2(xh)
    for n in (range(len(dims)) if modes is None else modes):
        say(f"gram dims={dims} mode={n} dtype={dtype}")
        s, sumsq = tucker.gram(xd, n)
        torch.cuda.synchronize()
        s = s.cpu().numpy()
        ref = oracle.gram(xh, n)
        k = xh.size // dims[n]
        tol = gram_tolerance(ref, k)
        err = np.abs(s - ref)
        assert np.all(err <= tol), f"max err/tol {np.max(err / tol)}"
        assert np.array_equal(s, s.T)
        assert math.isclose(float(sumsq.item()), nu, rel_tol=(xh.size + 2) * U64)


# Narrow modes (J <= 32) whose unfolding rows are runs of L contiguous
# elements, L a multiple of 8: the FP64 Gram streams them without an LDS
# tile.  Runs that are whole 32-column steps and ragged ones, one and several
# slabs (including slabs that change inside one wave's batch of steps),
# J = 1, J < 16, J = 16, 16 < J < 32, J = 32, a workgroup count at the grid
# cap with several batches per wave; offset = 1 shifts the data pointer by
# one element, so the vector loads' alignment fails and the tiled kernel
# runs instead.
NARROW_CASES = [
    ((96, 20, 7), 1),
    ((200, 16, 3), 1),
    ((72, 1, 5), 1),
    ((64, 32, 2), 1),
    ((8, 8, 5, 9), 2),
    ((1 << 21, 16), 1),
    ((1 << 20, 3, 11), 1),
    ((4096, 30), 1),
]


@pytest.mark.parametrize("offset", [0, 1])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dims,n", NARROW_CASES)
def test_gram_narrow_modes(dims, n, dtype, offset):
    say(f"narrow gram dims={dims} mode={n} dtype={dtype} offset={offset}")
    x = synth.random_tensor(dims, seed=sum(dims) + n, dtype=dtype)
    xh = x.double().numpy()
    size = xh.size
    buf = torch.empty(size + offset, dtype=dtype, device="cuda:0")
    xd = buf[offset:].view(tuple(reversed(dims))).permute(*reversed(range(len(dims))))
    xd.copy_(to_dev(x))
    assert xd.data_ptr() % 64 == (0 if offset == 0 else x.element_size())
    s, sumsq = tucker.gram(xd, n)
    torch.cuda.synchronize()
    s = s.cpu().numpy()
    ref = oracle.gram(xh, n)
    err = np.abs(s - ref)
    tol = gram_tolerance(ref, size // dims[n])
    assert np.all(err <= tol), f"max err/tol {np.max(err / tol)}"
    assert np.array_equal(s, s.T)
    nu = oracle.norm2(xh)
    assert math.isclose(float(sumsq.item()), nu, rel_tol=(size + 2) * U64)


def test_gram_is_deterministic():
    x = to_dev(synth.random_tensor((96, 40, 50), seed=5))
    for n in range(3):
        a, _ = tucker.gram(x, n)
        b, _ = tucker.gram(x, n)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_narrow_gram_and_ttm_are_deterministic(dtype):
    # the narrow kernels fold fixed per-wave partials in a fixed order
    x = to_dev(synth.random_tensor((1 << 14, 24, 9), seed=6, dtype=dtype))
    a, sa = tucker.gram(x, 1)
    b, sb = tucker.gram(x, 1)
    u = tucker.empty_colmajor(24, 8, "cuda:0").copy_(
        torch.as_tensor(np.asfortranarray(np.random.default_rng(6).standard_normal((24, 8)))))
    za = tucker.ttm(x, 1, u, transpose=True)
    zb = tucker.ttm(x, 1, u, transpose=True)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(sa, sb) and torch.equal(za, zb)


def test_sthosvd_is_deterministic():
    # extents 64 .. 200 run the eigensolver in three launches (the
    # multisection over one workgroup per eigenvalue) and the panel reduction
    x = to_dev(synth.planted_tucker((200, 96, 64), (10, 8, 6), rho=0.8, noise=1e-4, seed=8))
    r1 = tucker.sthosvd(x, 1e-3)
    r2 = tucker.sthosvd(x, 1e-3)
    assert r1.ranks == r2.ranks
    assert torch.equal(r1.core, r2.core)
    for u1, u2, l1, l2 in zip(r1.factors, r2.factors, r1.eigvals, r2.eigvals):
        assert torch.equal(u1, u2) and torch.equal(l1, l2)


TTM_CASES = [
    ((32, 32, 32), 0, 4), ((32, 32, 32), 1, 5), ((32, 32, 32), 2, 6),
    ((5, 7, 3), 1, 2), ((128, 64, 16), 0, 16), ((128, 64, 16), 1, 17),
    ((128, 64, 16), 2, 40), ((40, 33, 37, 6), 0, 3), ((40, 33, 37, 6), 1, 64),
    ((40, 33, 37, 6), 2, 100), ((40, 33, 37, 6), 3, 6), ((3, 16, 100), 1, 1),
    ((2, 200, 5), 1, 300), ((16, 300, 3), 1, 33), ((7,), 0, 3), ((512, 3), 0, 20),
    ((20, 30, 2), 2, 300), ((64, 9, 18), 0, 64),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("transpose", [True, False])
@pytest.mark.parametrize("dims,n,k", TTM_CASES)
def test_ttm_matches_oracle(dims, n, k, transpose, dtype):
    say(f"ttm dims={dims} mode={n} K={k} transpose={transpose} dtype={dtype}")
    x = synth.random_tensor(dims, seed=3 * sum(dims) + k, dtype=dtype)
    xh = x.double().numpy()
    rng = np.random.default_rng(k)
    v = rng.standard_normal((k, dims[n]))           # op(M), K x J_n
    m = v.T if transpose else v
    md = torch.as_tensor(np.asfortranarray(m)).to("cuda:0")
    md = tucker.empty_colmajor(m.shape[0], m.shape[1], "cuda:0").copy_(md)
    z = tucker.ttm(to_dev(x), n, md, transpose=transpose)
    torch.cuda.synchronize()
    ref = oracle.ttm(xh, n, v)
    tol = ttm_tolerance(xh, n, v)
    if dtype == torch.float32:  # output rounded to FP32 once
        tol = tol + U32 * np.abs(ref)
    err = np.abs(to_host(z).astype(np.float64) - ref)
    assert err.shape == ref.shape
    assert np.all(err <= tol), f"max err/tol {np.max(err / tol)}"


# Narrow modes (J <= 64, K <= 16, rows of Y_(n) made of runs of L contiguous
# elements, L a multiple of 8): the TTM runs in FP64 arithmetic without LDS
# whatever precision is asked for, so the FP64 bound (plus one rounding to
# FP32) holds for every option.  Ragged last steps, several slabs, J = 5,
# 16 < J <= 32 and 32 < J <= 64, K = 1 and K = 16, a large case with many
# steps per wave; offset = 1 misaligns the input pointer, which sends the
# call to the tiled kernels.
NARROW_TTM_CASES = [
    ((96, 16, 7), 1, 8),
    ((64, 64, 3), 1, 16),
    ((200, 40, 2), 1, 5),
    ((72, 33, 3), 1, 16),
    ((1 << 16, 64, 4), 1, 16),
    ((200, 5, 3), 1, 3),
    ((72, 20, 2), 1, 16),
    ((64, 32, 3), 1, 1),
    ((8, 8, 5, 9), 2, 4),
    ((1 << 20, 16), 1, 8),
    ((1 << 18, 3, 11), 1, 2),
]
NARROW_TTM_OPTIONS = [  # (dtype, precision, offset)
    (torch.float64, "fp64", 0), (torch.float64, "fp64", 1),
    (torch.float32, "fp64", 0), (torch.float32, "fp64", 1),
    (torch.float32, "bf16x3", 0), (torch.float32, "bf16", 0),
]


@pytest.mark.parametrize("dtype,precision,offset", NARROW_TTM_OPTIONS)
@pytest.mark.parametrize("transpose", [True, False])
@pytest.mark.parametrize("dims,n,k", NARROW_TTM_CASES)
def test_ttm_narrow_modes(dims, n, k, transpose, dtype, precision, offset):
    say(f"narrow ttm dims={dims} mode={n} K={k} transpose={transpose} {dtype} {precision} "
        f"offset={offset}")
    x = synth.random_tensor(dims, seed=5 * sum(dims) + k, dtype=dtype)
    xh = x.double().numpy()
    buf = torch.empty(xh.size + offset, dtype=dtype, device="cuda:0")
    xd = buf[offset:].view(tuple(reversed(dims))).permute(*reversed(range(len(dims))))
    xd.copy_(to_dev(x))
    rng = np.random.default_rng(k + dims[n])
    v = rng.standard_normal((k, dims[n]))           # op(M), K x J_n
    m = v.T if transpose else v
    md = tucker.empty_colmajor(m.shape[0], m.shape[1], "cuda:0").copy_(
        torch.as_tensor(np.asfortranarray(m)))
    z = tucker.ttm(xd, n, md, transpose=transpose, precision=precision)
    torch.cuda.synchronize()
    ref = oracle.ttm(xh, n, v)
    tol = ttm_tolerance(xh, n, v)
    if dtype == torch.float32:  # output rounded to FP32 once
        tol = tol + U32 * np.abs(ref)
    err = np.abs(to_host(z).astype(np.float64) - ref)
    assert err.shape == ref.shape
    assert np.all(err <= tol), f"max err/tol {np.max(err / tol)}"


def _compare_tucker(xh, res, ref, eps_sym):
    """Compare a GPU ST-HOSVD with the oracle's: ranks exactly; spectra and
    reconstructions within FP64 perturbation bounds."""
    assert res.ranks == ref.ranks
    n = xh.ndim
    nu = ref.norm2
    assert math.isclose(res.norm2, nu, rel_tol=(xh.size + 2) * U64)
    kappa = 1.0
    for k in range(n):
        lam = res.eigvals[k].cpu().numpy()
        lref = ref.eigvals[k]
        # Weyl: |d lambda| <= ||dS||, with ||dS|| <= J * K u ||S||
        jn = xh.shape[k]
        tol = 64 * jn * U64 * max(abs(lref[0]), 1e-300) * 8
        assert np.all(np.abs(lam - lref) <= tol + 1e-13 * abs(lref[0])), (k, np.abs(lam - lref).max())
        r = ref.ranks[k]
        gap = lref[r - 1] - (lref[r] if r < jn else 0.0)
        if gap > 0:
            kappa = max(kappa, lref[0] / gap)
        u = res.factors[k].cpu().numpy()
        np.testing.assert_allclose(u.T @ u, np.eye(r), atol=64 * jn * U64)
    xg = tucker.reconstruct(res.core, res.factors)
    xr = oracle.reconstruct(ref.core, ref.factors)
    diff = np.linalg.norm((to_host(xg) - xr).ravel())
    bound = 1e3 * n * U64 * kappa * math.sqrt(nu)
    assert diff <= bound, f"reconstruction differs by {diff:.3e} > {bound:.3e}"
    np.testing.assert_allclose(np.array(res.discarded), ref.discarded,
                               atol=1e3 * U64 * kappa * nu)
    return xg


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_sthosvd_planted32(seed):
    w = synth.WORKLOADS["planted32"]
    say(f"sthosvd planted32 seed={seed}")
    x = w.make(seed=seed)
    xh = x.numpy()
    res = tucker.sthosvd(to_dev(x), w.eps)
    ref = oracle.sthosvd(xh, w.eps)
    assert res.ranks == w.ranks
    xg = _compare_tucker(xh, res, ref, w.eps)
    e2, mx, n2 = tucker.error_metrics(to_dev(x), xg)
    re2, rmx, rn2 = oracle.error_metrics(xh, to_host(xg))
    assert math.isclose(e2, re2, rel_tol=1e-9) and math.isclose(n2, rn2, rel_tol=1e-12)
    assert mx == rmx
    assert math.sqrt(e2 / n2) <= w.eps


STHOSVD_CASES = [
    # dims, ranks, rho, eps, order, fixed ranks
    ((40, 33, 37, 6), (5, 4, 6, 2), 0.7, 1e-3, None, None),
    ((40, 33, 37, 6), (5, 4, 6, 2), 0.7, 1e-3, (3, 1, 0, 2), None),
    ((24, 20, 18), (3, 3, 3), 1.0, 0.0, None, None),             # eps = 0: full ranks
    ((24, 20, 18), (3, 3, 3), 1.0, 1e-2, None, (5, 2, 7)),        # fixed ranks
    ((64, 16, 12, 5), (8, 4, 3, 2), 0.6, 1e-4, (1, 3, 0, 2), None),
    ((1, 30, 9), (1, 4, 3), 0.8, 1e-3, None, None),               # extent-1 mode
    ((50,), (5,), 1.0, 1e-2, None, None),                         # N = 1
    ((130, 70), (10, 10), 0.5, 1e-5, None, None),                 # N = 2, ragged blocks
    # the 96-row register layout (64 < J <= 96): its largest and smallest
    # extents, and every vector of a full-rank J = 80 spectrum (eps = 0; the
    # noise eigenvalues form one cluster)
    ((96, 20, 10), (12, 6, 4), 0.8, 1e-4, None, None),
    ((65, 24, 9), (9, 5, 3), 0.7, 1e-3, None, None),
    ((80, 40, 30), (20, 8, 6), 0.9, 0.0, None, None),
    ((8, 8, 8, 8, 8), (2, 3, 2, 3, 2), 0.9, 1e-3, (4, 3, 2, 1, 0), None),
    # extents above 128: the tridiagonal reduction runs in global memory for
    # J - 128 columns (in panels of eight, the last one partial) before the
    # register finish; at J = 512 the whole reduction stays in global memory
    ((200, 40, 6), (10, 6, 3), 0.8, 1e-4, None, None),
    ((300, 20, 4), (12, 5, 3), 0.7, 1e-4, None, None),            # rank-deficient Gram
    ((512, 12, 3), (8, 4, 2), 0.7, 1e-3, None, None),
]


@pytest.mark.parametrize("dims,ranks,rho,eps,order,fixed", STHOSVD_CASES)
def test_sthosvd_matches_oracle(dims, ranks, rho, eps, order, fixed):
    say(f"sthosvd dims={dims} eps={eps} order={order} fixed={fixed}")
    x = synth.planted_tucker(dims, ranks, rho=rho, noise=1e-4, seed=len(dims) + sum(dims))
    xh = x.numpy()
    res = tucker.sthosvd(to_dev(x), eps, order=order, ranks=fixed)
    ref = oracle.sthosvd(xh, eps, order=order, ranks=fixed)
    _compare_tucker(xh, res, ref, eps)


def test_sthosvd_fp32_storage_fp64_compute():
    """FP32 storage with FP64 arithmetic: the oracle sees the same FP32 values
    widened; TTM outputs round to FP32 after every mode."""
    w = synth.WORKLOADS["planted32"]
    x32 = w.make(dtype=torch.float32)
    xh = x32.double().numpy()
    res = tucker.sthosvd(to_dev(x32), w.eps)
    ref = oracle.sthosvd(xh, w.eps)
    assert res.ranks == ref.ranks
    for k in range(3):
        lam = res.eigvals[k].cpu().numpy()
        # after the first mode the working tensor carries FP32 rounding
        assert np.all(np.abs(lam - ref.eigvals[k]) <= 1e-5 * ref.eigvals[k][0])


def test_reconstruct_matches_oracle_and_subtensor():
    x = synth.planted_tucker((30, 20, 10), (4, 3, 2), rho=0.8, noise=1e-3, seed=9).numpy()
    ref = oracle.sthosvd(x, 1e-2)
    core = to_dev(ref.core)
    facs = [tucker.empty_colmajor(u.shape[0], u.shape[1], "cuda:0").copy_(torch.as_tensor(u))
            for u in ref.factors]
    xg = tucker.reconstruct(core, facs)
    xr = oracle.reconstruct(ref.core, ref.factors)
    tol = 64 * U64 * np.abs(xr).max() * 30
    assert np.abs(to_host(xg) - xr).max() <= tol
    # subtensor from row subsets (Sec. II-C): rows 5..14 of mode 1, rows 3..5 of mode 3
    sub = [facs[0][5:15], facs[1], facs[2][3:6]]
    xs = tucker.reconstruct(core, sub)
    assert np.abs(to_host(xs) - xr[5:15, :, 3:6]).max() <= tol


def test_invalid_on_device_inputs_raise():
    x = to_dev(synth.random_tensor((8, 8), seed=1))
    with pytest.raises(tucker.TuckerError):
        tucker.sthosvd(x, -1.0)
    bad = x.clone()
    bad[3, 3] = float("nan")
    with pytest.raises(tucker.TuckerError) as e:
        tucker.sthosvd(bad, 1e-3)
    assert e.value.status == -5
