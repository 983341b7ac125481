"""Parity at the benchmark's full size (combustion128: 128x128x128x32x32,
17.2 GB in FP64, 8.6 GB in FP32), in the configuration bench.py times.

The oracle cannot process the whole tensor in a test's time, so it checks
what it can compute one by one -- Gram entries of mode 1 from two-row slices
of the unfolding, TTM output columns from single input columns -- and the
run is checked against properties that hold at any size: the planted ranks,
the identity ||X||^2 - ||G||^2 = sum of discarded eigenvalues = ||X - X~||^2
(ST-HOSVD, from orthogonality of the factors), orthonormal factors, and for
the mixed path ranks equal to the FP64 path's with every discarded sum and
the relative error within the bounds derived from the split Gram's reported
representation error and the TTMs' arithmetic (gpu_util.carried_errors).

The precision configuration (the same tensor stored FP32 at eps 1e-3 and
1e-5, split-bf16 Gram, bf16 or split-bf16 TTM) is checked against the FP64
path on the same FP32 data, which the parity tests tie to the oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1510_06689_amd import tucker
from gpu_util import U32, U64, check_against_oracle, mode1_rows, say, split_gram_bound

pytestmark = pytest.mark.gpu

W = synth.WORKLOADS["combustion128"]
PAIRS = [(0, 0), (3, 77), (64, 1), (127, 127), (90, 91)]
COLS = [0, 1, 12345, 2**23 + 7, 2**24 - 1]   # mode-1 columns (other-mode multi-index)


@pytest.fixture(scope="module")
def tensors():
    say(f"generating {W.name} {W.dims}")
    x64 = W.make(dtype=torch.float64, device="cuda:0")
    x32 = tucker.empty_fortran(W.dims, torch.float32, "cuda:0")
    x32.copy_(x64)
    torch.cuda.synchronize()
    yield x64, x32
    del x64, x32
    torch.cuda.empty_cache()


@pytest.mark.parametrize("path", ["fp64", "mixed"])
def test_fullsize_mode1_gram_entries(tensors, path):
    x = tensors[0] if path == "fp64" else tensors[1]
    prec = "fp64" if path == "fp64" else "split_bf16"
    s, sumsq = tucker.gram(x, 0, precision=prec)
    torch.cuda.synchronize()
    s = s.cpu().numpy()
    k = x.numel() // x.shape[0]
    for i, j in PAIRS:
        sub = mode1_rows(x, i, j)
        ref = oracle.gram(sub, 0)                       # [[S_ii, S_ij], [S_ji, S_jj]]
        d = np.sqrt(np.diag(ref))
        tol = (k + 2) * U64 * np.outer(d, d)
        if path == "mixed":
            tol = tol + split_gram_bound(sub)
        got = np.array([[s[i, i], s[i, j]], [s[j, i], s[j, j]]])
        say(f"{path} S[{i},{j}] = {got[0, 1]:.12e} oracle {ref[0, 1]:.12e}")
        assert np.all(np.abs(got - ref) <= tol), (i, j, got - ref, tol)


@pytest.mark.parametrize("path", ["fp64", "mixed"])
def test_fullsize_mode1_ttm_columns(tensors, path):
    x = tensors[0] if path == "fp64" else tensors[1]
    prec = "fp64" if path == "fp64" else "bf16x3"
    rng = np.random.default_rng(7)
    u = np.linalg.qr(rng.standard_normal((x.shape[0], 16)))[0]        # orthonormal, J x R
    ud = tucker.empty_colmajor(u.shape[0], u.shape[1], "cuda:0").copy_(torch.as_tensor(u))
    z = tucker.ttm(x, 0, ud, transpose=True, precision=prec)          # 16 x 128 x .. x 32
    torch.cuda.synchronize()
    xf = x.permute(*reversed(range(x.dim()))).reshape(-1, x.shape[0])   # column c -> row c
    zf = z.permute(*reversed(range(z.dim()))).reshape(-1, z.shape[0])
    ycols = xf[COLS].double().cpu().numpy().T                          # 128 x ncols
    zcols = zf[COLS].double().cpu().numpy().T
    ref = oracle.ttm(np.asfortranarray(ycols), 0, u.T)                   # Z_(1) = U^T Y_(1)
    absprod = oracle.ttm(np.asfortranarray(np.abs(ycols)), 0, np.abs(u.T))
    if path == "fp64":
        tol = 130 * U64 * absprod
    else:
        tol = (4 * 2.0**-16 + 16 * 2.0**-24) * absprod + U32 * np.abs(ref)
    assert np.all(np.abs(zcols - ref) <= tol + 1e-300), np.max(np.abs(zcols - ref) / (tol + 1e-300))


def _check_invariants(x, res, eps, tol_rel, tol_norm):
    nu = res.norm2
    g2 = float((res.core.double() ** 2).sum().item())
    disc = float(sum(res.discarded))
    xh = tucker.reconstruct(res.core, res.factors)
    e2, _, n2 = tucker.error_metrics(x, xh)
    del xh
    torch.cuda.empty_cache()
    assert math.isclose(n2, nu, rel_tol=tol_norm)   # ||X||^2: error metric vs first Gram's trace
    assert abs((nu - g2) - disc) <= tol_rel * nu, (nu - g2, disc)
    assert abs(e2 - disc) <= tol_rel * nu, (e2, disc)
    assert math.sqrt(e2 / nu) <= eps
    for u in res.factors:
        ut = u.cpu().numpy()
        assert np.abs(ut.T @ ut - np.eye(ut.shape[1])).max() <= 1e-12
    return math.sqrt(e2 / nu)


def test_fullsize_sthosvd_fp64_and_mixed(tensors):
    x64, x32 = tensors
    r64 = tucker.sthosvd(x64, W.eps)
    assert r64.ranks == W.ranks
    rel64 = _check_invariants(x64, r64, W.eps, 64 * U64 * 100, 1e-12)
    rm = tucker.sthosvd(x32, W.eps, gram_precision="split_bf16", ttm_precision="bf16x3")
    say(f"ranks fp64 {r64.ranks} mixed {rm.ranks} fp64-redone modes {rm.fp64_modes}")
    assert rm.ranks == r64.ranks
    # FP32 storage and split products: the identity holds to the TTMs' ~2^-17,
    # and the first Gram's trace carries the split's ~2^-16 / sqrt(K) relative error
    relm = _check_invariants(x32, rm, W.eps, 1e-6, 1e-6)
    say(f"relerr fp64 {rel64:.6e} mixed {relm:.6e}; bounds {rm.tail_error_bound}")
    # the FP64 run reads the FP64 tensor: the inputs differ by its FP32 rounding
    tol = check_against_oracle(rm, r64, W.dims, None, rm.ttm_precision, relm, rel64, e0=U32)
    assert tol <= len(W.dims) * W.eps ** 2 / len(W.dims)


def _relerr(x, res):
    xh = tucker.reconstruct(res.core, res.factors)
    e2, _, n2 = tucker.error_metrics(x, xh)
    del xh
    torch.cuda.empty_cache()
    return math.sqrt(e2 / n2)


@pytest.mark.parametrize("eps", [1e-3, 1e-5])
def test_fullsize_precision_config(tensors, eps):
    """The precision configuration on the full FP32 tensor: split-bf16 Gram
    with split-bf16 TTM, and with the bf16 TTM the configuration names, which
    the eps rule raises (its ~2^-8 output error would reach the threshold:
    to split-bf16 at eps = 1e-3, to FP64 arithmetic at 1e-5); ranks equal the
    FP64 path's on the same FP32 data (and the planted ranks at 1e-3), every
    discarded sum and the error within the derived bounds.  With the FP64
    path's ranks fixed, the bf16 TTM runs as requested and its end-to-end
    error is stated and held to its own bound."""
    x32 = tensors[1]
    r64 = tucker.sthosvd(x32, eps, gram_precision="fp64", ttm_precision="fp64")
    rel64 = _relerr(x32, r64)
    say(f"eps {eps}: fp64 path on FP32 data ranks {r64.ranks} relerr {rel64:.6e}")
    if eps == 1e-3:
        assert r64.ranks == W.ranks
    assert rel64 <= eps
    raised = "bf16x3" if eps == 1e-3 else "fp64"
    for ttm, expect in (("bf16x3", "bf16x3" if eps == 1e-3 else "fp64"), ("bf16", raised)):
        rm = tucker.sthosvd(x32, eps, gram_precision="split_bf16", ttm_precision=ttm)
        relm = _relerr(x32, rm)
        say(f"  split gram, ttm {ttm} (ran {rm.ttm_precision}): ranks {rm.ranks} redone "
            f"{rm.fp64_modes} relerr {relm:.6e} (|d| {abs(relm - rel64):.3e})")
        assert rm.ttm_precision == expect
        assert relm <= eps
        # both runs store their intermediate tensors in FP32
        check_against_oracle(rm, r64, W.dims, None, rm.ttm_precision, relm, rel64,
                             storage_u=U32 * math.sqrt(2))
    rf = tucker.sthosvd(x32, 0.0, ranks=r64.ranks, gram_precision="split_bf16",
                        ttm_precision="bf16")
    relf = _relerr(x32, rf)
    say(f"  fixed ranks, bf16 ttm as requested: relerr {relf:.6e} vs {rel64:.6e} "
        f"(|d| {abs(relf - rel64):.3e})")
    assert rf.ttm_precision == "bf16" and rf.ranks == r64.ranks
    check_against_oracle(rf, r64, W.dims, None, "bf16", relf, rel64,
                         storage_u=U32 * math.sqrt(2))


def test_fullsize_mode1_qr_r_gram_identity(tensors):
    # R of the 2^24 x 128 mode-1 unfolding (FP32 storage, the QR leg's input):
    # (R^T R)_ij equals the Gram entry S_ij up to Householder's columnwise
    # backward error, |d(R^T R)_ij| <= 2 gamma ||a_i|| ||a_j||
    x = tensors[1]
    r, sumsq = tucker.qr_r(x, 0)
    torch.cuda.synchronize()
    r = r.cpu().numpy()
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) >= 0)
    rtr = r.T @ r
    gamma = 4096 * U64
    for i, j in PAIRS:
        sub = mode1_rows(x, i, j)
        ref = oracle.gram(sub, 0)
        d = np.sqrt(np.diag(ref))
        got = np.array([[rtr[i, i], rtr[i, j]], [rtr[j, i], rtr[j, j]]])
        tol = 2 * gamma * np.outer(d, d) + 64 * U64 * np.outer(d, d)
        say(f"qr (R^T R)[{i},{j}] = {got[0, 1]:.12e} oracle {ref[0, 1]:.12e}")
        assert np.all(np.abs(got - ref) <= tol), (i, j, got - ref, tol)
    nu = float(np.trace(rtr))
    assert math.isclose(float(sumsq), nu, rel_tol=1e-12)


def test_fullsize_qr_path_eps_1e5(tensors):
    # the bench's QR leg: eps = 1e-5 on the FP32-stored tensor, QR path and
    # FP64 Gram path; ranks equal, ST-HOSVD identities on both
    x32 = tensors[1]
    eps = 1e-5
    rq = tucker.sthosvd(x32, eps, gram_precision="qr")
    rg = tucker.sthosvd(x32, eps, gram_precision="fp64")
    say(f"eps 1e-5 ranks qr {rq.ranks} fp64 gram {rg.ranks}")
    assert rq.ranks == rg.ranks
    # FP32 storage of the intermediate tensors bounds the identities at ~u32
    relq = _check_invariants(x32, rq, eps, 1e-6, 1e-9)
    relg = _check_invariants(x32, rg, eps, 1e-6, 1e-9)
    say(f"relerr qr {relq:.6e} fp64 gram {relg:.6e}")
    assert abs(relq - relg) <= 1e-3 * eps
    # the leading singular values agree (sigma from QR vs sqrt of the Gram's eigenvalues)
    sq = np.sqrt(np.maximum(rq.eigvals[0].cpu().numpy(), 0))
    sg = np.sqrt(np.maximum(rg.eigvals[0].cpu().numpy(), 0))
    s1 = math.sqrt(rq.norm2)
    assert np.abs(sq[:20] - sg[:20]).max() <= 1e-9 * s1
