"""Pins for the FP64 CPU oracle, against facts that do not come from the oracle.

Each check is chosen so that a plausible slip (a wrong unfolding index, a
transposed operand, a dropped term, a wrong sign in a rotation, an off-by-one
in the rank rule) fails at least one of them:

* the unfolding figure of Sec. IV-C (golden file) and its block structure;
* TTM through numpy's tensordot (an independent contraction), the unfolded
  identity and commutativity of products in different modes (Sec. II-A);
* Gram trace = squared norm, brute-force M M^T from a numpy-built unfolding;
* Jacobi eigenpairs against closed forms and LAPACK's eigh;
* the rank rule on hand-worked spectra (Alg. 1);
* whole ST-HOSVD: the N=2 closed form (Eckart-Young), rank-one and
  superdiagonal tensors, the fit identity (Sec. II-B), the error bound
  (Sec. VII-B), planted ranks, equivariance;
* the compression ratio against Table II.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def np_unfold(x, n):
    """Independent unfolding: move mode n first, then flatten the rest with
    the remaining modes in increasing order, first one fastest."""
    return np.reshape(np.moveaxis(x, n, 0), (x.shape[n], -1), order="F")


def np_ttm(x, n, v):
    return np.moveaxis(np.tensordot(v, x, axes=([1], [n])), 0, n)


def rng_tensor(shape, seed):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(shape))


# ---------------------------------------------------------------- unfolding

def test_unfolding_matches_paper_figure():
    expect = {}
    with open(os.path.join(GOLDEN, "unfold_2x2x2x2.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            head, vals = line.split(":")
            mode, row = (int(t) for t in head.split())
            expect[(mode, row)] = [int(v) for v in vals.split()]
    x = np.arange(16, dtype=float).reshape((2, 2, 2, 2), order="F")
    for mode in range(1, 5):
        m = oracle.unfold(x, mode - 1)
        for row in range(2):
            assert m[row].astype(int).tolist() == expect[(mode, row)]


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 4, 5), (5, 1, 3, 2, 2), (7,)])
def test_unfolding_block_structure(shape):
    """Sec. IV-C: the mode-n unfolding is prod_{m>n} block columns, each a
    row-major J_n x prod_{m<n} J_m block of consecutive memory."""
    x = np.arange(int(np.prod(shape)), dtype=float).reshape(shape, order="F")
    for n in range(len(shape)):
        m = oracle.unfold(x, n)
        lo = int(np.prod(shape[:n]))
        hi = int(np.prod(shape[n + 1:]))
        jn = shape[n]
        for b in range(hi):
            blk = m[:, b * lo:(b + 1) * lo]
            start = b * lo * jn
            assert np.array_equal(blk, start + np.arange(jn * lo).reshape(jn, lo))
        assert np.array_equal(m, np_unfold(x, n))


def test_fold_inverts_unfold():
    x = rng_tensor((3, 4, 2, 5), 1)
    for n in range(4):
        assert np.array_equal(oracle.fold(oracle.unfold(x, n), n, x.shape), x)


# --------------------------------------------------------------------- TTM

@pytest.mark.parametrize("shape,n,k", [((4, 5, 6), 0, 3), ((4, 5, 6), 1, 7), ((4, 5, 6), 2, 2),
                                       ((4, 5, 6), 1, 5), ((3, 2, 4, 5), 2, 6), ((6,), 0, 2)])
def test_ttm_against_tensordot(shape, n, k):
    x = rng_tensor(shape, 2)
    v = np.random.default_rng(3).standard_normal((k, shape[n]))
    z = oracle.ttm(x, n, v)
    assert z.shape == tuple(k if i == n else d for i, d in enumerate(shape))
    np.testing.assert_allclose(z, np_ttm(x, n, v), rtol=1e-13, atol=1e-13)
    # unfolded identity Z_(n) = V X_(n)
    np.testing.assert_allclose(oracle.unfold(z, n), v @ np_unfold(x, n), rtol=1e-13, atol=1e-13)


def test_ttm_commutes_across_modes():
    x = rng_tensor((4, 3, 5), 4)
    w = np.random.default_rng(5).standard_normal((2, 4))
    v = np.random.default_rng(6).standard_normal((6, 5))
    a = oracle.ttm(oracle.ttm(x, 0, w), 2, v)
    b = oracle.ttm(oracle.ttm(x, 2, v), 0, w)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13)


def test_ttm_closed_forms():
    x = rng_tensor((3, 4, 2), 7)
    np.testing.assert_array_equal(oracle.ttm(x, 1, np.eye(4)), x)
    ones = np.ones((1, 4))
    np.testing.assert_allclose(oracle.ttm(x, 1, ones)[:, 0, :], x.sum(axis=1), rtol=1e-14)
    sel = np.zeros((1, 3)); sel[0, 2] = 1.0  # picks the i_1 = 2 slice
    np.testing.assert_array_equal(oracle.ttm(x, 0, sel)[0], x[2])


def test_ttm_entry_matches_ttm():
    x = rng_tensor((4, 3, 5, 2), 8)
    v = np.random.default_rng(9).standard_normal((3, 5))
    z = oracle.ttm(x, 2, v)
    for idx in [(0, 0, 0, 0), (3, 2, 2, 1), (1, 1, 1, 0)]:
        assert math.isclose(oracle.ttm_entry(x, 2, v, idx), z[idx], rel_tol=1e-13, abs_tol=1e-14)


# -------------------------------------------------------------------- Gram

@pytest.mark.parametrize("shape", [(5, 4, 3), (2, 3, 4, 5), (9,), (1, 6)])
def test_gram_trace_and_brute_force(shape):
    x = rng_tensor(shape, 10)
    nrm2 = float(np.sum(x * x))
    assert math.isclose(oracle.norm2(x), nrm2, rel_tol=1e-14)
    for n in range(len(shape)):
        s = oracle.gram(x, n)
        m = np_unfold(x, n)
        np.testing.assert_allclose(s, m @ m.T, rtol=1e-12, atol=1e-12)
        assert np.array_equal(s, s.T)
        assert math.isclose(np.trace(s), nrm2, rel_tol=1e-13)
        for a, b in [(0, 0), (0, shape[n] - 1), (shape[n] - 1, shape[n] - 1)]:
            assert math.isclose(oracle.gram_entry(x, n, a, b), s[a, b], rel_tol=1e-12,
                                abs_tol=1e-12)


# ------------------------------------------------------------------ Jacobi

def test_jacobi_two_by_two_closed_form():
    a, b, c = 3.0, 1.5, -2.0
    lam, v, _ = oracle.sym_eig(np.array([[a, b], [b, c]]))
    mid, rad = (a + c) / 2, math.hypot((a - c) / 2, b)
    np.testing.assert_allclose(lam, [mid + rad, mid - rad], rtol=1e-15)
    # eigenvector of the larger eigenvalue is proportional to (b, lam - a)
    e = np.array([b, lam[0] - a]); e /= np.linalg.norm(e)
    assert abs(abs(e @ v[:, 0]) - 1) < 1e-15


def test_jacobi_known_spectrum_and_eigh():
    rng = np.random.default_rng(11)
    j = 40
    q, _ = np.linalg.qr(rng.standard_normal((j, j)))
    spec = np.sort(rng.uniform(-3, 5, j))[::-1]
    s = (q * spec) @ q.T
    s = (s + s.T) / 2
    lam, v, sweeps = oracle.sym_eig(s)
    assert 1 <= sweeps <= 20
    np.testing.assert_allclose(lam, spec, atol=1e-13)
    np.testing.assert_allclose(lam, np.linalg.eigvalsh(s)[::-1], atol=1e-13)
    np.testing.assert_allclose(v.T @ v, np.eye(j), atol=1e-13)
    np.testing.assert_allclose(s @ v, v * lam, atol=1e-12)
    # each eigenvector matches the planted one up to sign
    for k in range(j):
        assert abs(abs(v[:, k] @ q[:, k]) - 1) < 1e-11


def test_jacobi_sign_rule_and_degenerate():
    lam, v, _ = oracle.sym_eig(np.diag([1.0, 5.0, 3.0]))
    np.testing.assert_array_equal(lam, [5.0, 3.0, 1.0])
    np.testing.assert_array_equal(v, np.eye(3)[:, [1, 2, 0]])
    lam, v, _ = oracle.sym_eig(-np.eye(2)[:, ::-1])  # [[0,-1],[-1,0]], eigenvalues 1, -1
    np.testing.assert_allclose(lam, [1, -1], atol=1e-15)
    for k in range(2):
        col = v[:, k]
        assert col[np.argmax(np.abs(col))] > 0
    lam, v, _ = oracle.sym_eig(np.zeros((3, 3)))
    np.testing.assert_array_equal(lam, 0)


# -------------------------------------------------------------- rank rule

def test_truncation_rule_hand_cases():
    lam = np.array([4.0, 2.0, 1.0, 0.5])
    assert oracle.truncate(lam, 1.5) == (2, 1.5)       # inclusive <=
    assert oracle.truncate(lam, 1.49) == (3, 0.5)
    assert oracle.truncate(lam, 100.0) == (1, 3.5)     # never below 1
    assert oracle.truncate(lam, 0.0) == (4, 0.0)
    assert oracle.truncate(np.array([3.0, 1.0, 0.0, 0.0]), 0.0) == (2, 0.0)
    assert oracle.truncate(np.array([3.0, 1.0, -1e-20]), 0.0) == (2, 0.0)  # clamp
    assert oracle.truncate(lam, 0.0, fixed_rank=3) == (3, 0.5)


# ---------------------------------------------------------------- ST-HOSVD

def test_sthosvd_two_way_closed_form():
    """N = 2: ST-HOSVD is a truncated SVD (Eckart-Young)."""
    rng = np.random.default_rng(12)
    i1, i2 = 30, 20
    uu, _ = np.linalg.qr(rng.standard_normal((i1, i2)))
    vv, _ = np.linalg.qr(rng.standard_normal((i2, i2)))
    sig = 0.6 ** np.arange(i2)
    x = np.asfortranarray((uu * sig) @ vv.T)
    nu = float(np.sum(sig ** 2))
    for eps in [1e-1, 3e-2, 1e-3]:
        tau = eps * eps * nu / 2
        tails = np.array([np.sum(sig[r:] ** 2) for r in range(i2 + 1)])
        r1 = next(r for r in range(1, i2 + 1) if tails[r] <= tau)
        tails2 = np.array([np.sum(sig[r:r1] ** 2) for r in range(r1 + 1)])
        r2 = next(r for r in range(1, r1 + 1) if tails2[r] <= tau)
        res = oracle.sthosvd(x, eps)
        assert res.ranks == (r1, r2)
        xh = oracle.reconstruct(res.core, res.factors)
        best = (uu[:, :r2] * sig[:r2]) @ vv[:, :r2].T
        np.testing.assert_allclose(xh, best, atol=1e-12)
        e2, _, n2 = oracle.error_metrics(x, xh)
        assert math.isclose(e2 / n2, np.sum(sig[r2:] ** 2) / nu, rel_tol=1e-9, abs_tol=1e-15)
        np.testing.assert_allclose(res.eigvals[0], np.r_[sig ** 2, np.zeros(i1 - i2)],
                                   atol=1e-13)


def test_sthosvd_rank_one():
    rng = np.random.default_rng(13)
    a, b, c = rng.standard_normal(6), rng.standard_normal(7), rng.standard_normal(5)
    s = 2.5
    x = np.asfortranarray(s * np.einsum("i,j,k->ijk", a, b, c))
    res = oracle.sthosvd(x, 1e-6)
    assert res.ranks == (1, 1, 1)
    expect = s * np.linalg.norm(a) * np.linalg.norm(b) * np.linalg.norm(c)
    assert math.isclose(abs(res.core.item()), expect, rel_tol=1e-13)
    xh = oracle.reconstruct(res.core, res.factors)
    np.testing.assert_allclose(xh, x, atol=1e-13)


def test_sthosvd_superdiagonal():
    d = np.array([5.0, 3.0, 2.0, 1.0, 0.5])
    i = 7
    x = np.zeros((i, i, i), order="F")
    for r, v in enumerate(d):
        x[r, r, r] = v
    nu = float(np.sum(d ** 2))
    res = oracle.sthosvd(x, 0.0)
    for n in range(3):  # every mode spectrum is d^2 padded with zeros
        np.testing.assert_allclose(res.eigvals[n][:5], d ** 2, rtol=1e-15)
    assert res.ranks == (5, 5, 5)
    # eps with eps^2 nu / 3 between 0.25 and 1.25 keeps 4 components in every mode
    eps = math.sqrt(3 * 0.5 / nu)
    res = oracle.sthosvd(x, eps)
    assert res.ranks == (4, 4, 4)
    assert math.isclose(res.discarded[0], 0.25, rel_tol=1e-14)
    assert res.discarded[1] == 0.0 and res.discarded[2] == 0.0
    for n in range(3):
        np.testing.assert_allclose(np.abs(res.factors[n]), np.eye(i)[:, :4], atol=1e-15)


def _check_invariants(x, res, eps, tol_fit=1e-13, budget=True):
    nu = res.norm2
    assert math.isclose(nu, float(np.sum(x.astype(np.float64) ** 2)), rel_tol=1e-12)
    xh = oracle.reconstruct(res.core, res.factors)
    e2, _, _ = oracle.error_metrics(x, xh)
    g2 = float(np.sum(res.core ** 2))
    disc = float(np.sum(res.discarded))
    # fit identity (Sec. II-B) and ST-HOSVD error = sum of discarded eigenvalues
    assert abs((nu - g2) - e2) <= tol_fit * nu
    assert abs(disc - e2) <= tol_fit * nu
    # each discarded tail is within the per-mode budget; total within eps^2 nu
    if budget:
        assert np.all(res.discarded <= eps * eps * nu / x.ndim * (1 + 1e-12))
        assert e2 <= eps * eps * nu * (1 + 1e-9) + tol_fit * nu
    for u in res.factors:
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_planted_rank_recovery_32cube(seed):
    w = synth.WORKLOADS["planted32"]
    x = w.make(seed=seed).numpy()
    res = oracle.sthosvd(x, w.eps)
    assert res.ranks == w.ranks
    _check_invariants(x, res, w.eps)
    e2, _, n2 = oracle.error_metrics(x, oracle.reconstruct(res.core, res.factors))
    rel = math.sqrt(e2 / n2)
    # the residual is the noise outside a 120-dimensional subspace of 32768
    assert 0.98 * w.noise < rel < 1.0 * w.noise


def test_spectra_match_brute_force_svd():
    """lambda^(n) = squared singular values of the working tensor's unfolding;
    span(U_n) = its leading left singular subspace."""
    x = synth.planted_tucker((10, 9, 8, 7), (3, 4, 2, 3), rho=0.7, noise=1e-3, seed=21).numpy()
    eps = 1e-2
    order = (2, 0, 3, 1)
    res = oracle.sthosvd(x, eps, order=order)
    y = np.array(x)
    for n in order:
        m = np_unfold(y, n)
        uu, sv, _ = np.linalg.svd(m, full_matrices=False)
        lam = np.zeros(y.shape[n]); lam[:sv.size] = sv ** 2
        np.testing.assert_allclose(res.eigvals[n], lam, atol=1e-12 * lam[0])
        r = res.ranks[n]
        p_orc = res.factors[n] @ res.factors[n].T
        p_svd = uu[:, :r] @ uu[:, :r].T
        np.testing.assert_allclose(p_orc, p_svd, atol=1e-9)
        tau = eps * eps * res.norm2 / x.ndim
        tails = [np.sum(lam[k:]) for k in range(lam.size + 1)]
        assert r == next(k for k in range(1, lam.size + 1) if tails[k] <= tau)
        y = np_ttm(y, n, res.factors[n].T)
    np.testing.assert_allclose(res.core, y, atol=1e-12)


def test_invariants_on_unstructured_tensor():
    x = rng_tensor((6, 5, 7, 4), 30)
    for eps in [0.3, 0.1, 0.0]:
        res = oracle.sthosvd(x, eps)
        _check_invariants(x, res, eps)


def test_equivariance():
    x = synth.planted_tucker((8, 7, 6), (3, 2, 3), rho=0.8, noise=1e-4, seed=31).numpy()
    eps = 1e-3
    base = oracle.sthosvd(x, eps)
    # orthogonal change of basis on mode 1
    q, _ = np.linalg.qr(np.random.default_rng(32).standard_normal((7, 7)))
    xq = np_ttm(x, 1, q)
    rq = oracle.sthosvd(xq, eps)
    assert rq.ranks == base.ranks
    for n in range(3):
        np.testing.assert_allclose(rq.eigvals[n], base.eigvals[n], atol=1e-12)
    uq = q @ base.factors[1]
    np.testing.assert_allclose(rq.factors[1] @ rq.factors[1].T, uq @ uq.T, atol=1e-10)
    # scaling: eigenvalues scale by c^2, ranks unchanged
    c = 3.0
    rc = oracle.sthosvd(c * x, eps)
    assert rc.ranks == base.ranks
    for n in range(3):
        np.testing.assert_allclose(rc.eigvals[n], c * c * base.eigvals[n], rtol=1e-12,
                                   atol=1e-12 * c * c * base.eigvals[n][0])
    # permuting the modes together with the order permutes every output
    perm = (2, 0, 1)
    xp = np.asfortranarray(np.transpose(x, perm))
    rp = oracle.sthosvd(xp, eps, order=(1, 2, 0))  # same processing sequence as 0,1,2
    for k, m in enumerate(perm):
        assert rp.ranks[k] == base.ranks[m]
        np.testing.assert_allclose(rp.eigvals[k], base.eigvals[m], atol=1e-12)
    np.testing.assert_allclose(np.abs(rp.core), np.abs(np.transpose(base.core, perm)),
                               atol=1e-12)


def test_threshold_uses_original_norm_and_full_mode_count():
    """tau = eps^2 ||X||^2 / N for every mode, whatever the order (Alg. 1)."""
    x = rng_tensor((5, 6, 4), 40)
    eps = 0.4
    nu = float(np.sum(x * x))
    for order in [(0, 1, 2), (2, 1, 0)]:
        res = oracle.sthosvd(x, eps, order=order)
        tau = eps * eps * nu / 3
        for n in order:
            lam = np.maximum(res.eigvals[n], 0)
            tails = [np.sum(lam[k:]) for k in range(lam.size + 1)]
            assert res.ranks[n] == next(k for k in range(1, lam.size + 1) if tails[k] <= tau)


def test_fixed_ranks():
    x = rng_tensor((6, 5, 4), 41)
    res = oracle.sthosvd(x, 0.0, ranks=(2, 3, 1))
    assert res.ranks == (2, 3, 1)
    assert res.core.shape == (2, 3, 1)
    _check_invariants(x, res, 0.0, budget=False)


def test_compression_ratio_table2():
    rows = []
    with open(os.path.join(GOLDEN, "table2_ranks.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, dims, ranks, printed = (t.strip() for t in line.split("|"))
            rows.append((name, [int(v) for v in dims.split()], [int(v) for v in ranks.split()],
                         int(printed)))
    assert len(rows) == 3
    for name, dims, ranks, printed in rows:
        c = oracle.compression_ratio(dims, ranks)
        assert round(c) == printed, (name, c)


def test_error_metrics_hand_cases():
    """Table II's two error columns on hand-worked tensors (all values exact
    in binary).  The largest deviation is negative (X~ above X), sits away
    from the largest |X| and from the largest |X~|, and in the later cases at
    the first and at the last element, so a missing absolute value, a maximum
    taken over X or X~ instead of X - X~, a signed maximum or a loop that
    skips an end element each give a different max-abs value."""
    # 2 x 2 x 2, Fortran order: element k of the flat array is offset k
    x = np.asfortranarray(np.array([5.0, -1.0, 2.0, 0.5, -3.0, 0.25, 1.5, 0.0])
                          .reshape((2, 2, 2), order="F"))
    xh = np.asfortranarray(np.array([4.75, -1.0, 2.75, 0.5, -3.0, 0.0, 1.5, 0.125])
                           .reshape((2, 2, 2), order="F"))
    e2, mx, n2 = oracle.error_metrics(x, xh)
    # X - X~ = [0.25, 0, -0.75, 0, 0, 0.25, 0, -0.125]
    assert mx == 0.75
    assert e2 == 0.0625 + 0.5625 + 0.0625 + 0.015625
    assert n2 == 25.0 + 1.0 + 4.0 + 0.25 + 9.0 + 0.0625 + 2.25
    # largest deviation at the first element, negative; |X| largest elsewhere
    a = np.array([1.0, 8.0, -2.0, 0.5, 0.0, -0.5])
    b = np.array([2.5, 8.0, -2.0, 0.25, -0.5, 0.0])
    e2, mx, n2 = oracle.error_metrics(np.asfortranarray(a.reshape(2, 3, order="F")),
                                      np.asfortranarray(b.reshape(2, 3, order="F")))
    assert (mx, e2, n2) == (1.5, 2.25 + 0.0625 + 0.25 + 0.25, 1.0 + 64.0 + 4.0 + 0.25 + 0.25)
    # largest deviation at the last element, negative
    a = np.array([3.0, -4.0, 0.0, 1.0])
    b = np.array([3.0, -4.0, 0.5, 3.0])
    e2, mx, n2 = oracle.error_metrics(np.asfortranarray(a.reshape(2, 2, order="F")),
                                      np.asfortranarray(b.reshape(2, 2, order="F")))
    assert (mx, e2, n2) == (2.0, 0.25 + 4.0, 9.0 + 16.0 + 1.0)
    # X~ = X gives zero error; the metrics are symmetric only in the first two
    e2, mx, n2 = oracle.error_metrics(x, x)
    assert (e2, mx) == (0.0, 0.0)
    e2b, mxb, n2b = oracle.error_metrics(xh, x)
    e2a, mxa, _ = oracle.error_metrics(x, xh)
    assert (e2b, mxb) == (e2a, mxa) and n2b == float(np.sum(xh * xh))


def test_synthetic_generator_contract():
    """The generator's planted part has exactly the requested multilinear
    rank and the noise has the requested relative size."""
    x, core, factors = synth.planted_tucker((9, 8, 7), (2, 3, 4), rho=0.5, noise=0.0, seed=3,
                                            return_parts=True)
    xn = x.numpy()
    for n, r in enumerate((2, 3, 4)):
        sv = np.linalg.svd(np_unfold(xn, n), compute_uv=False)
        assert sv[r - 1] > 1e-8 * sv[0] and sv[r] < 1e-12 * sv[0]
        np.testing.assert_allclose(factors[n].T @ factors[n], np.eye(r), atol=1e-14)
    assert math.isclose(np.linalg.norm(xn), torch.linalg.vector_norm(core).item(), rel_tol=1e-12)
    xe = synth.planted_tucker((9, 8, 7), (2, 3, 4), rho=0.5, noise=1e-3, seed=3).numpy()
    assert math.isclose(np.linalg.norm(xe - xn) / np.linalg.norm(xn), 1e-3, rel_tol=1e-9)
