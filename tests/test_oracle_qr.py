"""Pins for the oracle's QR-preprocessed SVD path (Sec. IX), against facts that
do not come from the oracle.

* Householder R against closed forms: A = Q T with Q from a Sylvester
  Hadamard matrix (orthonormal columns, exact in binary) and T upper
  triangular, so R = D T with D the diagonal sign matrix; the m < j case;
  a zero column; the identity R^T R = A^T A.
* One-sided Jacobi SVD against B = Q1 diag(sigma) Q2^T with exact orthogonal
  Q1, Q2 and singular values spread over 45 binary orders of magnitude, and
  against LAPACK's SVD on random matrices.
* ST-HOSVD through QR on a tensor whose per-mode spectra are known exactly
  (superdiagonal core, Hadamard factors) at eps near sqrt(u): exact ranks,
  tail sums and spectra; the fit identity; agreement with the Gram path of
  the oracle where both are accurate (eps well above sqrt(u)).
A transposed operand, a wrong reflector sign, a dropped row sign or a
rotation applied to the wrong side fails at least one of these.
"""
import numpy as np
import pytest
from scipy.linalg import hadamard

import oracle
import synth

U = np.finfo(np.float64).eps


def orthonormal_columns(m, j):
    """First j columns of a Sylvester Hadamard matrix of order m (a power of
    4), scaled to unit norm: exactly representable, exactly orthonormal."""
    h = hadamard(m).astype(np.float64) / np.sqrt(m)
    assert np.sqrt(m) == int(np.sqrt(m))
    return h[:, :j]


def test_qr_r_closed_form_with_signs():
    m, j = 64, 8
    q = orthonormal_columns(m, j)
    t = np.triu(np.arange(1, j * j + 1, dtype=np.float64).reshape(j, j) % 7 - 3)
    np.fill_diagonal(t, [5, -3, 2, -7, 1, 4, -2, 6])
    a = q @ t  # exact: entries are sums of +-t/8
    d = np.sign(np.diag(t))
    r = oracle.qr_r(a)
    np.testing.assert_allclose(r, d[:, None] * t, rtol=0, atol=1e-13 * np.abs(t).max())
    assert np.all(np.diag(r) >= 0)
    assert np.all(np.tril(r, -1) == 0)


def test_qr_r_wide_matrix():
    m, j = 4, 6
    q = orthonormal_columns(4, 4)
    t = np.triu(np.array([[3, 1, -2, 0, 1, 2],
                          [0, 2, 1, 1, -1, 0],
                          [0, 0, 4, -1, 2, 1],
                          [0, 0, 0, 1, 3, -2]], dtype=np.float64))
    a = q @ t
    r = oracle.qr_r(a)
    np.testing.assert_allclose(r[:m], t, rtol=0, atol=1e-14 * np.abs(t).max())
    assert np.all(r[m:] == 0)
    np.testing.assert_allclose(r.T @ r, a.T @ a, rtol=0, atol=1e-13)


def test_qr_r_zero_column_and_gram_identity():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((300, 9))
    a[:, 4] = 0.0
    r = oracle.qr_r(a)
    assert np.all(r[:, 4] == 0)
    assert np.all(np.diag(r) >= 0)
    g = a.T @ a
    np.testing.assert_allclose(r.T @ r, g, rtol=0, atol=64 * U * np.abs(g).max())


def test_svd_jacobi_closed_form_wide_range():
    j = 16
    q1 = orthonormal_columns(16, j)
    q2 = hadamard(16).astype(np.float64)[::-1] / 4.0  # rows reversed: still orthogonal
    sig = 2.0 ** (-3.0 * np.arange(j))  # 1 .. 2^-45
    b = (q1 * sig) @ q2.T  # exact: each entry is a sum of distinct powers of two
    s, v, sweeps = oracle.svd_jacobi(b)
    assert sweeps > 0
    np.testing.assert_allclose(s, sig, rtol=0, atol=8 * j * U * sig[0])
    # leading singular vectors: the columns of q2 (every |entry| is 1/4, so
    # the sign rule's tie-break is decided by rounding: compare up to sign)
    for k in range(6):
        assert abs(abs(v[:, k] @ q2[:, k]) - 1.0) < 1e-12
    np.testing.assert_allclose(v.T @ v, np.eye(j), rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape", [(7, 7), (40, 40), (1, 1)])
def test_svd_jacobi_vs_lapack(shape):
    rng = np.random.default_rng(shape[0])
    b = rng.standard_normal(shape)
    s, v, _ = oracle.svd_jacobi(b)
    ref = np.linalg.svd(b, compute_uv=False)
    np.testing.assert_allclose(s, ref, rtol=0, atol=32 * shape[0] * U * ref[0])
    # B V has orthogonal columns of norms s
    bv = b @ v
    np.testing.assert_allclose(bv.T @ bv, np.diag(s * s), rtol=0, atol=1e-12 * ref[0] ** 2)


def planted_superdiagonal(i, g):
    """X = G x_1 Q x_2 Q x_3 Q with a superdiagonal core diag(g) and
    Q = Hadamard(i)/sqrt(i): every unfolding's singular values are |g|."""
    q = orthonormal_columns(i, i)
    core = np.zeros((i, i, i))
    for r, gr in enumerate(g):
        core[r, r, r] = gr
    x = np.einsum("abc,ia,jb,kc->ijk", core, q, q, q)
    return np.asfortranarray(x)


def test_mode_svd_qr_resolves_tiny_singular_values():
    i = 16
    g = 2.0 ** (-2.0 * np.arange(i))  # sigma down to 2^-30 ~ 9e-10
    x = planted_superdiagonal(i, g)
    lam, v, _ = oracle.mode_svd_qr(x, 0)
    s = np.sqrt(lam)
    np.testing.assert_allclose(s, g, rtol=0, atol=64 * U * g[0])
    # relative accuracy of the squared values right down to the tail
    assert np.all(np.abs(lam - g * g) <= 2 * g * 64 * U * g[0] + 1e-300)


def test_sthosvd_qr_exact_ranks_near_sqrt_u():
    i = 16
    g = 2.0 ** (-2.0 * np.arange(i))
    x = planted_superdiagonal(i, g)
    nu = float(np.sum(g * g))
    eps = 2.0 ** -24  # eps^2 = 2^-48: the cut falls at sigma ~ 2^-26
    tau = eps * eps * nu / 3
    # exact rank: smallest R with sum_{r >= R} g_r^2 <= tau
    tails = np.array([np.sum(g[r:] ** 2) for r in range(i + 1)])
    r_exact = int(np.argmax(tails[1:] <= tau)) + 1
    assert r_exact == 13
    res = oracle.sthosvd_qr(x, eps)
    assert res.ranks == (r_exact,) * 3
    for n in range(3):
        lam = res.eigvals[n]
        ref = np.zeros(i)
        ref[: (i if n == 0 else r_exact)] = (g * g)[: (i if n == 0 else r_exact)]
        assert np.all(np.abs(lam - ref) <= 2 * np.sqrt(ref) * 64 * U + (64 * U) ** 2)
        np.testing.assert_allclose(res.discarded[n], tails[r_exact] if n == 0 else 0.0,
                                   rtol=1e-6, atol=1e-30)
    # fit identity of Sec. II-B: ||X - X~||^2 = ||X||^2 - ||G||^2 = sum of discards
    xh = oracle.reconstruct(res.core, res.factors)
    err2, _, _ = oracle.error_metrics(x, xh)
    assert abs(err2 - np.sum(res.discarded)) <= 1e-30 + 1e-3 * np.sum(res.discarded)


def test_sthosvd_qr_agrees_with_gram_path_at_moderate_eps():
    x = synth.planted_tucker((12, 10, 9), (4, 3, 5), seed=11, noise=1e-3)
    if isinstance(x, tuple):
        x = x[0]
    x = np.asfortranarray(np.asarray(x, dtype=np.float64))
    a = oracle.sthosvd_qr(x, 0.05)
    b = oracle.sthosvd(x, 0.05)
    assert a.ranks == b.ranks
    for n in range(3):
        np.testing.assert_allclose(a.eigvals[n], b.eigvals[n], rtol=0, atol=1e-11 * a.norm2)
        np.testing.assert_allclose(a.factors[n], b.factors[n], rtol=0, atol=1e-8)
    np.testing.assert_allclose(a.core, b.core, rtol=0, atol=1e-8 * np.sqrt(a.norm2))
