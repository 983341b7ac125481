"""Helpers shared by the GPU tests: moving Fortran-strided tensors between the
host and the device, and rounding-error bounds used as tolerances."""
import math
import sys

import numpy as np
import torch

U64 = np.finfo(np.float64).eps / 2  # unit roundoff of FP64
U32 = np.finfo(np.float32).eps / 2


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype=None, device="cuda:0"):
    """Host numpy/torch tensor -> device tensor with Fortran strides."""
    from paper_1510_06689_amd import tucker
    t = torch.as_tensor(np.asfortranarray(x)) if isinstance(x, np.ndarray) else x
    dtype = t.dtype if dtype is None else dtype
    out = tucker.empty_fortran(tuple(t.shape), dtype, device)
    out.copy_(t.to(dtype))
    return out


def to_host(t):
    return np.asfortranarray(t.detach().cpu().numpy())


def gram_tolerance(s_ref, k_terms, u=U64):
    """Worst-case bound for a sum of K products in any order:
    |dS_ij| <= K u sum_k |y_ik y_jk| <= K u sqrt(S_ii S_jj) (Cauchy-Schwarz)."""
    d = np.sqrt(np.abs(np.diag(s_ref)))
    return (k_terms + 2) * u * np.outer(d, d) + 1e-300


def ttm_tolerance(y, n, v, u=U64):
    """|dZ| <= J u (|V| |Y|)_(n) elementwise (standard dot-product bound)."""
    import oracle
    jn = y.shape[n]
    return (jn + 2) * u * oracle.ttm(np.abs(y), n, np.abs(v)) + 1e-300


def mode1_rows(x, i, j):
    """Rows i and j of the mode-1 unfolding of a device tensor, as a
    2 x I_2 x .. x I_N host array (FP64)."""
    out = np.empty((2,) + tuple(x.shape[1:]), order="F")
    out[0] = x[i].double().cpu().numpy()
    out[1] = x[j].double().cpu().numpy()
    return out


# The split Gram's quantum for a row with largest magnitude m is at most
# SPLIT_STEP 2^-14 m: its exponent is that of 1.004 m rounded up.
SPLIT_STEP = 1.004


def split_gram_bound(sub):
    """Elementwise bound of the split Gram (mode 1) of a row slice:
    c 2^-15 (m_i |x_j|_1 + m_j |x_i|_1) + c^2 2^-30 K m_i m_j, c = SPLIT_STEP
    (16-bit fixed-point representation to c 2^-15 m_i, exact products, the
    diagonal of D D^T subtracted)."""
    import oracle
    m = oracle.unfold(sub, 0)
    rmax = np.abs(m).max(axis=1)
    l1 = np.abs(m).sum(axis=1)
    k = m.shape[1]
    c = SPLIT_STEP
    return (c * 2.0**-15 * (np.outer(rmax, l1) + np.outer(l1, rmax))
            + c * c * 2.0**-30 * k * np.outer(rmax, rmax))


# Relative error per element of one TTM's output, by arithmetic (taken as a
# bound on ||dZ|| / ||Y|| for the product): split-bf16 keeps 16 bits of both
# operands (about 2^-17 per product; 2^-16 allows for the sum), plain bf16 8
# bits; FP64 arithmetic leaves only the output's storage rounding (below).
TTM_REL = {"bf16x3": 2.0**-16, "bf16": 2.0**-7, "fp64": 0.0}


def carried_errors(res, ref, dims, order, ttm, storage_u, e0=0.0):
    """Per mode n (processing order), how far the GPU's discarded sum may lie
    from the oracle's when both pick the same ranks:

      tol_n = b_n + 2 sqrt(t_n) e_n + e_n^2 + 16 (sqrt(K_n) + J_n) u nu

    b_n   the library's own bound for a split-bf16 Gram of the GPU's Y_n
          (tk_tucker.tail_error_bound; 0 for FP64 Grams),
    e_n   the norm of the difference between the GPU's Y_n and the oracle's:
          the errors of the earlier TTMs, e_n^2 = nu sum_{m before n} c_m^2
          (|sqrt(t(A)) - sqrt(t(B))| <= ||A - B||_F for the tail energy t of a
          fixed-rank truncation, so |dt| <= 2 sqrt(t) e + e^2), c_m from
          TTM_REL plus the storage rounding storage_u of each product,
    the last term FP64 rounding of either Gram (K_n columns, J_n rows).
    e0 (relative to ||X||) is a difference already in the inputs (another
    storage of the same tensor).  Returns ({mode: tol_n}, e_N^2) with e_N the
    same for the core."""
    nu = ref.norm2
    c2 = TTM_REL[ttm] ** 2 + storage_u ** 2
    cur = list(dims)
    e2 = e0 * e0 * nu
    tol = {}
    for n in order:
        k = math.prod(cur) // cur[n]
        t = max(ref.discarded[n], 0.0)
        tol[n] = (res.tail_error_bound[n] + 2 * math.sqrt(t * e2) + e2 +
                  16 * (math.sqrt(k) + cur[n]) * U64 * nu)
        e2 += c2 * nu
        cur[n] = res.ranks[n]
    return tol, e2


def check_against_oracle(res, ref, dims, order, ttm, rel, rel_ref, storage_u=U32, e0=0.0):
    """Same ranks; every mode's discarded sum within carried_errors; and the
    reconstruction errors (rel of the GPU's X~, stored with unit roundoff
    storage_u, rel_ref the oracle's) within what those imply: by the ST-HOSVD
    identity ||X - X~||^2 = sum of discarded, up to the core's carried error
    e_N and the storage rounding of X~.  Returns sum of tol_n / nu."""
    assert res.ranks == ref.ranks, (res.ranks, ref.ranks)
    order = tuple(range(len(dims))) if order is None else tuple(order)
    tol, eN2 = carried_errors(res, ref, dims, order, ttm, storage_u, e0)
    for n in order:
        d = abs(res.discarded[n] - ref.discarded[n])
        assert d <= tol[n], (n, res.discarded[n], ref.discarded[n], tol[n],
                             res.tail_error_bound[n])
    nu = ref.norm2
    ex2 = eN2 + storage_u ** 2 * nu
    slack = sum(tol.values()) + 2 * math.sqrt(rel_ref ** 2 * nu * ex2) + ex2
    assert abs(rel ** 2 - rel_ref ** 2) * nu <= slack, (rel, rel_ref, slack / nu)
    return sum(tol.values()) / nu
