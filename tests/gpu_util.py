"""Helpers shared by the GPU tests: moving Fortran-strided tensors between the
host and the device, and rounding-error bounds used as tolerances."""
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


def split_gram_bound(sub):
    """Elementwise bound of the split-bf16 Gram (mode 1) of a row slice:
    2^-16 (m_i |x_j|_1 + m_j |x_i|_1) + 2^-24 K m_i m_j."""
    import oracle
    m = oracle.unfold(sub, 0)
    rmax = np.abs(m).max(axis=1)
    l1 = np.abs(m).sum(axis=1)
    k = m.shape[1]
    return 2.0**-16 * (np.outer(rmax, l1) + np.outer(l1, rmax)) + 2.0**-24 * k * np.outer(rmax, rmax)
