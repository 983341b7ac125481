"""HOOI (Alg. 2) on the GPU against the oracle's HOOI on the same input: the
fit after the ST-HOSVD and after every sweep, the final factors (same sign
rule) and core, and convergence under the "ceases to decrease" rule."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1510_06689_amd import tucker
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _x(dims, ranks, noise, seed, dtype=torch.float64):
    return synth.planted_tucker(dims, ranks, rho=0.8, factor_kind="gaussian", noise=noise,
                                noise_mode="exact", seed=seed, dtype=dtype)


CASES = [((14, 12, 10), (4, 4, 3), 0.3, 1, None),
         ((8, 7, 6, 5), (2, 3, 2, 2), 0.2, 2, (3, 1, 0, 2)),
         ((40, 33, 37, 6), (5, 4, 6, 2), 0.1, 3, None),
         ((130, 20, 9), (6, 5, 3), 0.05, 4, None)]


@pytest.mark.parametrize("dims,ranks,noise,seed,order", CASES)
def test_hooi_sweeps_match_oracle(dims, ranks, noise, seed, order):
    say(f"hooi {dims} ranks {ranks} order {order}")
    x = _x(dims, ranks, noise, seed)
    xh = x.numpy()
    res, fits = tucker.hooi(to_dev(x), 0.0, order=order, ranks=ranks, max_sweeps=4, tol=-1.0)
    ref = oracle.hooi(xh, 0.0, ranks=ranks, order=order, max_sweeps=4, tol=-1.0)
    nu = ref.norm2
    assert len(fits) == len(ref.fits) == 5
    assert all(abs(a - b) <= 1e-10 * nu for a, b in zip(fits, ref.fits)), (fits, ref.fits)
    assert all(b <= a + 1e-12 * nu for a, b in zip(fits, fits[1:]))
    for u, v in zip(res.factors, ref.factors):
        u = u.cpu().numpy()
        assert np.abs(u @ u.T - v @ v.T).max() <= 1e-8
        assert np.abs(u - v).max() <= 1e-7
    assert np.abs(res.core.cpu().numpy() - ref.core).max() <= 1e-8 * math.sqrt(nu)
    xr = tucker.reconstruct(res.core, res.factors)
    e2, _, _ = tucker.error_metrics(to_dev(x), xr)
    assert abs(e2 - fits[-1]) <= 1e-10 * nu


def test_hooi_converges_like_oracle_from_eps_start():
    x = _x((16, 14, 12), (4, 3, 3), 0.1, 8)
    res, fits = tucker.hooi(to_dev(x), 0.2, max_sweeps=100, tol=0.0)
    ref = oracle.hooi(x.numpy(), 0.2, max_sweeps=100, tol=0.0)
    say(f"eps start: ranks {res.ranks} sweeps gpu {len(fits) - 1} oracle {ref.sweeps}")
    assert res.ranks == tuple(ref.ranks)
    assert len(fits) - 1 < 100 and ref.sweeps < 100
    assert abs(fits[-1] - ref.fits[-1]) <= 1e-10 * ref.norm2
    assert fits[-1] < fits[0]


def test_hooi_mixed_precision():
    """FP32 storage, split-bf16 Grams and bf16x3 TTMs: the fits follow the
    FP64 oracle's on the same values to the TTMs' ~2^-16 of ||X||^2."""
    x = _x((48, 40, 36), (6, 5, 4), 0.1, 9, dtype=torch.float32)
    res, fits = tucker.hooi(to_dev(x), 0.0, ranks=(6, 5, 4), max_sweeps=3, tol=-1.0,
                            gram_precision="split_bf16", ttm_precision="bf16x3")
    ref = oracle.hooi(x.double().numpy(), 0.0, ranks=(6, 5, 4), max_sweeps=3, tol=-1.0)
    assert all(abs(a - b) <= 2.0**-14 * ref.norm2 for a, b in zip(fits, ref.fits))
    for u, v in zip(res.factors, ref.factors):
        u = u.cpu().numpy()
        assert np.abs(u @ u.T - v @ v.T).max() <= 1e-3


def test_hooi_rejects_negative_sweeps():
    x = to_dev(_x((6, 5, 4), (2, 2, 2), 0.1, 1))
    with pytest.raises(tucker.TuckerError) as e:
        tucker.hooi(x, 0.0, ranks=(2, 2, 2), max_sweeps=-1)
    assert e.value.status == -1
