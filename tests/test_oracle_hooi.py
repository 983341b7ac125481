"""Pins of the oracle's HOOI (Alg. 2) against facts that do not depend on
its own code: Eckart-Young for N = 2, the per-mode lower bound, monotone
fits (the paper: HOOI improves the error monotonically), the fit identity
against a reconstruction, exact recovery of a noiseless low-rank tensor, and
the stationarity of the converged factors."""
import numpy as np
import pytest
import torch

import oracle
import synth


def _x(dims, ranks, noise, seed, rho=0.8):
    return synth.planted_tucker(dims, ranks, rho=rho, factor_kind="gaussian", noise=noise,
                                noise_mode="exact", seed=seed).numpy()


def test_matrix_case_is_the_truncated_svd():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((30, 20)) @ np.diag(0.8 ** np.arange(20)) @ rng.standard_normal((20, 20))
    r = oracle.hooi(np.asfortranarray(a), 0.0, ranks=(5, 5), max_sweeps=3, tol=-1.0)
    sv = np.linalg.svd(a, compute_uv=False)
    tail = float(np.sum(sv[5:] ** 2))
    assert all(abs(f - tail) <= 1e-10 * float(np.sum(sv ** 2)) for f in r.fits)


@pytest.mark.parametrize("dims,ranks,seed", [((12, 10, 9), (3, 4, 2), 1),
                                             ((8, 7, 6, 5), (2, 3, 2, 2), 2)])
def test_fits_decrease_and_respect_the_mode_bounds(dims, ranks, seed):
    x = _x(dims, ranks, 0.3, seed)
    r = oracle.hooi(x, 0.0, ranks=ranks, max_sweeps=8, tol=-1.0)
    nu = r.norm2
    assert all(b <= a + 1e-12 * nu for a, b in zip(r.fits, r.fits[1:]))
    # any Tucker model of multilinear rank R misses at least the mode-n tail
    for n in range(len(dims)):
        lam = np.linalg.eigvalsh(oracle.unfold(x, n) @ oracle.unfold(x, n).T)[::-1]
        assert r.fits[-1] >= float(np.sum(lam[ranks[n]:])) - 1e-12 * nu
    # the fit is the model error of the returned core and factors
    xh = oracle.reconstruct(r.core, r.factors)
    assert abs(float(np.sum((x - xh) ** 2)) - r.fits[-1]) <= 1e-10 * nu
    for u in r.factors:
        assert np.abs(u.T @ u - np.eye(u.shape[1])).max() <= 1e-12


def test_noiseless_low_rank_is_recovered():
    x = _x((10, 9, 8), (3, 2, 2), 0.0, 5)
    r = oracle.hooi(x, 0.0, ranks=(3, 2, 2), max_sweeps=2, tol=-1.0)
    assert max(r.fits) <= 1e-24 * r.norm2 + 1e-28


def test_converged_factors_are_stationary():
    x = _x((10, 9, 8), (3, 3, 2), 0.2, 7)
    r = oracle.hooi(x, 0.0, ranks=(3, 3, 2), max_sweeps=200, tol=0.0)
    assert r.sweeps < 200
    for n in range(3):
        y = x
        for m in range(3):
            if m != n:
                y = oracle.ttm(y, m, r.factors[m].T)
        w, v = np.linalg.eigh(oracle.gram(y, n))
        top = v[:, ::-1][:, :r.ranks[n]]
        assert np.abs(top @ top.T - r.factors[n] @ r.factors[n].T).max() <= 1e-6


def test_improves_on_sthosvd_and_stops():
    x = _x((14, 12, 10), (4, 4, 3), 0.3, 9)
    r = oracle.hooi(x, 0.0, ranks=(4, 4, 3), max_sweeps=50, tol=1e-12)
    assert r.fits[-1] < r.fits[0]
    assert r.sweeps <= 50 and len(r.fits) == r.sweeps + 1
