"""Batched compression (one launch sequence per mode step for a whole batch of
uneven FP32 problems) against the FP64 oracle per problem, graph replays
against the eager run, and the in-run FP64 recomputation of modes whose rank
the split Gram could not certify."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1510_06689_amd import tucker
from gpu_util import check_against_oracle, say, to_dev
from test_gpu_mixed import _first_mode_tie_case

pytestmark = pytest.mark.gpu


def _problems(sizes, ranks, noise=1e-5, seed=30):
    xs = []
    for t, s in enumerate(sizes):
        dims = (s, s, s, 8)
        rk = tuple(min(r, d) for r, d in zip(ranks, dims))
        xs.append(synth.planted_tucker(dims, rk, rho=0.6, factor_kind="cosine", noise=noise,
                                       noise_mode="sigma", seed=seed + t, dtype=torch.float32))
    return xs


def _relerr(xd, res):
    xh = tucker.reconstruct(res.core, res.factors)
    e2, _, n2 = tucker.error_metrics(xd, xh)
    return math.sqrt(e2 / n2)


def test_batch_matches_oracle_per_problem():
    xs = _problems([20, 33, 48, 64, 90], (5, 5, 5, 3))
    xd = [to_dev(x) for x in xs]
    c = tucker.BatchCompressor(xd, 1e-4)
    c.run()
    c.finish()
    res = c.results()
    for x, d, r in zip(xs, xd, res):
        xh = x.double().numpy()
        ref = oracle.sthosvd(xh, 1e-4)
        say(f"batch problem {x.shape}: ranks {r.ranks} oracle {ref.ranks} redone {r.fp64_modes}")
        assert r.ranks == ref.ranks
        xr = oracle.reconstruct(ref.core, ref.factors)
        rel_ref = math.sqrt(float(np.sum((xh - xr) ** 2)) / ref.norm2)
        rel = _relerr(d, r)
        assert rel <= 1e-4
        check_against_oracle(r, ref, x.shape, None, "bf16x3", rel, rel_ref)
        assert math.isclose(r.norm2, ref.norm2, rel_tol=1e-6)
        for u in r.factors:
            ut = u.cpu().numpy()
            assert np.abs(ut.T @ ut - np.eye(ut.shape[1])).max() <= 1e-12


def test_batch_graph_replays_equal_eager_run():
    xs = [to_dev(x) for x in _problems([24, 40, 57, 96], (6, 6, 6, 3), seed=50)]
    c = tucker.BatchCompressor(xs, 1e-4)
    c.run()
    torch.cuda.synchronize()
    ref_ranks = c.ranks_dev.clone()
    nvalid = [math.prod(r) for r in ref_ranks.view(len(xs), -1).cpu().tolist()]
    ref_cores = [t[:k].clone() for t, k in zip(c.core_bufs, nvalid)]
    c.capture()
    for rep in range(3):
        for t in c.core_bufs:
            t.zero_()                       # eager work between replays
        c.ranks_dev.zero_()
        torch.cuda.synchronize()
        c.replay()
        torch.cuda.synchronize()
        assert torch.equal(c.ranks_dev, ref_ranks), rep
        for a, b, k in zip(c.core_bufs, ref_cores, nvalid):
            assert torch.equal(a[:k], b), rep


def test_batch_redo_keeps_oracle_ranks_where_uncertain():
    """eps = 1e-3 with the noise of one problem near the threshold: whatever
    the guard flags is recomputed within the run, and every rank equals the
    oracle's."""
    xs = _problems([30, 44], (5, 5, 5, 3), seed=70) + \
        _problems([36], (5, 5, 5, 3), noise=5e-4, seed=90)
    xd = [to_dev(x) for x in xs]
    c = tucker.BatchCompressor(xd, 1e-3)
    c.run()
    c.finish()
    for x, r in zip(xs, c.results()):
        ref = oracle.sthosvd(x.double().numpy(), 1e-3)
        say(f"problem {x.shape}: ranks {r.ranks} oracle {ref.ranks} redone {r.fp64_modes}")
        assert r.ranks == ref.ranks


def test_batch_guard_recomputes_on_device():
    """A batch holding the near-tie case (the first-processed mode, J = 128,
    cut at t_R = (1 - 1e-4) tau: no split-Gram bound is that small) and three
    problems of the 64-problem benchmark batch (s^3 x 16, ranks (12,12,12,6),
    eps = 1e-4): the run must resolve every uncertain rank on the device (no
    status bit 4 left; the near tie recomputed in FP64 and recorded), with
    every rank equal to the oracle's, and batch and single-problem results
    each within their derived bounds of the oracle's discarded sums and
    error."""
    xt, xth, eps_t, order_t = _first_mode_tie_case()
    ws = synth.batch_workload()
    pick = [19, 15, 1]                       # s = 56, 28, 57
    xs = [ws[i].make(dtype=torch.float64).float() for i in pick]
    for eps, order, batch in ((eps_t, order_t, [xt]), (ws[0].eps, None, xs)):
        xd = [to_dev(x) for x in batch]
        c = tucker.BatchCompressor(xd, eps, order=order)
        c.run()
        torch.cuda.synchronize()
        status = c.status_dev.view(-1, 2).cpu().numpy()
        # no uncertain rank (4) left, and no FP64-only mark (8) of a later
        # step's small problem outlives its eigensolver pass
        assert not (status[:, 0] & 12).any(), status
        c.finish()
        res = c.results()
        if batch is not xs:
            assert 1 in res[0].fp64_modes, res[0].fp64_modes
        for x, d, r in zip(batch, xd, res):
            xh = x.double().numpy()
            ref = oracle.sthosvd(xh, eps, order=order)
            single = tucker.sthosvd(d, eps, order=order, gram_precision="split_bf16",
                                    ttm_precision="bf16x3")
            say(f"problem {tuple(x.shape)} eps {eps:.3e}: ranks {r.ranks} oracle {ref.ranks} "
                f"fp64 modes batch {r.fp64_modes} single {single.fp64_modes}")
            xr = oracle.reconstruct(ref.core, ref.factors)
            rel_ref = math.sqrt(float(np.sum((xh - xr) ** 2)) / ref.norm2)
            rel, rel1 = _relerr(d, r), _relerr(d, single)
            assert rel <= eps and rel1 <= eps
            check_against_oracle(r, ref, x.shape, order, "bf16x3", rel, rel_ref)
            check_against_oracle(single, ref, x.shape, order, single.ttm_precision, rel1,
                                 rel_ref)


def test_batch_rejects_unsupported():
    x64 = to_dev(synth.random_tensor((10, 10, 10, 4), seed=1))
    with pytest.raises(tucker.TuckerError) as e:
        tucker.BatchCompressor([x64], 1e-3)
    assert e.value.status == -2
    big = to_dev(synth.random_tensor((130, 4, 4, 2), seed=2, dtype=torch.float32))
    with pytest.raises(tucker.TuckerError) as e:
        tucker.BatchCompressor([big], 1e-3)
    assert e.value.status == -2


def test_batch_of_many_large_problems_matches_single_path():
    """Sixteen problems of extent 80..93 from the 64-problem benchmark batch.
    At this size and count the later steps' workgroups per task are capped
    (the last mode's FP64 Gram, counted at the capacity shape, would take
    about 1500 per task; the cap is max(256, 16384 / 16) = 1024), so the capped
    partition must still give every problem the single-problem path's ranks
    and the planted ones, within the error target."""
    ws = synth.batch_workload()
    pick = [i for i, w in enumerate(ws) if w.dims[0] >= 80][:16]
    assert len(pick) == 16
    eps = ws[0].eps
    xd = [to_dev(ws[i].make(dtype=torch.float64).float()) for i in pick]
    c = tucker.BatchCompressor(xd, eps)
    c.run()
    c.finish()
    res = c.results()
    for i, d, r in zip(pick, xd, res):
        single = tucker.sthosvd(d, eps, gram_precision="split_bf16", ttm_precision="bf16x3")
        say(f"problem {i} {tuple(d.shape)}: batch {r.ranks} single {single.ranks} "
            f"planted {ws[i].ranks}")
        assert r.ranks == single.ranks == tuple(ws[i].ranks)
        rel, rel1 = _relerr(d, r), _relerr(d, single)
        assert rel <= eps and rel1 <= eps
        # the same truncation through both paths: at errors near the noise
        # (1e-5 here) the split-bf16 TTM's rounding, 2^-16 relative per mode,
        # is of the same size, so the two paths (different kernels and
        # summation orders) may differ by up to N 2^-16
        assert abs(rel - rel1) <= d.dim() * 2.0**-16, (rel, rel1)
