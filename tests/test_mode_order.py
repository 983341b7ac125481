"""Mode-order rules of sthosvd_mode_order (host-only C-ABI call, no GPU).

Pins: Sec. VIII-C's mode-order experiment (25x250x250x250 tensor of multilinear
rank 10x10x100x100) states that the greedy least-flops heuristic does not
find the best order there and that the best order starts with the second
mode, the one with the largest compression ratio; the byte rule is checked
against a brute-force search over all orders of the same traffic model."""
import itertools
import math

import pytest

from paper_1510_06689_amd import tucker

PAPER_DIMS, PAPER_RANKS = (25, 250, 250, 250), (10, 10, 100, 100)


def traffic(dims, ranks, order, elem):
    """Every Gram reads Y_n, every TTM reads Y_n and writes Y_{n+1}."""
    cur, total = list(dims), 0
    for n in order:
        ny = math.prod(cur)
        cur[n] = ranks[n]
        total += (2 * ny + math.prod(cur)) * elem
    return total


def test_paper_example_heuristics():
    flops = tucker.mode_order(PAPER_DIMS, PAPER_RANKS, "flops", 8)
    ratio = tucker.mode_order(PAPER_DIMS, PAPER_RANKS, "ratio", 8)
    best = tucker.mode_order(PAPER_DIMS, PAPER_RANKS, "bytes", 8)
    assert flops[0] == 0          # cheapest first step: the smallest mode
    assert ratio[0] == 1          # largest I_n / R_n = 25
    assert best[0] == 1           # the paper's best order starts with the second mode
    assert flops == (0, 1, 2, 3) and ratio == (1, 0, 2, 3)


@pytest.mark.parametrize("dims,ranks", [
    (PAPER_DIMS, PAPER_RANKS),
    ((128, 128, 128, 32, 32), (16, 16, 16, 8, 8)),
    ((256, 256, 256, 64, 16), (32, 32, 32, 16, 8)),
    ((7, 30, 5, 12, 9, 4), (7, 2, 1, 11, 3, 2)),
    ((10, 10, 10), (5, 5, 5)),
])
def test_bytes_rule_is_the_exhaustive_minimum(dims, ranks):
    got = tucker.mode_order(dims, ranks, "bytes", 4)
    costs = {p: traffic(dims, ranks, p, 4) for p in itertools.permutations(range(len(dims)))}
    low = min(costs.values())
    assert costs[got] == low
    assert got == min(p for p, c in costs.items() if c == low)   # ties: lexicographically first


def test_combustion256_orders_match_the_bench_byte_counts():
    dims, ranks = (256, 256, 256, 64, 16), (32, 32, 32, 16, 8)
    assert traffic(dims, ranks, range(5), 4) == 166950076416
    assert traffic(dims, ranks, (4, 3, 2, 1, 0), 4) == 269928628224
    assert tucker.mode_order(dims, ranks, "bytes", 4) == (0, 1, 2, 3, 4)


def test_greedy_rules_step_by_step():
    dims, ranks = (40, 9, 100, 60), (4, 3, 50, 6)
    # flops: I + R = 44, 12, 150, 66 -> 1, 0, 3, 2
    assert tucker.mode_order(dims, ranks, "flops", 8) == (1, 0, 3, 2)
    # ratio: I / R = 10, 3, 2, 10 -> ties go to the lower index: 0, 3, 1, 2
    assert tucker.mode_order(dims, ranks, "ratio", 8) == (0, 3, 1, 2)


@pytest.mark.parametrize("dims,ranks,rule", [
    ((), (), "bytes"),
    ((5, 5), (6, 5), "bytes"),
    ((5, 5), (0, 5), "ratio"),
    ((5,) * 9, (1,) * 9, "flops"),
])
def test_invalid_arguments(dims, ranks, rule):
    with pytest.raises(tucker.TuckerError) as e:
        tucker.mode_order(dims, ranks, rule, 8)
    assert e.value.status == -1
