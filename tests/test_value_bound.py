"""Pins of the value-error bounds (tests/value_bound.py) that the GPU tests use
as tolerances: on the noiseless slot-level shadow, which computes exactly what
the circuits compute, the error of every order statistic, window and sorted
slot must lie within its bound taken with no noise allowance (eta = 0).  The
bounds are sound, not tight: on these seeds the errors reach up to a tenth
of their bounds."""
import numpy as np
import pytest

from oracle import shadow as S
from paper_2412_15126_amd import workloads as W

import value_bound as VB

SLOTS = 1 << 12


@pytest.mark.parametrize("N", [8, 16, 32, 64])
def test_order_statistics_within_bound(N):
    cmp, ind = W.ORDER_CMP[N]
    worst = 0.0
    for seed in range(4):
        v, _, _ = W.rank_workload(N, 2.0 ** -10 if N > 8 else 0.01, 300 + seed)
        delta = VB.rank_error(v, cmp, False, SLOTS)
        for a, b in ((1, 1), (N // 2, N // 2), (N, N), (2, N // 2 + 1)):
            _, val, _ = S.order_range_circuit(v, SLOTS, a, b, cmp, ind, False)
            err = abs(val[0] - np.mean(np.sort(v)[a - 1:b]))
            bound = VB.value_bound(v, a, b, ind, delta, 0.0)
            assert err <= bound, (seed, a, b, err, bound)
            worst = max(worst, err / bound)
    assert worst > 1e-2        # not vacuous: some errors reach a percent of their bound


@pytest.mark.parametrize("N", [8, 32])
def test_tie_corrected_order_statistics_within_bound(N):
    cmp, ind = (W.ORDER_TIE_CMP.get(N) or W.ARGMIN_CMP[N])
    for seed in range(4):
        v, _, _ = W.tied_workload(N, 500 + seed, gap=2.0 ** -10 if N > 8 else 0.01)
        delta = VB.rank_error(v, cmp, True, SLOTS)
        for a, b in ((1, 1), (N // 2, N // 2 + 1), (N, N)):
            _, val, _ = S.order_range_circuit(v, SLOTS, a, b, cmp, ind, True)
            err = abs(val[0] - np.mean(np.sort(v)[a - 1:b]))
            assert err <= VB.value_bound(v, a, b, ind, delta, 0.0), (seed, a, b, err)


def test_direct_rank_error_equals_circuit_rank_error():
    """the all-pairs definition of k_j gives the circuit's rank error"""
    for N in (8, 32, 64):
        cmp = W.SORT_CMP[N][0]
        v, _, _ = W.rank_workload(N, 2.0 ** -10, 7)
        assert abs(VB.direct_rank_error(v, cmp) - VB.rank_error(v, cmp, False, SLOTS)) < 1e-9


@pytest.mark.parametrize("N", [8, 16, 32, 64])
def test_sorts_within_bound(N):
    cmp, ind = W.SORT_CMP[N]
    for seed in range(3):
        v, _, _ = W.rank_workload(N, 2.0 ** -10 if N > 8 else 0.01, 700 + seed)
        bound = VB.sort_bound(v, ind, VB.direct_rank_error(v, cmp), 0.0)
        for circuit in (S.sort_circuit, S.sort_col_circuit):
            out = circuit(v, N, SLOTS, cmp, ind)
            err = np.max(np.abs(out[:N] - np.sort(v)))
            assert err <= bound, (seed, circuit.__name__, err, bound)


def test_sort_bound_is_the_per_slot_window_bound():
    """a sorted slot is the two-sided window [i, i]: the vectorised sort bound
    equals the largest per-slot window bound (the one-sided forms that
    value_bound uses for i = 1 and i = N are smaller)"""
    v, _, _ = W.rank_workload(16, 2.0 ** -10, 3)
    cmp, ind = W.SORT_CMP[16]
    d = VB.direct_rank_error(v, cmp)
    mid = max(VB.value_bound(v, i, i, ind, d, VB.ETA) for i in range(2, 16))
    assert VB.sort_bound(v, ind, d, VB.ETA) >= mid


@pytest.mark.slow
def test_multi_ciphertext_sort_within_bound():
    N, b = 512, 256
    cmp, ind = W.MULTI_SORT_CMP[N]
    v, _, _ = W.rank_workload(N, 2.0 ** -10, 0)
    out = np.concatenate([s[:b] for s in S.sort_multi_circuit(v, b, 1 << 16, cmp, ind)])
    err = np.max(np.abs(out - np.sort(v)))
    assert err <= VB.sort_bound(v, ind, VB.direct_rank_error(v, cmp), 0.0), err


@pytest.mark.parametrize("N", [8, 16, 32])
def test_division_within_bound(N):
    """the order statistic with the value by division: the tripled value's
    shared rank and the empty rank below it, on the noiseless shadow"""
    cmp, ind = W.ORDER_CMP[N]
    for seed in range(3):
        v, _, _ = W.tripled_workload(N, 40 + seed, triples=1, gap=0.01 if N == 8 else 2.0 ** -10)
        u, c = np.unique(v, return_counts=True)
        t = u[np.argmax(c)]
        below = int(np.sum(v < t))
        for k, want in ((below + 2, t), (below + 1, 0.0)):
            _, val = S.order_stat_div_circuit(v, N, SLOTS, k, cmp, ind, 6)
            err = abs(val[0] - want)
            assert err <= VB.division_bound(v, k, cmp, ind, 6, eta=0.0), (seed, k, err)


def test_average_ranks_are_the_circuit_ranks():
    """with Cmp(0) = 1/2 the rank sum of c equal values is #smaller + (c + 1)/2"""
    from oracle import shadow
    v, _, _ = W.tripled_workload(16, 3, triples=2)
    cmp = W.ORDER_CMP[16][0]
    k = shadow.cmp_of(v[:, None] - v[None, :], cmp).sum(axis=1) + 0.5
    assert np.max(np.abs(k - VB.average_ranks(v))) < 0.45
    assert set(VB.average_ranks(v)) >= {float(np.sum(v < x)) + 2.0 for x in v if np.sum(v == x) == 3}
