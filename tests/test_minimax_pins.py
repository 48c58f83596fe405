"""Pins of the minimax composite comparator (section 2.2's pointer to composite
minimax approximations of the sign function).

The coefficient table (oracle/shadow.py MM_COEF, repeated in oracle/ora.c and
the library) must be the greedy minimax composite designed on [2^-8.5, 1]:
each stage equioscillates on its interval (Chebyshev's alternation theorem
characterises the minimax polynomial), the intervals chain, an independent
Remez exchange reproduces the table, and four stages rank N = 128 values at
the 2^-10 gap exactly in the slot-level shadow, where the best four-fold f/g
split does not."""
import numpy as np
import pytest

from oracle import shadow as S
from paper_2412_15126_amd import workloads as W

import remez


def _p(c, x):
    return sum(c[k] * x ** (2 * k + 1) for k in range(4))


def _chain():
    a, b, out = S.MM_DESIGN_LO, 1.0, []
    for c in S.MM_COEF:
        out.append((a, b))
        xs = np.linspace(a, b, 400001)
        y = _p(c, xs)
        a, b = float(y.min()), float(y.max())
    return out


def test_stages_equioscillate_on_their_intervals():
    for s, (c, (a, b)) in enumerate(zip(S.MM_COEF, _chain())):
        xs = np.linspace(a, b, 2000001)
        err = 1.0 - _p(c, xs)
        E = np.max(np.abs(err))
        # the runs of constant sign and their extrema: 5 alternation points
        # (4 coefficients + the levelled error), all of magnitude E
        sgn = np.sign(err)
        cuts = np.flatnonzero(sgn[1:] != sgn[:-1]) + 1
        runs = np.split(np.arange(len(xs)), cuts)
        ext = [np.max(np.abs(err[r])) for r in runs]
        assert len(runs) == 5, (s, len(runs))
        assert np.allclose(ext, E, rtol=1e-6, atol=0), (s, ext, E)
        assert err[0] > 0 and err[-1] > 0, s      # the error starts and ends on the same side


def test_table_matches_independent_remez():
    ref = remez.composite(S.MM_DESIGN_LO, len(S.MM_COEF))
    for s, ((c, (a, b)), got, (ga, gb)) in enumerate(zip(ref, S.MM_COEF, _chain())):
        assert np.allclose(got, c, rtol=1e-8, atol=1e-10), s
        assert abs(a - ga) < 1e-9 and abs(b - gb) < 1e-9, s


def test_final_errors_fall_stage_by_stage():
    errs = []
    for c, (a, b) in zip(S.MM_COEF, _chain()):
        xs = np.linspace(a, b, 400001)
        errs.append(np.max(np.abs(1.0 - _p(c, xs))))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[3] < 0.01 and errs[4] < 1e-8


@pytest.mark.slow
def test_four_stages_rank_128_exactly_at_gap_2m10():
    """Four minimax stages (12 levels) rank N = 128 exactly over 100 seeds at
    the 2^-10 gap; the f/g split g^3 f (also four compositions) misses by up
    to a whole rank."""
    N, slots = 128, 1 << 14
    worst_mm, worst_fg = 0.0, 0.0
    for seed in range(100):
        v, _, _ = W.rank_workload(N, 2.0 ** -10, seed)
        d = v[None, :] - v[:, None]
        exact = np.argsort(np.argsort(v)) + 1
        r = S.cmp_of(d, (0, 0, 0, 4)).sum(axis=0) + 0.5
        worst_mm = max(worst_mm, float(np.max(np.abs(r - exact))))
        if seed < 20:
            r = S.cmp_of(d, (3, 1)).sum(axis=0) + 0.5
            worst_fg = max(worst_fg, float(np.max(np.abs(r - exact))))
    assert worst_mm < 0.45, worst_mm
    assert worst_fg > 0.5, worst_fg
    # the circuit's own slot layout gives the same ranks
    v, _, _ = W.rank_workload(N, 2.0 ** -10, 0)
    R, _ = S.rank(v, N, slots, (0, 0, 0, 4))
    assert np.max(np.abs(R[:N] - (np.argsort(np.argsort(v)) + 1))) < 0.45
