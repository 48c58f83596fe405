"""Pins of the Chebyshev comparator (section 2.2; the paper's choice for rank
and minimum at N <= 256, section 6.1).

The comparison function of Eq. (1), as a function of d = x - y, is
interpolated on [-1, 1] at the 2^(D-1) Chebyshev nodes and evaluated with the
Paterson-Stockmeyer algorithm in the Chebyshev basis, taking D levels.
Pinned here:
  * the closed-form coefficients against the interpolation sum itself;
  * the whole construction (function, interval, degree per depth) against the
    ranking errors the paper plots for N = 128 in its appendix on the
    approximation degree;
  * the oracle's homomorphic Paterson-Stockmeyer evaluation against a direct
    evaluation of the Chebyshev series on the decrypted input;
  * the oracle's rank and order statistics with this comparator against the
    shadow and the exact plaintext results.
"""
import json
import os

import numpy as np
import pytest
from numpy.polynomial import chebyshev as Ch

from oracle import shadow as S
from paper_2412_15126_amd import workloads as W

FIG = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_rank_degree.json")))


def _node_sum_coeffs(D):
    """c_k = (2/n) sum_j f(x_j) T_k(x_j) at the n = 2^(D-1) nodes x_j = cos(pi (j + 1/2) / n), c_0 halved"""
    n = 1 << (D - 1)
    th = np.pi * (np.arange(n) + 0.5) / n
    f = np.where(np.cos(th) > 0, 1.0, 0.0)          # no node sits at 0 (n is even)
    c = (2.0 / n) * np.cos(np.outer(np.arange(n), th)) @ f
    c[0] /= 2
    return c


@pytest.mark.parametrize("D", [2, 3, 5, 8, 12])
def test_cheb_closed_form_equals_node_sum(ora, D):
    want = _node_sum_coeffs(D)
    assert np.max(np.abs(ora.cheb_step_coeffs(D) - want)) < 1e-12
    assert np.max(np.abs(S.cheb_step_coeffs(D) - want)) < 1e-12
    c = ora.cheb_step_coeffs(D)
    assert c[0] == 0.5 and np.all(c[2::2] == 0.0)      # odd around 1/2: exact zeros
    # the interpolant passes through f at every node
    n = 1 << (D - 1)
    x = np.cos(np.pi * (np.arange(n) + 0.5) / n)
    assert np.max(np.abs(Ch.chebval(x, c) - (x > 0))) < 1e-9


def test_cheb_comparator_reproduces_paper_rank_error_figure():
    """Mean |rank - true rank| over N = 128 values uniform in [0, 1), averaged
    over seeds, against the appendix figure: within 10% at every plotted
    depth.  An even-degree interpolant (a node at 0, where the comparison
    jumps) or another interval misses by far more at depth 11 and above."""
    N = FIG["N"]
    rng = np.random.default_rng(2412)
    vs = [rng.uniform(0.0, 1.0, N) for _ in range(60)]
    for D, want in zip(FIG["depth"], FIG["avg_error"]):
        c = S.cheb_step_coeffs(D)
        errs = []
        for v in vs:
            r = Ch.chebval(v[None, :] - v[:, None], c).sum(axis=0) + 0.5
            errs.append(np.mean(np.abs(r - (np.argsort(np.argsort(v)) + 1))))
        got = float(np.mean(errs))
        assert abs(got - want) < 0.10 * want, (D, got, want)


@pytest.fixture(scope="module")
def t10(ora):
    P = ora.Params(**W.PSETS["T10"])
    return P, ora.Keys(P, bytes(range(32)), P.L, [])


@pytest.mark.parametrize("deg1", [2, 4, 8, 16, 64])
def test_oracle_cheb_eval_equals_chebyshev_series(ora, t10, deg1):
    """Paterson-Stockmeyer in the Chebyshev basis computes sum_i c_i T_i(x):
    random coefficients (some exactly zero, so that the skipped terms are
    exercised), inputs in [-1, 1]; B = log2(deg1) + 1 levels consumed."""
    P, keys = t10
    rng = np.random.default_rng(deg1)
    c = rng.uniform(-1.0, 1.0, deg1)
    c[rng.random(deg1) < 0.3] = 0.0
    x = rng.uniform(-1.0, 1.0, 64)
    ct = ora.encrypt(keys, x, P.L, bytes([deg1]) * 32)
    out = ora.cheb_eval(keys, ct, c)
    assert out.level == P.L - ora.cheb_depth(deg1) == P.L - (int(np.log2(deg1)) + 1)
    got = ora.decrypt(keys, out, 64)
    want = Ch.chebval(x, c)
    assert np.max(np.abs(got - want)) < 1e-5 * np.sum(np.abs(c)), np.max(np.abs(got - want))


@pytest.fixture(scope="module")
def t12d(ora):
    P = ora.Params(**W.PSETS["T12D"])
    keys = ora.Keys(P, bytes(range(32)), P.L, P.circuit_galois(8, 6))
    return P, keys


def test_oracle_rank8_chebyshev_matches_shadow_and_exact(ora, t12d):
    P, keys = t12d
    N, cmp = 8, W.CHEB_CMP[8]
    for seed in (0, 1):
        v, _, eseed = W.rank_workload(N, 0.01, seed)
        depth = ora.rank_depth(*cmp)
        assert depth == 2 + cmp[2]
        r = ora.rank(keys, ora.encrypt(keys, v, depth, eseed), N, *cmp)
        assert r.level == 0
        got = ora.decrypt(keys, r, N)
        sh, _ = S.rank(v, N, P.n // 2, cmp)
        assert np.max(np.abs(got - sh[:N])) < 1e-3
        assert np.array_equal(np.round(got), np.argsort(np.argsort(v)) + 1)


def _kth(v, k):
    order = np.argsort(v, kind="stable")
    return order[k - 1], v[order[k - 1]]


@pytest.mark.parametrize("k,tie", [(1, True), (3, False), (8, False)])
def test_oracle_order_statistic_chebyshev_matches_shadow(ora, t12d, k, tie):
    """Order statistics with the Chebyshev comparator and indicator (the
    paper's pairing for the minimum, section 6.1)."""
    P, keys = t12d
    N = 8
    cmp = ind = W.CHEB_CMP[N]
    v, _, eseed = (W.tied_workload(N, 3, 0.01) if tie else W.rank_workload(N, 0.01, 3))
    depth = ora.order_stat_depth(N, k, cmp, ind, tie)
    ct = ora.encrypt(keys, v, depth, eseed)
    oh, val = ora.order_stat(keys, ct, N, k, cmp, ind, tie)
    got_oh, got_val = ora.decrypt(keys, oh, N), ora.decrypt(keys, val, 1)[0]
    sh_oh, sh_val, _ = S.order_stat_circuit(v, N, P.n // 2, k, cmp, ind, tie)
    assert np.max(np.abs(got_oh - sh_oh[:N])) < 1e-3 and abs(got_val - sh_val[0]) < 1e-3
    j, want = _kth(v, k)
    assert np.array_equal(np.round(got_oh), np.eye(N)[j])
    assert abs(got_val - want) < 0.05
