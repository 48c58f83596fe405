"""Circuit-level pins: the paper's worked examples and closed forms.

The slot-level shadow (oracle/shadow.py) is checked against Figures 1-4 and
the proofs' closed forms; the oracle's decrypted CKKS outputs are then
checked against the shadow (same circuit, composite comparator) and against
exact plaintext ranks.
"""
import json
import os

import numpy as np
import pytest

from oracle import shadow as S
from paper_2412_15126_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def _mat(x, N):
    return np.asarray(x[:N * N]).reshape(N, N)


def test_fig1_transc_steps():
    g = GOLD["fig1_transc_n8"]
    N = g["N"]
    x = np.zeros(N * N)
    x[0:N * N:N] = np.arange(1, N + 1)       # column vector v_1..v_8
    trace = []
    out = S.trans_c(x, N, trace)
    assert np.array_equal(_mat(x, N), np.array(g["steps"][0]))
    for t, want in zip(trace, g["steps"][1:4]):
        assert np.array_equal(_mat(t, N), np.array(want))
    assert np.array_equal(_mat(out, N), np.array(g["steps"][4]))
    assert [N * (N - 1) >> i for i in (1, 2, 3)] == g["shifts"]


@pytest.mark.parametrize("slots", [64, 2048])
def test_transr_transc_roundtrip_and_row0(slots):
    N = 8
    v = np.arange(1, N + 1, dtype=float)
    col = S.trans_r(S.embed(v, slots), N)
    assert np.array_equal(col[0:N * N:N], v) and np.count_nonzero(col) == N
    row = S.trans_c(col, N)
    assert np.array_equal(row[:N], v) and np.count_nonzero(row) == N


def test_fig2_rank_intermediates():
    g = GOLD["fig2_rank"]
    N = 4
    R, it = S.rank(np.array(g["v"], float), N, 64)
    assert np.array_equal(_mat(it["VR"], N), np.array(g["VR"]))
    assert np.array_equal(_mat(it["VC"], N), np.array(g["VC"]))
    assert np.array_equal(_mat(it["C"], N), np.array(g["C"]))
    assert np.array_equal(it["S"][:N], np.array(g["sumR"]))
    assert np.array_equal(R[:N], np.array(g["rank"], float))


def test_fractional_rank_example_with_padding():
    g = GOLD["fractional_rank"]
    v = np.array(g["v"], float)
    # pad to the next power of two with values above every input
    padded = np.concatenate([v, [1e9, 2e9, 3e9]])
    R, _ = S.rank(padded, 8, 128)
    assert np.array_equal(R[:5], np.array(g["rank"]))


def test_fig3_sort_intermediates():
    g = GOLD["fig3_sort"]
    N = 4
    out, it = S.sort(np.array(g["v"], float), N, 64)
    assert np.array_equal(it["R"][:N], np.array(g["rank"], float))
    assert np.array_equal(_mat(it["D"], N), np.array(g["D"]))
    assert np.array_equal(_mat(it["M"], N), np.array(g["M"]))
    assert np.array_equal(_mat(it["P"], N), np.array(g["P"]))
    assert np.array_equal(it["SC"][0:N * N:N], np.array(g["sumC"], float))
    assert np.array_equal(out[:N], np.array(g["sorted"], float))


def test_fig4_tie_offset():
    g = GOLD["fig4_ties"]
    N = 4
    v = np.array(g["v"], float)
    R, it = S.rank(v, N, 64)
    assert np.array_equal(R[:N], np.array(g["rank"]))
    F, t = S.tie_offset(it["C"], N, 64)
    assert np.array_equal(_mat(t["E"], N), np.array(g["E"]))
    assert np.array_equal(_mat(t["delta"], N), np.array(g["delta"]))
    assert np.array_equal(_mat(t["E"] * t["delta"], N), np.array(g["Edelta"]))
    assert np.array_equal(t["T"][:N], np.array(g["T"], float))
    assert np.array_equal(t["U"][:N], np.array(g["U"], float))
    assert np.array_equal(F[:N], np.array(g["F"]))
    assert np.array_equal((R + F)[:N], np.array(g["k"], float))


@pytest.mark.parametrize("seed", range(20))
def test_rank_closed_form_and_tie_permutation(seed):
    """r_j = |L_j| + (|E_j| + 1)/2 (section 3.1 proof); R + F is a permutation with
    v_j the k_j-th order statistic (section 4 proof)."""
    rng = np.random.default_rng(seed)
    N = 16
    v = rng.integers(0, 6, N).astype(float)           # many ties
    R, it = S.rank(v, N, 512)
    L = np.array([(v < x).sum() for x in v])
    E = np.array([(v == x).sum() for x in v])
    assert np.array_equal(R[:N], L + 0.5 * (E + 1))
    F, _ = S.tie_offset(it["C"], N, 512)
    k = (R + F)[:N]
    assert sorted(k.tolist()) == list(range(1, N + 1))
    assert np.array_equal(np.sort(v)[k.astype(int) - 1], v)
    # merged form used by the circuits: k = SumR(C + E*(delta - 1/2)) (linearity of SumR)
    Em = 4 * it["C"] * (1 - it["C"])
    delta = np.zeros(512)
    for i in range(N):
        delta[i * N + i:(i + 1) * N] = 1
    merged = S.sum_r(it["C"] + Em * (delta - 0.5), N)
    assert np.array_equal(merged[:N], k)


@pytest.mark.parametrize("N,seeds", [(8, range(100)), (128, range(20))])
def test_composite_comparator_ranks_round_exactly(N, seeds):
    dg, df = W.RANK_CMP[N]
    gap = 0.01 if N == 8 else 2.0 ** -10
    worst = 0.0
    for s in seeds:
        v, _, _ = W.rank_workload(N, gap, s)
        R, _ = S.rank(v, N, 2 * N * N, (dg, df))
        exact = np.argsort(np.argsort(v)) + 1
        worst = max(worst, np.max(np.abs(R[:N] - exact)))
    assert worst < 0.45


@pytest.fixture(scope="module")
def p12(ora):
    P = ora.Params(**W.PSETS["P12"])
    return P


def test_oracle_rank8_matches_shadow_and_exact(ora, p12):
    N = 8
    dg, df = W.RANK_CMP[N]
    errs = []
    for seed in range(3):
        v, kseed, eseed = W.rank_workload(N, 0.01, seed)
        keys = ora.Keys(p12, kseed, p12.L, p12.rank_galois(N))
        ct = ora.encrypt(keys, v, p12.L, eseed)
        R = ora.rank(keys, ct, N, dg, df)
        assert R.level == 0
        got = ora.decrypt(keys, R, N)
        sh, _ = S.rank(v, N, p12.n // 2, (dg, df))
        errs.append(np.max(np.abs(got - sh[:N])))
        assert np.array_equal(np.round(got), np.argsort(np.argsort(v)) + 1)
    assert max(errs) < 1e-3


def test_oracle_matrix_ops_match_shadow(ora, p12):
    N = 8
    h = p12.n // 2
    v = np.linspace(0.05, 0.9, N)
    gal = sorted(set(p12.rank_galois(N)) | {p12.galois_left(N * (N - 1) >> i) for i in (1, 2, 3)}
                 | {p12.galois_left(1 << i) for i in range(3)})
    keys = ora.Keys(p12, bytes(range(32)), p12.L, gal)
    ct = ora.encrypt(keys, v, p12.L, bytes([5] * 32))
    x = S.embed(v, h)
    for name, fn, sfn in [("trans_r", ora.trans_r, S.trans_r), ("repl_r", ora.repl_r, S.repl_r),
                          ("sum_r", ora.sum_r, S.sum_r)]:
        got = ora.decrypt(keys, fn(keys, ct, N), 2 * N * N)
        want = sfn(x, N)[:2 * N * N]
        assert np.max(np.abs(got - want)) < 1e-4, name
    col = ora.trans_r(keys, ct, N)
    for name, fn, sfn in [("repl_c", ora.repl_c, S.repl_c), ("sum_c", ora.sum_c, S.sum_c),
                          ("trans_c", ora.trans_c, S.trans_c)]:
        got = ora.decrypt(keys, fn(keys, col, N), 2 * N * N)
        want = sfn(S.trans_r(x, N), N)[:2 * N * N]
        assert np.max(np.abs(got - want)) < 1e-4, name


@pytest.fixture(scope="module")
def t12d(ora):
    P = ora.Params(**W.PSETS["T12D"])
    keys = ora.Keys(P, bytes(range(32)), P.L, P.circuit_galois(8, 6))
    return P, keys


@pytest.mark.parametrize("seed", [0, 1])
def test_oracle_argmin8_ties_matches_shadow(ora, t12d, seed):
    P, keys = t12d
    N = 8
    cmp, ind = W.ARGMIN_CMP[N]
    v, _, eseed = W.tied_workload(N, seed, 0.01)
    assert len(set(v.tolist())) < N                   # the workload has ties
    ct = ora.encrypt(keys, v, P.L, eseed)
    oh, val = ora.argmin(keys, ct, N, cmp, ind)
    assert oh.level == P.L - ora.argmin_depth(cmp, ind) + 1 and val.level == P.L - ora.argmin_depth(cmp, ind)
    got_oh, got_val = ora.decrypt(keys, oh, N), ora.decrypt(keys, val, 1)[0]
    sh_oh, sh_val, _ = S.argmin_circuit(v, N, P.n // 2, cmp, ind)
    assert np.max(np.abs(got_oh - sh_oh[:N])) < 1e-3 and abs(got_val - sh_val[0]) < 1e-3
    want = np.zeros(N)
    want[int(np.argmin(v))] = 1.0                    # lowest index among the minima
    assert np.array_equal(np.round(got_oh), want)
    assert abs(got_val - v.min()) < 0.01


def test_oracle_sort8_matches_shadow(ora, t12d):
    P, keys = t12d
    N = 8
    cmp, ind = W.SORT_CMP[N]
    v, _, eseed = W.rank_workload(N, 0.01, 3)
    ct = ora.encrypt(keys, v, P.L, eseed)
    s = ora.sort(keys, ct, N, cmp, ind)
    assert s.level == P.L - ora.sort_depth(cmp, ind)
    got = ora.decrypt(keys, s, N)
    assert np.max(np.abs(got - S.sort_circuit(v, N, P.n // 2, cmp, ind)[:N])) < 1e-3
    assert np.max(np.abs(got - np.sort(v))) < 1e-3


@pytest.mark.parametrize("N", [8, 32, 128])
def test_shadow_argmin_and_sort_compositions(N):
    """The compositions used per N give a correct one-hot / sorted vector (plaintext shadow)."""
    cmp, ind = W.ARGMIN_CMP[N]
    gap = 0.01 if N == 8 else 2.0 ** -10
    for seed in range(10):
        v, _, _ = W.tied_workload(N, seed, gap)
        oh, val, _ = S.argmin_circuit(v, N, 2 * N * N, cmp, ind)
        want = np.zeros(N)
        want[int(np.argmin(v))] = 1.0
        assert np.max(np.abs(oh[:N] - want)) < 0.1
    cmp, ind = W.SORT_CMP[N]
    for seed in range(10):
        v, _, _ = W.rank_workload(N, gap, seed)
        assert np.max(np.abs(S.sort_circuit(v, N, 2 * N * N, cmp, ind)[:N] - np.sort(v))) < 1e-3


def _kth(v, k):
    """index of the k-th smallest (ties: lowest index first) and its value"""
    order = np.argsort(v, kind="stable")
    return int(order[k - 1]), float(np.sort(v)[k - 1])


@pytest.mark.parametrize("N", [8, 16, 32, 64, 128])
def test_shadow_order_statistic_without_ties(N):
    """Order statistic k (section 3.2) on distinct values: the one-hot lands on
    the k-th smallest and the value equals it, for k = 1, N/2 and N."""
    cmp, ind = W.ORDER_CMP[N]
    gap = 0.01 if N == 8 else 2.0 ** -10
    for seed in range(12):
        v, _, _ = W.rank_workload(N, gap, 300 + seed)
        for k in sorted({1, max(2, N // 2), N}):
            oh, val, kv = S.order_stat_circuit(v, N, 2 * N * N, k, cmp, ind, tie=False)
            j, want = _kth(v, k)
            assert np.array_equal(np.round(oh[:N]), np.eye(N)[j]), (seed, k)
            assert abs(val[0] - want) < 1e-3, (seed, k)
            # without tie-correction k_j is the rank (section 3.1)
            assert np.array_equal(np.round(kv[:N]), np.argsort(np.argsort(v)) + 1)


@pytest.mark.parametrize("N", [8, 128])
def test_shadow_order_statistic_with_ties(N):
    """Tie-corrected order statistic (section 4): among equal values the lowest
    index comes first, so argmax lands on the highest index of the maxima."""
    for seed in range(6 if N == 128 else 20):
        v, _, _ = W.tied_workload(N, 40 + seed, 0.01 if N == 8 else 2.0 ** -10)
        assert len(set(v.tolist())) < N
        for k in (1, N // 2 + 1, N):
            cmp, ind = W.ARGMIN_CMP[N] if k == 1 else W.ORDER_TIE_CMP[N]
            oh, val, kv = S.order_stat_circuit(v, N, 2 * N * N, k, cmp, ind, tie=True)
            j, want = _kth(v, k)
            assert np.array_equal(np.round(oh[:N]), np.eye(N)[j]), (seed, k)
            assert abs(val[0] - want) < 1e-2, (seed, k)
            assert sorted(np.round(kv[:N]).astype(int).tolist()) == list(range(1, N + 1))


def test_oracle_argmin_is_tie_corrected_order_statistic_one(ora, t12d):
    P, keys = t12d
    N = 8
    cmp, ind = W.ARGMIN_CMP[N]
    v, _, eseed = W.tied_workload(N, 5, 0.01)
    ct = ora.encrypt(keys, v, P.L, eseed)
    a_oh, a_val = ora.argmin(keys, ct, N, cmp, ind)
    o_oh, o_val = ora.order_stat(keys, ct, N, 1, cmp, ind, True)
    assert np.array_equal(a_oh.export(), o_oh.export()) and np.array_equal(a_val.export(), o_val.export())
    assert ora.argmin_depth(cmp, ind) == ora.order_stat_depth(N, 1, cmp, ind, True)


@pytest.mark.parametrize("k,tie", [(1, False), (3, False), (8, False), (3, True), (8, True)])
def test_oracle_order_statistic_matches_shadow(ora, t12d, k, tie):
    P, keys = t12d
    N = 8
    cmp, ind = (W.ARGMIN_CMP[N] if k == 1 else W.ORDER_TIE_CMP[N]) if tie else W.ORDER_CMP[N]
    v, _, eseed = (W.tied_workload(N, 7, 0.01) if tie else W.rank_workload(N, 0.01, 7))
    ct = ora.encrypt(keys, v, P.L, eseed)
    oh, val = ora.order_stat(keys, ct, N, k, cmp, ind, tie)
    depth = ora.order_stat_depth(N, k, cmp, ind, tie)
    assert oh.level == P.L - depth + 1 and val.level == P.L - depth
    got_oh, got_val = ora.decrypt(keys, oh, N), ora.decrypt(keys, val, 1)[0]
    sh_oh, sh_val, _ = S.order_stat_circuit(v, N, P.n // 2, k, cmp, ind, tie)
    assert np.max(np.abs(got_oh - sh_oh[:N])) < 1e-3 and abs(got_val - sh_val[0]) < 1e-3
    j, want = _kth(v, k)
    assert np.array_equal(np.round(got_oh), np.eye(N)[j])
    assert abs(got_val - want) < 0.01


def test_oracle_tie_corrected_rank_is_a_permutation(ora, t12d):
    """Rank plus the tie-correction offset (section 4): equal values take
    consecutive ranks in index order, so the result is a permutation."""
    P, keys = t12d
    N = 8
    cmp = W.ORDER_TIE_CMP[N][0]
    v, _, eseed = W.tied_workload(N, 11, 0.01)
    assert len(set(v.tolist())) < N
    ct = ora.encrypt(keys, v, P.L, eseed)
    r = ora.rank_tie(keys, ct, N, *cmp)
    assert r.level == P.L - ora.rank_depth(*cmp) - 2
    got = ora.decrypt(keys, r, N)
    want = np.empty(N)
    want[np.argsort(v, kind="stable")] = np.arange(1, N + 1)
    assert np.max(np.abs(got - want)) < 0.05
    _, _, kv = S.order_stat_circuit(v, N, P.n // 2, 1, cmp, W.ORDER_TIE_CMP[N][1], True)
    assert np.max(np.abs(got - kv[:N])) < 5e-3    # values up to N; CKKS error of E = C (4 - 4C)


@pytest.mark.parametrize("N,b", [(64, 32), (256, 64), (512, 128)])
def test_shadow_multi_ciphertext_rank(N, b):
    """Multi-ciphertext ranking (section 5) with Equation (3) for the lower
    blocks equals the all-pairs sum over one N x N matrix and the exact ranks."""
    cmp = W.MULTI_RANK_CMP[N]
    for seed in range(3):
        v, _, _ = W.rank_workload(N, 2.0 ** -10, 500 + seed)
        R = np.concatenate([r[:b] for r in S.rank_multi_circuit(v, b, 2 * b * b, cmp)])
        C = (S.sign_composite(v[None, :] - v[:, None], *cmp) + 1.0) / 2.0   # C[m][n] = Cmp(v_n, v_m)
        assert np.max(np.abs(R - (C.sum(axis=0) + 0.5))) < 1e-9
        assert np.array_equal(np.round(R), np.argsort(np.argsort(v)) + 1)


@pytest.mark.parametrize("N", [64, 128])
def test_oracle_multi_ciphertext_rank_matches_shadow(ora, t12d, N):
    """the oracle's decoded multi-ciphertext ranks match the shadow and are exact"""
    P, _ = t12d
    b = 32                                   # 2^floor(log2 sqrt(n/2)) at n = 2^12
    cmp = W.MULTI_RANK_CMP[N]
    v, _, eseed = W.rank_workload(N, 2.0 ** -10, 600 + N)
    level = ora.rank_multi_depth(*cmp) + 1
    keys = ora.Keys(P, bytes(range(32)), level, P.circuit_galois(b, 4))
    blocks = [ora.encrypt(keys, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    R = ora.rank_multi(keys, blocks, b, *cmp)
    assert all(r.level == level - ora.rank_multi_depth(*cmp) for r in R)
    got = np.concatenate([ora.decrypt(keys, r, b) for r in R])
    sh = np.concatenate([r[:b] for r in S.rank_multi_circuit(v, b, P.n // 2, cmp)])
    # each key-switched rotation leaves a systematic ~5e-6 error in slot 0 of
    # every block; the self-comparisons on the diagonal (difference ~0, where
    # g^4 f is steepest, slope ~880) carry it into the ranks as ~0.01
    assert np.max(np.abs(got - sh)) < 0.02
    assert np.array_equal(np.round(got), np.argsort(np.argsort(v)) + 1)


def test_oracle_refuses_circuit_without_its_rotation_keys(ora, t12d):
    P, keys = t12d                           # keys for N = 8 only
    ct = ora.encrypt(keys, np.linspace(0, 1, 32), P.L, bytes([3] * 32))
    with pytest.raises(ora.OracleError):
        ora.rank(keys, ct, 32, 3, 1)


@pytest.mark.parametrize("N,b", [(64, 32), (128, 32)])
def test_shadow_multi_ciphertext_sort(N, b):
    """Multi-ciphertext sorting (section 5) returns the sorted vector block by block."""
    cmp, ind = W.MULTI_SORT_CMP[N]
    for seed in range(3):
        v, _, _ = W.rank_workload(N, 0.01 if N == 64 else 2.0 ** -10, 900 + seed)
        got = np.concatenate([s[:b] for s in S.sort_multi_circuit(v, b, 2 * b * b, cmp, ind)])
        assert np.max(np.abs(got - np.sort(v))) < 1e-4


def test_oracle_multi_ciphertext_sort_matches_shadow(ora):
    ps = W.PSETS["T12E"]
    P = ora.Params(**ps)
    N, b = 64, 32
    cmp, ind = W.MULTI_SORT_CMP[N]
    level = ora.sort_multi_depth(cmp, ind)
    keys = ora.Keys(P, bytes(range(4, 36)), level, P.circuit_galois(b, 4))
    v, _, eseed = W.rank_workload(N, 0.01, 950)
    blocks = [ora.encrypt(keys, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    out = ora.sort_multi(keys, blocks, b, cmp, ind)
    assert all(o.level == 0 for o in out)
    got = np.concatenate([ora.decrypt(keys, o, b) for o in out])
    sh = np.concatenate([s[:b] for s in S.sort_multi_circuit(v, b, P.n // 2, cmp, ind)])
    assert np.max(np.abs(got - sh)) < 1e-3
    assert np.max(np.abs(got - np.sort(v))) < 1e-3


@pytest.mark.parametrize("N", [8, 16, 64])
def test_shadow_column_form_sort_is_exact_and_equals_row_form(N):
    """Column-form sorting (section 3.3): with the ideal comparator and
    indicator it returns the sorted vector in row 0 (nothing elsewhere), and
    with the f/g composites it equals the row-form sort."""
    rng = np.random.default_rng(N)
    v = W.min_gap_uniform(N, 0.01 if N <= 16 else 2.0 ** -10, rng)
    slots = 4 * N * N
    out = S.sort_col_circuit(v, N, slots, "ideal", "ideal")
    assert np.array_equal(out[:N], np.sort(v)) and not np.any(out[N:])
    cmp, ind = W.SORT_CMP[N]
    col = S.sort_col_circuit(v, N, slots, cmp, ind)
    row = S.sort_circuit(v, N, slots, cmp, ind)
    assert np.max(np.abs(col[:N] - row[:N])) < 1e-9


def test_oracle_column_form_sort_matches_shadow(ora, t12d):
    P, keys = t12d
    N = 8
    cmp, ind = W.SORT_CMP[N]
    depth = ora.sort_col_depth(cmp, ind)
    assert depth == ora.sort_depth(cmp, ind) - 1        # no TransC mask
    v, _, eseed = W.rank_workload(N, 0.01, 4)
    s = ora.sort_col(keys, ora.encrypt(keys, v, depth, eseed), N, cmp, ind)
    assert s.level == 0
    got = ora.decrypt(keys, s, N)
    sh = S.sort_col_circuit(v, N, P.n // 2, cmp, ind)
    assert np.max(np.abs(got - sh[:N])) < 1e-3
    assert np.max(np.abs(got - np.sort(v))) < 1e-3


@pytest.mark.parametrize("x", [0.02, 0.3, 1.0, 1.7])
def test_goldschmidt_closed_form(x):
    """prod_{i<d} (1 + b^(2^i)) = (1 - b^(2^d)) / (1 - b) with b = 1 - x: the
    inverse of x up to the relative error b^(2^d)."""
    for d in (2, 5, 9):
        b = 1.0 - x
        assert abs(S.goldschmidt_inverse(x, d) - (1.0 - b ** (2 ** d)) / x) < 1e-9 / x


def _tripled_case(N, seed):
    v, _, eseed = W.tripled_workload(N, seed, triples=1, gap=0.01 if N <= 16 else 2.0 ** -10)
    u, c = np.unique(v, return_counts=True)
    t = u[np.argmax(c)]                       # the tripled value
    below = int(np.sum(v < t))
    return v, eseed, t, below


@pytest.mark.parametrize("N", [8, 32])
def test_shadow_order_stat_division(N):
    """Section 3.2's value by division: with the ideal comparator and
    indicator, the mask of rank |L| + 2 has the three copies of the tripled
    value and the quotient is that value; rank |L| + 1 has no element and
    the value is 0; a one-hot rank gives its element."""
    v, _, t, below = _tripled_case(N, 3)
    d = 9
    for k, want in ((below + 2, t), (below + 1, 0.0)):
        O, val = S.order_stat_div_circuit(v, N, 4 * N * N, k, "ideal", "ideal", d)
        assert np.sum(O[:N]) == (3 if want else 0)
        assert abs(val[0] - want) < 1e-6
    distinct = [k for k in range(1, N + 1) if k < below + 1 or k > below + 3]
    k = distinct[0]
    _, val = S.order_stat_div_circuit(v, N, 4 * N * N, k, "ideal", "ideal", d)
    rank = (np.argsort(np.argsort(v)) + 1).astype(float)
    assert abs(val[0] - v[rank == k][0]) < 1e-6 * N


@pytest.fixture(scope="module")
def t12e(ora):
    P = ora.Params(**W.PSETS["T12E"])
    return P, ora.Keys(P, bytes(range(1, 33)), P.L, P.circuit_galois(8, 2))


def test_oracle_order_stat_division_matches_shadow(ora, t12e):
    P, keys = t12e
    N, d = 8, 6
    cmp, ind = W.ORDER_CMP[N]
    v, eseed, t, below = _tripled_case(N, 5)
    k = below + 2
    depth = ora.order_stat_div_depth(N, k, cmp, ind, d)
    assert depth == ora.order_stat_depth(N, k, cmp, ind, False) + d + 2
    oh, val = ora.order_stat_div(keys, ora.encrypt(keys, v, depth, eseed), N, k, cmp, ind, d)
    assert val.level == 0
    got = ora.decrypt(keys, val, 1)[0]
    sO, sval = S.order_stat_div_circuit(v, N, P.n // 2, k, cmp, ind, d)
    assert abs(got - sval[0]) < 1e-3 and abs(got - t) < 1e-3
    assert np.array_equal(np.round(ora.decrypt(keys, oh, N)), (v == t).astype(float))


@pytest.mark.parametrize("N", [3, 5, 6, 7, 12])
def test_shadow_padded_rank_is_exact(N):
    """Rank of N values that are not a power of two (section 3.1): padded with
    zeros and the comparison matrix masked to its N x N block, the ideal
    comparator gives the exact ranks of the real values (the zeros of the
    padding are not counted), ties included."""
    rng = np.random.default_rng(N)
    v = rng.uniform(0.0, 1.0, N)
    v[N // 2] = v[0]                          # a tie
    Np = 1 << (N - 1).bit_length()
    R = S.rank_padded(v, 4 * Np * Np, "ideal")
    less = (v[None, :] < v[:, None]).sum(axis=1)
    equal = (v[None, :] == v[:, None]).sum(axis=1)
    assert np.array_equal(R[:N], less + 0.5 * (equal + 1))


def test_oracle_padded_rank_matches_shadow(ora, t12d):
    P, keys = t12d
    cmp = W.RANK_CMP[8]
    for N in (5, 7):
        depth = ora.rank_depth_n(N, cmp)
        assert depth == ora.rank_depth(*cmp) + 1
        assert ora.rank_depth_n(8, cmp) == ora.rank_depth(*cmp)
        v, _, eseed = W.rank_workload(N, 0.01, N)
        r = ora.rank(keys, ora.encrypt(keys, v, depth, eseed), N, *cmp)
        assert r.level == 0
        got = ora.decrypt(keys, r, N)
        assert np.max(np.abs(got - S.rank_padded(v, P.n // 2, cmp)[:N])) < 1e-3
        assert np.array_equal(np.round(got), np.argsort(np.argsort(v)) + 1)


def test_oracle_padded_tie_rank_is_a_permutation(ora, t12d):
    P, keys = t12d
    cmp = W.ORDER_TIE_CMP[8][0]
    N = 6
    v = np.array([0.3, 0.7, 0.3, 0.1, 0.9, 0.7])
    depth = ora.rank_depth_n(N, cmp, True)
    r = ora.rank_tie(keys, ora.encrypt(keys, v, depth, bytes(range(2, 34))), N, *cmp)
    got = ora.decrypt(keys, r, N)
    want = np.empty(N)
    want[np.argsort(v, kind="stable")] = np.arange(1, N + 1)
    assert np.max(np.abs(got - want)) < 0.05


def _window_mean(v, a, b):
    """mean of the order statistics a..b (1-based) of v"""
    return float(np.mean(np.sort(v)[a - 1:b]))


@pytest.mark.parametrize("N", [5, 6, 7, 8, 12, 16])
def test_shadow_order_range_ideal_is_exact(N):
    """The rank window with the ideal comparator and indicator: the mask holds
    exactly the elements of tie-corrected rank a..b (lowest index first among
    equal values), the value is the mean of the statistics a..b, the median
    of section 4 included (both middle statistics halved for an even N, the
    middle one for an odd N), padded layouts included."""
    rng = np.random.default_rng(70 + N)
    v = np.round(rng.uniform(0.0, 1.0, N), 2)
    v[N - 1] = v[1]                                   # a tie
    Np = 1 << (N - 1).bit_length()
    order = np.argsort(v, kind="stable")
    windows = {(1, 1), (N, N), (1, N - 1), (2, N), (2, max(2, N - 2))}
    windows.add((N // 2, N // 2 + 1) if N % 2 == 0 else ((N + 1) // 2, (N + 1) // 2))
    for a, b in sorted(windows):
        oh, val, kv = S.order_range_circuit(v, 4 * Np * Np, a, b, "ideal", "ideal", True)
        want = np.zeros(N)
        want[order[a - 1:b]] = 1.0
        assert np.array_equal(oh[:N], want), (a, b)
        assert abs(val[0] - _window_mean(v, a, b)) < 1e-12, (a, b)
        assert np.all(oh[N:] == 0.0)
    med = S.order_range_circuit(v, 4 * Np * Np, *(((N // 2, N // 2 + 1)) if N % 2 == 0 else
                                                  ((N + 1) // 2, (N + 1) // 2)), "ideal", "ideal", True)[1][0]
    assert abs(med - np.median(v)) < 1e-12


@pytest.mark.parametrize("N", [8, 128])
def test_shadow_order_range_reduces_to_order_statistic(N):
    """a = b = k is the order statistic: identical slot vectors, both with and
    without tie-correction, under the composite comparators."""
    for tie in (False, True):
        gap = 0.01 if N == 8 else 2.0 ** -10
        v, _, _ = (W.tied_workload(N, 3, gap) if tie else W.rank_workload(N, gap, 3))
        for k in (1, N // 2, N):
            cmp, ind = (W.ARGMIN_CMP[N] if k == 1 else W.ORDER_TIE_CMP[N]) if tie else W.ORDER_CMP[N]
            o1, v1, k1 = S.order_stat_circuit(v, N, 2 * N * N, k, cmp, ind, tie)
            o2, v2, k2 = S.order_range_circuit(v, 2 * N * N, k, k, cmp, ind, tie)
            assert np.array_equal(k1, k2) and np.array_equal(v1, v2) and np.array_equal(o1, o2)


@pytest.mark.parametrize("N", [8, 128])
def test_shadow_median_with_composites(N):
    """Median of an even N (section 4) with the tabled composites: the
    window [N/2, N/2 + 1] selects both middle elements, the value is their
    mean, distinct and tied inputs."""
    gap = 0.01 if N == 8 else 2.0 ** -10
    for seed in range(4):
        for tie in (False, True):
            v, _, _ = (W.tied_workload(N, 90 + seed, gap) if tie else W.rank_workload(N, gap, 90 + seed))
            cmp, ind = W.ORDER_TIE_CMP[N] if tie else W.ORDER_CMP[N]
            oh, val, _ = S.order_range_circuit(v, 2 * N * N, N // 2, N // 2 + 1, cmp, ind, tie)
            order = np.argsort(v, kind="stable")
            want = np.zeros(N)
            want[order[N // 2 - 1:N // 2 + 1]] = 1.0
            assert np.array_equal(np.round(oh[:N]), want), (seed, tie)
            assert abs(val[0] - np.median(v)) < 1e-2, (seed, tie)


def test_oracle_order_range_k_equals_order_statistic_bits(ora, t12d):
    """The order statistic is the window a = b = k: identical ciphertexts."""
    P, keys = t12d
    N = 8
    v, _, eseed = W.tied_workload(N, 11, 0.01)
    ct = ora.encrypt(keys, v, P.L, eseed)
    for k, tie in ((1, True), (5, True), (8, False)):
        cmp, ind = (W.ARGMIN_CMP[N] if k == 1 else W.ORDER_TIE_CMP[N]) if tie else W.ORDER_CMP[N]
        assert ora.order_range_depth(N, k, k, cmp, ind, tie) == ora.order_stat_depth(N, k, cmp, ind, tie)
        a_oh, a_val = ora.order_stat(keys, ct, N, k, cmp, ind, tie)
        b_oh, b_val = ora.order_range(keys, ct, N, k, k, cmp, ind, tie)
        assert np.array_equal(a_oh.export(), b_oh.export()) and np.array_equal(a_val.export(), b_val.export())


@pytest.mark.parametrize("N,a,b,tie", [(8, 4, 5, True), (8, 4, 5, False), (8, 1, 3, True), (8, 6, 8, False),
                                       (6, 3, 4, True), (7, 4, 4, True), (5, 1, 2, True), (7, 5, 7, True)])
def test_oracle_order_range_matches_shadow(ora, t12d, N, a, b, tie):
    """Encrypted rank window (median, lower and upper ranges, padded N) against
    the slot shadow and the exact mean of the statistics a..b."""
    P, keys = t12d
    cmp, ind = W.ORDER_TIE_CMP[8] if tie else W.ORDER_CMP[8]
    v, _, eseed = (W.tied_workload(N, 20 + N, 0.01) if tie else W.rank_workload(N, 0.01, 20 + N))
    depth = ora.order_range_depth(N, a, b, cmp, ind, tie)
    pad = 1 if (N & (N - 1)) else 0
    assert depth == ora.order_stat_depth(8, 2 if (a > 1 and b < N) else 1, cmp, ind, tie) + pad
    oh, val = ora.order_range(keys, ora.encrypt(keys, v, depth, eseed), N, a, b, cmp, ind, tie)
    assert val.level == 0 and oh.level == 1
    got_oh, got_val = ora.decrypt(keys, oh, N), ora.decrypt(keys, val, 1)[0]
    sh_oh, sh_val, _ = S.order_range_circuit(v, P.n // 2, a, b, cmp, ind, tie)
    assert np.max(np.abs(got_oh - sh_oh[:N])) < 1e-3 and abs(got_val - sh_val[0]) < 1e-3
    want = np.zeros(N)
    want[np.argsort(v, kind="stable")[a - 1:b]] = 1.0
    assert np.array_equal(np.round(got_oh), want)
    assert abs(got_val - _window_mean(v, a, b)) < 0.01


def test_oracle_order_range_rejects(ora, t12d):
    P, keys = t12d
    cmp, ind = W.ORDER_TIE_CMP[8]
    ct = ora.encrypt(keys, np.linspace(0.1, 0.8, 8), P.L, bytes(32))
    for N, a, b, tie in ((8, 1, 8, True), (8, 0, 2, True), (8, 3, 2, True), (8, 2, 9, True), (6, 2, 3, False)):
        with pytest.raises(ora.OracleError, match="invalid"):
            ora.order_range(keys, ct, N, a, b, cmp, ind, tie)
    with pytest.raises(ora.OracleError, match="depth"):
        ora.order_range(keys, ora.encrypt(keys, np.linspace(0.1, 0.8, 8), 3, bytes(32)), 8, 4, 5, cmp, ind, True)


@pytest.mark.parametrize("name,N,seed", [("median128_p17o", 128, 3), ("median101_p17s", 101, 4)])
def test_stored_median_goldens_are_medians(name, N, seed):
    """The stored full-size median digests decode to a median: the mask marks
    the middle element(s) of the regenerated workload (lowest index first
    among equal values) and the value is np.median within 5e-3."""
    path = os.path.join(os.path.dirname(__file__), "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip("golden not written")
    d = json.load(open(path))
    v, _, _ = W.tied_workload(N, seed)
    a, b = d["window"]
    assert (a, b) == ((N // 2, N // 2 + 1) if N % 2 == 0 else ((N + 1) // 2, (N + 1) // 2))
    want = np.zeros(N)
    want[np.argsort(v, kind="stable")[a - 1:b]] = 1.0
    assert np.array_equal(np.round(d["mask"]), want)
    assert abs(d["median"] - float(np.median(v))) == 0.0
    assert abs(d["value"] - float(np.median(v))) < 5e-3
