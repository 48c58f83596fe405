"""GPU parity of the tie-corrected argmin and of sorting.

Small ring (n = 2^12, 35 primes): element-by-element against the oracle run
in the test.  Full size (n = 2^17, 41 + 10 primes, N = 128): against the
digests written by tests/golden/make_golden.py (oracle only)."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_2412_15126_amd import workloads as W

import value_bound as VB

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small(ora):
    import paper_2412_15126_amd as ckr
    ps = W.PSETS["T12D"]
    P = ora.Params(**ps)
    seed = bytes(range(32))
    say("[gpu] T12D keys")
    okeys = ora.Keys(P, seed, P.L, P.circuit_galois(8, 6))
    ctx = ckr.Context(ps)
    gkeys = ctx.keygen(seed, P.L, [8], what=6)
    return dict(P=P, okeys=okeys, ctx=ctx, gkeys=gkeys, ckr=ckr)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_argmin8_with_ties_bit_exact(ora, small, seed):
    P, ctx = small["P"], small["ctx"]
    N = 8
    cmp, ind = W.ARGMIN_CMP[N]
    v, _, eseed = W.tied_workload(N, seed, 0.01)
    say(f"[gpu] argmin8 seed {seed}")
    o = ora.encrypt(small["okeys"], v, P.L, eseed)
    g = ctx.encrypt(small["gkeys"], v, P.L, eseed)
    ooh, oval = ora.argmin(small["okeys"], o, N, cmp, ind)
    goh, gval = ctx.argmin(small["gkeys"], g, N, cmp, ind)
    assert np.array_equal(ooh.export(), goh.export())
    assert np.array_equal(oval.export(), gval.export())
    want = np.zeros(N)
    want[int(np.argmin(v))] = 1.0
    assert np.array_equal(np.round(ctx.decrypt(small["gkeys"], goh, N)), want)
    assert abs(ctx.decrypt(small["gkeys"], gval, 1)[0] - v.min()) <= VB.tolerance(v, 1, 1, cmp, ind, True, 12)


def test_argmin8_all_equal_picks_first(ora, small):
    P, ctx = small["P"], small["ctx"]
    N = 8
    cmp, ind = W.ARGMIN_CMP[N]
    v = np.full(N, 0.375)
    o = ora.encrypt(small["okeys"], v, P.L, bytes([7] * 32))
    g = ctx.encrypt(small["gkeys"], v, P.L, bytes([7] * 32))
    ooh, oval = ora.argmin(small["okeys"], o, N, cmp, ind)
    goh, gval = ctx.argmin(small["gkeys"], g, N, cmp, ind)
    assert np.array_equal(ooh.export(), goh.export()) and np.array_equal(oval.export(), gval.export())
    assert np.array_equal(np.round(ctx.decrypt(small["gkeys"], goh, N)), np.eye(N)[0])


@pytest.mark.parametrize("seed", [0, 1])
def test_sort8_bit_exact(ora, small, seed):
    P, ctx = small["P"], small["ctx"]
    N = 8
    cmp, ind = W.SORT_CMP[N]
    v, _, eseed = W.rank_workload(N, 0.01, 20 + seed)
    say(f"[gpu] sort8 seed {seed}")
    o = ora.encrypt(small["okeys"], v, P.L, eseed)
    g = ctx.encrypt(small["gkeys"], v, P.L, eseed)
    so = ora.sort(small["okeys"], o, N, cmp, ind)
    sg = ctx.sort(small["gkeys"], g, N, cmp, ind)
    assert np.array_equal(so.export(), sg.export())
    assert np.max(np.abs(ctx.decrypt(small["gkeys"], sg, N) - np.sort(v))) <= VB.sort_tolerance(v, cmp, ind)


def test_circuit_depth_errors(small):
    ckr, ctx = small["ckr"], small["ctx"]
    g = ctx.encrypt(small["gkeys"], np.linspace(0, 1, 8), 20, bytes([1] * 32))
    for call in (lambda: ctx.argmin(small["gkeys"], g, 8, *W.ARGMIN_CMP[8]),
                 lambda: ctx.sort(small["gkeys"], g, 8, *W.SORT_CMP[8])):
        with pytest.raises(ckr.CkrError) as e:
            call()
        assert e.value.status == -3


@pytest.fixture(scope="module")
def p17():
    import paper_2412_15126_amd as ckr
    say("[gpu] P17 context")
    ps = W.PSETS["P17"]
    return ckr.Context(ps), ps


def test_argmin128_full_size_matches_golden(p17o):
    ctx, ps = p17o
    gold = json.load(open(os.path.join(GOLD, "argmin128_p17o.json")))
    N = 128
    cmp, ind = W.ARGMIN_CMP[N]
    import paper_2412_15126_amd as ckr
    level = ckr.argmin_depth(cmp, ind)
    assert level == gold["level"] == 43
    v, kseed, eseed = W.tied_workload(N, 0)
    say("[gpu] P17O argmin keygen")
    keys = ctx.keygen(kseed, level, [N], what=2)
    g = ctx.encrypt(keys, v, level, eseed)
    say("[gpu] P17O argmin")
    oh, val = ctx.argmin(keys, g, N, cmp, ind)
    assert hashlib.sha256(oh.export().tobytes()).hexdigest() == gold["sha256_onehot"]
    assert hashlib.sha256(val.export().tobytes()).hexdigest() == gold["sha256_value"]
    dec = ctx.decrypt(keys, oh, N)
    assert int(np.argmax(dec)) == int(np.argmin(v)) == gold["argmin"]
    assert np.array_equal(np.round(dec), np.eye(N)[gold["argmin"]])
    # the derived bound (tests/value_bound.py): indicator leakage at each rank's
    # distance from 1.5, times the value, plus the noise allowance; the mask's
    # decoded deviations lie within their per-slot bounds plus that allowance
    delta = VB.rank_error(v, cmp, True, 1 << 16)
    assert np.all(np.abs(dec - np.eye(N)[gold["argmin"]]) <= VB.mask_bound(v, 1, 1, ind, delta) + VB.ETA)
    tol = VB.value_bound(v, 1, 1, ind, delta, VB.ETA)
    assert tol < 2.0 ** -11          # below half the workload's value gap
    assert abs(ctx.decrypt(keys, val, 1)[0] - v.min()) <= tol


def test_argmin128_hundred_seeds_one_hot_and_value_within_bound(p17o):
    """Tie-corrected argmin of N = 128 over seeds 0..99 (tied workloads, one key), in
    batches of 4: every one-hot rounds to the first minimum, and every value
    lies within its derived bound (reading of Algorithm Order Statistic's
    value, tests/value_bound.py)."""
    ctx, ps = p17o
    N = 128
    cmp, ind = W.ARGMIN_CMP[N]
    import paper_2412_15126_amd as ckr
    level = ckr.argmin_depth(cmp, ind)
    keys = ctx.keygen(W.tied_workload(N, 0)[1], level, [N], what=2)
    qs = [W.tied_workload(N, s) for s in range(100)]
    worst = 0.0
    for b0 in range(0, 100, 4):
        part = qs[b0:b0 + 4]
        say(f"[gpu] P17O argmin-128 seeds {b0}..{b0 + 3}")
        outs = ctx.run_batch(keys, "argmin", [ctx.encrypt(keys, v, level, e) for v, _, e in part], N, cmp, ind)
        for (v, _, _), (oh, val) in zip(part, outs):
            assert np.array_equal(np.round(ctx.decrypt(keys, oh, N)), np.eye(N)[np.argmin(v)])
            err = abs(ctx.decrypt(keys, val, 1)[0] - v.min())
            assert err <= VB.tolerance(v, 1, 1, cmp, ind, True, 17), (b0, err)
            worst = max(worst, err)
    say(f"[gpu] argmin-128, 100 seeds: max |value - min| {worst:.2e}")


def test_argmin128_chebyshev_full_size_matches_golden(p17):
    """The paper's setting for the minimum: Chebyshev comparator and
    indicator of degree 2^11 - 1 (12 levels each), tie-corrected, N = 128."""
    ctx, ps = p17
    gold = json.load(open(os.path.join(GOLD, "argmin128_p17_cheb.json")))
    N = 128
    cmp = ind = W.CHEB_CMP[N]
    level = gold["level"]
    import paper_2412_15126_amd as ckr
    assert level == ckr.order_stat_depth(N, 1, cmp, ind, True)
    v, kseed, eseed = W.tied_workload(N, 0)
    say("[gpu] P17 chebyshev argmin keygen")
    keys = ctx.keygen(kseed, level, [N], what=2)
    say("[gpu] P17 chebyshev argmin")
    oh, val = ctx.order_stat(keys, ctx.encrypt(keys, v, level, eseed), N, 1, cmp, ind, True)
    assert [hashlib.sha256(c.export().tobytes()).hexdigest() for c in (oh, val)] == gold["sha256"]
    assert np.array_equal(np.round(ctx.decrypt(keys, oh, N)), np.eye(N)[gold["argmin"]])
    # the derived bound is loose here: with the Chebyshev comparator the
    # tie-corrected k_j miss their integers by up to ~0.88 (Gibbs overshoot at
    # one gap), and the indicator cannot separate ranks 1 and 2 by its bound
    assert abs(ctx.decrypt(keys, val, 1)[0] - v.min()) <= VB.tolerance(v, 1, 1, cmp, ind, True, 17)


def test_argmin128_chebyshev_real_part_projection(p17):
    """The Chebyshev indicator's argument is projected onto its real part:
    without it, an imaginary part of ~1e-3 inherited from the comparator made
    one slot of one of these queries blow up to 231 (the degree-2047
    indicator grows like cosh(n y / sqrt(1 - x^2)) off the real axis).  Every
    query's one-hot is right and agrees with the slot-level shadow."""
    from oracle import shadow as S
    import paper_2412_15126_amd as ckr
    ctx, ps = p17
    N = 128
    cmp = ind = W.CHEB_CMP[N]
    level = ckr.order_stat_depth(N, 1, cmp, ind, True)
    keys = ctx.keygen(bytes(range(11, 43)), level, [N], what=2)
    for seed in range(2000, 2004):
        v, _, eseed = W.tied_workload(N, seed)
        say(f"[gpu] P17 chebyshev argmin seed {seed}")
        oh, val = ctx.order_stat(keys, ctx.encrypt(keys, v, level, eseed), N, 1, cmp, ind, True)
        d = ctx.decrypt(keys, oh, N)
        sh, _, _ = S.order_stat_circuit(v, N, 1 << 16, 1, cmp, ind, True)
        # a guard against the blow-up (231 without the projection), not a
        # precision claim: the rest is CKKS noise through the indicator's
        # steep flanks; the one-hot's exactness below is the parity check
        assert np.max(np.abs(d - sh[:N])) < 0.02, seed
        assert np.array_equal(np.round(d), np.eye(N)[np.argsort(v, kind="stable")[0]]), seed


@pytest.mark.parametrize("seed", [0, 1])
def test_sort8_column_form_bit_exact(ora, small, seed):
    P, ctx = small["P"], small["ctx"]
    N = 8
    cmp, ind = W.SORT_CMP[N]
    level = ora.sort_col_depth(cmp, ind)
    assert level == small["ckr"].sort_col_depth(cmp, ind) == ora.sort_depth(cmp, ind) - 1
    v, _, eseed = W.rank_workload(N, 0.01, 20 + seed)
    say(f"[gpu] column-form sort8 seed {seed}")
    o = ora.sort_col(small["okeys"], ora.encrypt(small["okeys"], v, level, eseed), N, cmp, ind)
    g = ctx.sort_col(small["gkeys"], ctx.encrypt(small["gkeys"], v, level, eseed), N, cmp, ind)
    assert np.array_equal(o.export(), g.export())
    assert np.max(np.abs(ctx.decrypt(small["gkeys"], g, N) - np.sort(v))) <= VB.sort_tolerance(v, cmp, ind)


def test_sort8_column_form_batch_equals_single(small):
    ctx = small["ctx"]
    N = 8
    cmp, ind = W.SORT_CMP[N]
    level = small["ckr"].sort_col_depth(cmp, ind)
    qs = [W.rank_workload(N, 0.01, 40 + i) for i in range(3)]
    cts = [ctx.encrypt(small["gkeys"], v, level, e) for v, _, e in qs]
    singles = [ctx.sort_col(small["gkeys"], c, N, cmp, ind).export() for c in cts]
    for rep in range(3):
        say(f"[gpu] column-form sort8 batch pass {rep}")
        outs = ctx.run_batch(small["gkeys"], "sort_col", cts, N, cmp, ind)
        assert all(np.array_equal(a.export(), b) for a, b in zip(outs, singles))


def test_sort128_column_form_full_size_matches_golden(p17):
    ctx, ps = p17
    gold = json.load(open(os.path.join(GOLD, "sort128_p17_col.json")))
    N = 128
    cmp, ind = W.SORT_CMP[N]
    level = gold["level"]
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    say("[gpu] P17 column-form sort keygen")
    keys = ctx.keygen(kseed, level, [N], what=2)
    say("[gpu] P17 column-form sort")
    s = ctx.sort_col(keys, ctx.encrypt(keys, v, level, eseed), N, cmp, ind)
    assert hashlib.sha256(s.export().tobytes()).hexdigest() == gold["sha256"]
    assert np.max(np.abs(ctx.decrypt(keys, s, N) - np.sort(v))) <= VB.sort_tolerance(v, cmp, ind)


def test_kth64_division_full_size_matches_golden(ora):
    """Order statistic with the value by division at n = 2^17 (48 + 12
    primes): N = 64 with four tripled values, k = the smallest tripled value's
    rank, 8 Goldschmidt steps, against the oracle-written digests."""
    import paper_2412_15126_amd as ckr
    gold = json.load(open(os.path.join(GOLD, "kth64_p17s_div.json")))
    N = 64
    cmp, ind = W.ORDER_CMP[N]
    v, kseed, eseed = W.tripled_workload(N, 0, triples=4)
    ctx = ckr.Context(W.PSETS["P17S"])
    say("[gpu] P17S division keygen")
    keys = ctx.keygen(kseed, gold["level"], [N], what=2)
    say("[gpu] P17S order statistic with division")
    (oh, val), = ctx.order_stat_div(keys, [ctx.encrypt(keys, v, gold["level"], eseed)], N, gold["k"], cmp, ind,
                                    gold["iters"])
    assert [hashlib.sha256(c.export().tobytes()).hexdigest() for c in (oh, val)] == gold["sha256"]
    assert abs(ctx.decrypt(keys, val, 1)[0] - gold["value_expected"]) <= VB.division_bound(v, gold["k"], cmp, ind,
                                                                                          gold["iters"])
    assert np.array_equal(np.round(ctx.decrypt(keys, oh, N)), (v == gold["value_expected"]).astype(float))


def test_sort128_full_size_matches_golden(p17):
    ctx, ps = p17
    gold = json.load(open(os.path.join(GOLD, "sort128_p17.json")))
    N = 128
    cmp, ind = W.SORT_CMP[N]
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    say("[gpu] P17 sort keygen")
    keys = ctx.keygen(kseed, ps["L"], [N], what=4)
    g = ctx.encrypt(keys, v, ps["L"], eseed)
    say("[gpu] P17 sort")
    s = ctx.sort(keys, g, N, cmp, ind)
    assert hashlib.sha256(s.export().tobytes()).hexdigest() == gold["sha256"]
    assert np.max(np.abs(ctx.decrypt(keys, s, N) - np.sort(v))) <= VB.sort_tolerance(v, cmp, ind)


def test_p17_encrypt_mul_bit_exact(ora, p17):
    """n = 2^17 transforms, relinearisation and rescale against the oracle."""
    ctx, ps = p17
    ora.set_threads(min(16, os.cpu_count() or 1))
    P = ora.Params(**ps)
    seed = bytes(range(5, 37))
    say("[gpu] P17 relin keys")
    okeys = ora.Keys(P, seed, ps["L"], [])
    gkeys = ctx.keygen(seed, ps["L"], [])
    v = np.random.default_rng(3).uniform(0, 1, 1000)
    for level in (ps["L"], 9):
        o = ora.encrypt(okeys, v, level, bytes([2] * 32))
        g = ctx.encrypt(gkeys, v, level, bytes([2] * 32))
        assert np.array_equal(o.export(), g.export())
        assert np.array_equal(ora.mul(okeys, o, o).export(), ctx.mul(gkeys, g, g).export())


def test_argmin_and_sort_batched_graphs_equal_single(ora, small):
    """run_batch for argmin and sort (eager, then captured, then replayed) equals single calls."""
    ctx, keys, P = small["ctx"], small["gkeys"], small["P"]
    N = 8
    for kind in ("argmin", "sort"):
        cmp, ind = (W.ARGMIN_CMP if kind == "argmin" else W.SORT_CMP)[N]
        cts, singles = [], []
        for seed in range(3):
            v, _, eseed = (W.tied_workload(N, seed, 0.01) if kind == "argmin" else W.rank_workload(N, 0.01, seed))
            g = ctx.encrypt(keys, v, P.L, eseed)
            cts.append(g)
            if kind == "argmin":
                oh, val = ctx.argmin(keys, g, N, cmp, ind)
                singles.append((oh.export(), val.export()))
            else:
                singles.append((ctx.sort(keys, g, N, cmp, ind).export(),))
        for rep in range(3):
            outs = ctx.run_batch(keys, kind, cts, N, cmp, ind)
            for s, o in zip(singles, outs):
                o = o if isinstance(o, tuple) else (o,)
                assert all(np.array_equal(a, b.export()) for a, b in zip(s, o)), (kind, rep)


def _order_cmp(N, k, tie):
    return (W.ARGMIN_CMP[N] if k == 1 else W.ORDER_TIE_CMP[N]) if tie else W.ORDER_CMP[N]


def _kth_index(v, k):
    return int(np.argsort(v, kind="stable")[k - 1])


@pytest.mark.parametrize("k,tie", [(1, False), (4, False), (8, False), (4, True), (8, True)])
def test_order_statistic8_bit_exact(ora, small, k, tie):
    """Order statistic k with and without tie-correction (one-sided indicator at
    the ends, window in the middle) against the oracle."""
    P, ctx = small["P"], small["ctx"]
    N = 8
    cmp, ind = _order_cmp(N, k, tie)
    v, _, eseed = W.tied_workload(N, 20 + k, 0.01) if tie else W.rank_workload(N, 0.01, 20 + k)
    say(f"[gpu] order statistic k={k} tie={tie}")
    o = ora.encrypt(small["okeys"], v, P.L, eseed)
    g = ctx.encrypt(small["gkeys"], v, P.L, eseed)
    ooh, oval = ora.order_stat(small["okeys"], o, N, k, cmp, ind, tie)
    goh, gval = ctx.order_stat(small["gkeys"], g, N, k, cmp, ind, tie)
    assert np.array_equal(ooh.export(), goh.export())
    assert np.array_equal(oval.export(), gval.export())
    assert np.array_equal(np.round(ctx.decrypt(small["gkeys"], goh, N)), np.eye(N)[_kth_index(v, k)])
    assert abs(ctx.decrypt(small["gkeys"], gval, 1)[0] - np.sort(v)[k - 1]) <= VB.tolerance(v, k, k, cmp, ind,
                                                                                              tie, 12)


def test_tie_corrected_rank8_bit_exact(ora, small):
    P, ctx = small["P"], small["ctx"]
    N = 8
    cmp = W.ORDER_TIE_CMP[N][0]
    v, _, eseed = W.tied_workload(N, 11, 0.01)
    o = ora.encrypt(small["okeys"], v, P.L, eseed)
    g = ctx.encrypt(small["gkeys"], v, P.L, eseed)
    ro = ora.rank_tie(small["okeys"], o, N, *cmp)
    rg = ctx.rank(small["gkeys"], g, N, cmp, tie=True)
    assert np.array_equal(ro.export(), rg.export())
    want = np.empty(N)
    want[np.argsort(v, kind="stable")] = np.arange(1, N + 1)
    assert np.array_equal(np.round(ctx.decrypt(small["gkeys"], rg, N)), want)


def test_mixed_batch_small_ring_bit_exact(ora, small):
    """Queries of every kind, several levels and group sizes in one run_mixed
    call (eager, then captured, then replayed): every output equals the
    oracle's result for that query alone."""
    P, ctx, okeys, gkeys = small["P"], small["ctx"], small["okeys"], small["gkeys"]
    N = 8
    specs = [dict(kind="rank", cmp=W.RANK_CMP[N]), dict(kind="rank", cmp=W.RANK_CMP[N]),
             dict(kind="order", k=1, tie=False), dict(kind="rank", cmp=W.RANK_CMP[N], level=P.L),
             dict(kind="order", k=3, tie=True), dict(kind="order", k=1, tie=False),
             dict(kind="sort"), dict(kind="argmin"), dict(kind="rank", cmp=W.ORDER_TIE_CMP[N][0], tie=True)]
    queries, want = [], []
    for i, s in enumerate(specs):
        tie = s.get("tie", False)
        v, _, eseed = W.tied_workload(N, 60 + i, 0.01) if tie or s["kind"] == "argmin" else W.rank_workload(N, 0.01, 60 + i)
        if s["kind"] == "rank":
            cmp, ind = s["cmp"], (0, 0)
            level = s.get("level", ora.rank_depth(*cmp) + (2 if tie else 0))
        elif s["kind"] == "order":
            cmp, ind = _order_cmp(N, s["k"], tie)
            level = ora.order_stat_depth(N, s["k"], cmp, ind, tie)
        elif s["kind"] == "sort":
            cmp, ind = W.SORT_CMP[N]
            level = ora.sort_depth(cmp, ind)
        else:
            cmp, ind = W.ARGMIN_CMP[N]
            level = ora.argmin_depth(cmp, ind)
        o = ora.encrypt(okeys, v, level, eseed)
        if s["kind"] == "rank":
            want.append([(ora.rank_tie(okeys, o, N, *cmp) if tie else ora.rank(okeys, o, N, *cmp)).export()])
        elif s["kind"] == "order":
            want.append([x.export() for x in ora.order_stat(okeys, o, N, s["k"], cmp, ind, tie)])
        elif s["kind"] == "sort":
            want.append([ora.sort(okeys, o, N, cmp, ind).export()])
        else:
            want.append([x.export() for x in ora.argmin(okeys, o, N, cmp, ind)])
        q = dict(kind=s["kind"], N=N, cmp=cmp, ind=ind, k=s.get("k", 1), tie=tie,
                 ct=ctx.encrypt(gkeys, v, level, eseed))
        queries.append(q)
    for rep in range(3):
        say(f"[gpu] mixed batch, call {rep}")
        outs = ctx.run_mixed(gkeys, queries)
        for i, (o, w) in enumerate(zip(outs, want)):
            got = [x.export() for x in (o if isinstance(o, tuple) else (o,))]
            assert len(got) == len(w) and all(np.array_equal(a, b) for a, b in zip(got, w)), (rep, i, specs[i])


@pytest.fixture(scope="module")
def p17o():
    import paper_2412_15126_amd as ckr
    say("[gpu] P17O context")
    ps = W.PSETS["P17O"]
    return ckr.Context(ps), ps


def test_argmax128_with_ties_matches_golden(p17o):
    ctx, ps = p17o
    gold = json.load(open(os.path.join(GOLD, "argmax128_p17o.json")))
    N = 128
    cmp, ind = W.ORDER_TIE_CMP[N]
    v, kseed, eseed = W.tied_workload(N, 0)
    say("[gpu] P17O argmax keygen")
    keys = ctx.keygen(kseed, ps["L"], [N], what=2)
    g = ctx.encrypt(keys, v, ps["L"], eseed)
    say("[gpu] P17O argmax")
    oh, val = ctx.order_stat(keys, g, N, N, cmp, ind, True)
    assert hashlib.sha256(oh.export().tobytes()).hexdigest() == gold["sha256_onehot"]
    assert hashlib.sha256(val.export().tobytes()).hexdigest() == gold["sha256_value"]
    top = int(np.flatnonzero(v == v.max())[-1])          # ties: the highest index among the maxima
    assert top == gold["argmax"]
    dec = ctx.decrypt(keys, oh, N)
    assert np.array_equal(np.round(dec), np.eye(N)[top])
    delta = VB.rank_error(v, cmp, True, 1 << 16)
    assert np.all(np.abs(dec - np.eye(N)[top]) <= VB.mask_bound(v, N, N, ind, delta) + VB.ETA)
    tol = VB.value_bound(v, N, N, ind, delta, VB.ETA)
    assert tol < 2.0 ** -11
    assert abs(ctx.decrypt(keys, val, 1)[0] - v.max()) <= tol


@pytest.mark.parametrize("N", [64, 128])
def test_multi_ciphertext_rank_bit_exact(ora, N):
    """Multi-ciphertext ranking (section 5) on blocks of 32 at n = 2^12 against
    the oracle, block for block."""
    import paper_2412_15126_amd as ckr
    ps = W.PSETS["T12D"]
    P = ora.Params(**ps)
    b = 32
    cmp = W.MULTI_RANK_CMP[N]
    level = ora.rank_multi_depth(*cmp) + 1
    seed = bytes(range(2, 34))
    okeys = ora.Keys(P, seed, level, P.circuit_galois(b, 4))
    ctx = ckr.Context(ps)
    gkeys = ctx.keygen(seed, level, [b], what=4)
    v, _, eseed = W.rank_workload(N, 2.0 ** -10, 700 + N)
    say(f"[gpu] multi-ciphertext rank N={N}")
    ob = [ora.encrypt(okeys, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    gb = [ctx.encrypt(gkeys, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    Ro = ora.rank_multi(okeys, ob, b, *cmp)
    Rg = ctx.rank_multi(gkeys, gb, b, cmp)
    assert len(Rg) == N // b
    for o, g in zip(Ro, Rg):
        assert np.array_equal(o.export(), g.export())
    got = np.concatenate([ctx.decrypt(gkeys, r, b) for r in Rg])
    assert np.array_equal(np.round(got), np.argsort(np.argsort(v)) + 1)


def test_multi_ciphertext_rank512_full_size_matches_golden():
    """N = 512 values in 4 blocks of 128 at n = 2^16 against oracle digests."""
    import paper_2412_15126_amd as ckr
    gold = json.load(open(os.path.join(GOLD, "rank512_p16_multi.json")))
    ps = W.PSETS["P16"]
    N, b = 512, 128
    cmp = W.MULTI_RANK_CMP[N]
    level = ckr.rank_multi_depth(cmp)
    assert level == gold["level"]
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    ctx = ckr.Context(ps)
    say("[gpu] P16 multi-ciphertext keys")
    keys = ctx.keygen(kseed, level, [b], what=4)
    blocks = [ctx.encrypt(keys, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    say("[gpu] P16 multi-ciphertext rank of 512")
    R = ctx.rank_multi(keys, blocks, b, cmp)
    assert [hashlib.sha256(r.export().tobytes()).hexdigest() for r in R] == gold["sha256"]
    got = np.concatenate([ctx.decrypt(keys, r, b) for r in R])
    assert np.array_equal(np.round(got), np.argsort(np.argsort(v)) + 1)


def test_multi_ciphertext_sort_bit_exact(ora):
    """Multi-ciphertext sorting (section 5) of 64 values in 2 blocks of 32 at
    n = 2^12 against the oracle, block for block."""
    import paper_2412_15126_amd as ckr
    ps = W.PSETS["T12E"]
    P = ora.Params(**ps)
    N, b = 64, 32
    cmp, ind = W.MULTI_SORT_CMP[N]
    level = ora.sort_multi_depth(cmp, ind)
    seed = bytes(range(4, 36))
    okeys = ora.Keys(P, seed, level, P.circuit_galois(b, 4))
    ctx = ckr.Context(ps)
    gkeys = ctx.keygen(seed, level, [b], what=4)
    assert ckr.sort_multi_depth(cmp, ind) == level
    v, _, eseed = W.rank_workload(N, 0.01, 950)
    say("[gpu] multi-ciphertext sort of 64")
    ob = [ora.encrypt(okeys, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    gb = [ctx.encrypt(gkeys, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    So = ora.sort_multi(okeys, ob, b, cmp, ind)
    Sg = ctx.sort_multi(gkeys, gb, b, cmp, ind)
    for o, g in zip(So, Sg):
        assert np.array_equal(o.export(), g.export())
    got = np.concatenate([ctx.decrypt(gkeys, s, b) for s in Sg])
    assert np.max(np.abs(got - np.sort(v))) <= VB.sort_tolerance(v, cmp, ind)



@pytest.mark.parametrize("N,cmp", [(2, (2, 1)), (32, (3, 1))])
def test_rank_smallest_and_largest_N_bit_exact(ora, N, cmp):
    """N = 2 (one rotation per re-encoding) and N = 32 (the largest power of two
    whose N x N matrix fits the 2048 slots of n = 2^12) against the oracle."""
    import paper_2412_15126_amd as ckr
    ps = W.PSETS["T12D"]
    P = ora.Params(**ps)
    level = ora.rank_depth(*cmp)
    seed = bytes(range(7, 39))
    okeys = ora.Keys(P, seed, level, P.rank_galois(N))
    ctx = ckr.Context(ps)
    gkeys = ctx.keygen(seed, level, [N])
    v, _, eseed = W.rank_workload(N, 0.01, 31 + N)
    say(f"[gpu] rank of {N}")
    ro = ora.rank(okeys, ora.encrypt(okeys, v, level, eseed), N, *cmp)
    rg = ctx.rank(gkeys, ctx.encrypt(gkeys, v, level, eseed), N, cmp)
    assert np.array_equal(ro.export(), rg.export())
    assert np.array_equal(np.round(ctx.decrypt(gkeys, rg, N)), np.argsort(np.argsort(v)) + 1)


def test_circuit_argument_errors(small):
    """Range, argument and level errors come back as status codes, with no
    output and no kernel launched on bad input."""
    ckr, ctx, keys, P = small["ckr"], small["ctx"], small["gkeys"], small["P"]
    g = ctx.encrypt(keys, np.linspace(0.1, 0.9, 8), P.L, bytes([9] * 32))
    h = ctx.encrypt(keys, np.linspace(0.1, 0.9, 8), P.L - 1, bytes([9] * 32))
    cases = [
        (lambda: ctx.rank(keys, g, 64, (3, 1)), -2),                       # 64^2 > 2048 slots
        (lambda: ctx.order_stat(keys, g, 8, 0, (3, 1), (2, 2), False), -1),  # k outside [1, N]
        (lambda: ctx.order_stat(keys, g, 8, 9, (3, 1), (2, 2), False), -1),
        (lambda: ctx.order_stat(keys, g, 8, 1, (0, 0), (2, 2), False), -1),  # empty comparator
        (lambda: ctx.rank_multi(keys, [g, h], 8, (3, 1)), -1),             # blocks of two levels
        (lambda: ctx.sort_multi(keys, [g, h], 8, (3, 1), (3, 2)), -1),
        (lambda: ctx.run_mixed(keys, [dict(kind="order", N=8, k=12, cmp=(3, 1), ind=(2, 2), ct=g)]), -1),
    ]
    for i, (call, status) in enumerate(cases):
        with pytest.raises(ckr.CkrError) as e:
            call()
        assert e.value.status == status, i




def test_multi_ciphertext_sort512_full_size_matches_golden():
    """N = 512 values in 2 blocks of 256 at n = 2^17 against oracle digests."""
    import paper_2412_15126_amd as ckr
    gold = json.load(open(os.path.join(GOLD, "sort512_p17s_multi.json")))
    ps = W.PSETS["P17S"]
    N, b = 512, 256
    cmp, ind = W.MULTI_SORT_CMP[N]
    level = ckr.sort_multi_depth(cmp, ind)
    assert level == gold["level"]
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    ctx = ckr.Context(ps)
    say("[gpu] P17S multi-ciphertext keys")
    keys = ctx.keygen(kseed, level, [b], what=4)
    blocks = [ctx.encrypt(keys, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    say("[gpu] P17S multi-ciphertext sort of 512")
    S = ctx.sort_multi(keys, blocks, b, cmp, ind)
    assert [hashlib.sha256(s.export().tobytes()).hexdigest() for s in S] == gold["sha256"]
    got = np.concatenate([ctx.decrypt(keys, s, b) for s in S])
    assert np.max(np.abs(got - np.sort(v))) <= VB.sort_tolerance(v, cmp, ind)


@pytest.fixture(scope="module")
def t12e(ora):
    import paper_2412_15126_amd as ckr
    ps = W.PSETS["T12E"]
    P = ora.Params(**ps)
    seed = bytes(range(1, 33))
    say("[gpu] T12E keys")
    okeys = ora.Keys(P, seed, P.L, P.circuit_galois(8, 2))
    ctx = ckr.Context(ps)
    return dict(P=P, okeys=okeys, ctx=ctx, gkeys=ctx.keygen(seed, P.L, [8], what=2), ckr=ckr)


def _tripled(N, seed):
    v, _, eseed = W.tripled_workload(N, seed, triples=1, gap=0.01)
    u, c = np.unique(v, return_counts=True)
    t = u[np.argmax(c)]
    return v, eseed, t, int(np.sum(v < t))


def test_order_stat_division_bit_exact(ora, t12e):
    """Section 3.2's value by division: a mask with three ones (the tripled
    value's rank), an empty one (no element of that rank) and a batch of
    three inputs, against the oracle bit for bit."""
    P, ctx = t12e["P"], t12e["ctx"]
    N, d = 8, 6
    cmp, ind = W.ORDER_CMP[N]
    v, eseed, t, below = _tripled(N, 5)
    for k, want in ((below + 2, t), (below + 1, 0.0)):
        level = ora.order_stat_div_depth(N, k, cmp, ind, d)
        assert level == t12e["ckr"].order_stat_div_depth(N, k, cmp, ind, d)
        say(f"[gpu] order statistic with division k={k}")
        ooh, oval = ora.order_stat_div(t12e["okeys"], ora.encrypt(t12e["okeys"], v, level, eseed), N, k, cmp, ind, d)
        (goh, gval), = ctx.order_stat_div(t12e["gkeys"], [ctx.encrypt(t12e["gkeys"], v, level, eseed)], N, k, cmp,
                                          ind, d)
        assert np.array_equal(ooh.export(), goh.export()) and np.array_equal(oval.export(), gval.export())
        assert abs(ctx.decrypt(t12e["gkeys"], gval, 1)[0] - want) <= VB.division_bound(v, k, cmp, ind, d)
    k = below + 2
    level = ora.order_stat_div_depth(N, k, cmp, ind, d)
    cts = [ctx.encrypt(t12e["gkeys"], v, level, bytes([i]) + eseed[1:]) for i in range(3)]
    singles = [ctx.order_stat_div(t12e["gkeys"], [c], N, k, cmp, ind, d)[0] for c in cts]
    batch = ctx.order_stat_div(t12e["gkeys"], cts, N, k, cmp, ind, d)
    for (a, b), (c, e) in zip(batch, singles):
        assert np.array_equal(a.export(), c.export()) and np.array_equal(b.export(), e.export())


def test_order_stat_division_rejects_bad_iterations(t12e):
    ctx, ckr = t12e["ctx"], t12e["ckr"]
    ct = ctx.encrypt(t12e["gkeys"], np.zeros(8), 10, bytes(32))
    for iters in (0, 1, 25):
        with pytest.raises(ckr.CkrError) as e:
            ctx.order_stat_div(t12e["gkeys"], [ct], 8, 2, W.ORDER_CMP[8][0], W.ORDER_CMP[8][1], iters)
        assert e.value.status == -1


@pytest.mark.parametrize("N,tie", [(5, False), (7, False), (6, True)])
def test_padded_rank_bit_exact(ora, small, N, tie):
    """Rank of N values that are not a power of two (section 3.1): zero-padded,
    comparison matrix masked to its N x N block; single, batched and replayed
    against the oracle."""
    P, ctx = small["P"], small["ctx"]
    cmp = W.ORDER_TIE_CMP[8][0] if tie else W.RANK_CMP[8]
    level = ora.rank_depth_n(N, cmp, tie)
    assert level == small["ckr"].rank_depth_n(N, cmp, tie)
    qs = [(W.tied_workload(N, 30 + i, 0.01) if tie else W.rank_workload(N, 0.01, 30 + i)) for i in range(3)]
    say(f"[gpu] padded rank N={N} tie={tie}")
    for v, _, eseed in qs[:1]:
        o = ora.encrypt(small["okeys"], v, level, eseed)
        ro = ora.rank_tie(small["okeys"], o, N, *cmp) if tie else ora.rank(small["okeys"], o, N, *cmp)
        rg = ctx.rank(small["gkeys"], ctx.encrypt(small["gkeys"], v, level, eseed), N, cmp, tie=tie)
        assert np.array_equal(ro.export(), rg.export())
        want = np.empty(N)
        want[np.argsort(v, kind="stable")] = np.arange(1, N + 1)
        if not tie:
            want = np.argsort(np.argsort(v)) + 1
        assert np.array_equal(np.round(ctx.decrypt(small["gkeys"], rg, N)), want)
    if not tie:
        cts = [ctx.encrypt(small["gkeys"], v, level, e) for v, _, e in qs]
        singles = [ctx.rank(small["gkeys"], c, N, cmp).export() for c in cts]
        for rep in range(3):
            outs = ctx.run_batch(small["gkeys"], "rank", cts, N, cmp)
            assert all(np.array_equal(a.export(), b) for a, b in zip(outs, singles))


def _window_mask(v, a, b):
    m = np.zeros(len(v))
    m[np.argsort(v, kind="stable")[a - 1:b]] = 1.0
    return m


@pytest.mark.parametrize("N,a,b,tie", [(8, 4, 5, True), (8, 4, 5, False), (8, 1, 3, True), (8, 6, 8, False),
                                       (8, 2, 7, True), (6, 3, 4, True), (7, 4, 4, True), (5, 1, 2, True),
                                       (7, 5, 7, True)])
def test_order_range_bit_exact(ora, small, N, a, b, tie):
    """Order statistics over a rank window (the median of section 4, lower,
    upper and inner windows, padded N) against the oracle bit for bit."""
    P, ctx = small["P"], small["ctx"]
    cmp, ind = W.ORDER_TIE_CMP[8] if tie else W.ORDER_CMP[8]
    v, _, eseed = W.tied_workload(N, 20 + N, 0.01) if tie else W.rank_workload(N, 0.01, 20 + N)
    level = ora.order_range_depth(N, a, b, cmp, ind, tie)
    assert level == small["ckr"].order_range_depth(N, a, b, cmp, ind, tie)
    say(f"[gpu] order range N={N} [{a}, {b}] tie={tie}")
    ooh, oval = ora.order_range(small["okeys"], ora.encrypt(small["okeys"], v, level, eseed), N, a, b, cmp, ind, tie)
    (goh, gval), = ctx.order_range(small["gkeys"], [ctx.encrypt(small["gkeys"], v, level, eseed)], N, a, b, cmp,
                                   ind, tie)
    assert np.array_equal(ooh.export(), goh.export()) and np.array_equal(oval.export(), gval.export())
    assert np.array_equal(np.round(ctx.decrypt(small["gkeys"], goh, N)), _window_mask(v, a, b))
    assert abs(ctx.decrypt(small["gkeys"], gval, 1)[0] - np.mean(np.sort(v)[a - 1:b])) <= VB.tolerance(
        v, a, b, cmp, ind, tie, 12)


@pytest.mark.parametrize("N", [8, 7])
def test_median_batch_and_replays_equal_single(ora, small, N):
    """A batch of three medians (eager, captured, replayed) equals three single
    calls bit for bit; the window a = b = k equals the order statistic."""
    P, ctx, ckr = small["P"], small["ctx"], small["ckr"]
    cmp, ind = W.ORDER_TIE_CMP[8]
    a, b = ckr.median_window(N)
    level = ckr.order_range_depth(N, a, b, cmp, ind, True)
    qs = [W.tied_workload(N, 60 + i, 0.01) for i in range(3)]
    cts = [ctx.encrypt(small["gkeys"], v, level, e) for v, _, e in qs]
    say(f"[gpu] median batch N={N}")
    singles = [ctx.median(small["gkeys"], [c], N, cmp, ind)[0] for c in cts]
    for rep in range(3):
        outs = ctx.median(small["gkeys"], cts, N, cmp, ind)
        for (x, y), (s, t) in zip(outs, singles):
            assert np.array_equal(x.export(), s.export()) and np.array_equal(y.export(), t.export()), rep
    for (v, _, _), (_, val) in zip(qs, singles):
        assert abs(ctx.decrypt(small["gkeys"], val, 1)[0] - np.median(v)) <= VB.tolerance(v, a, b, cmp, ind, True,
                                                                                            12)
    if N == 8:
        k = 5
        lk = ckr.order_stat_depth(N, k, cmp, ind, True)
        c = ctx.encrypt(small["gkeys"], qs[0][0], lk, qs[0][2])
        (r_oh, r_val), = ctx.order_range(small["gkeys"], [c], N, k, k, cmp, ind, True)
        s_oh, s_val = ctx.order_stat(small["gkeys"], c, N, k, cmp, ind, True)
        assert np.array_equal(r_oh.export(), s_oh.export()) and np.array_equal(r_val.export(), s_val.export())


def test_order_range_errors(small):
    ctx, ckr = small["ctx"], small["ckr"]
    cmp, ind = W.ORDER_TIE_CMP[8]
    ct = ctx.encrypt(small["gkeys"], np.linspace(0.1, 0.8, 8), small["P"].L, bytes(32))
    for N, a, b, tie, st in ((8, 1, 8, True, -1), (8, 0, 2, True, -1), (8, 3, 2, True, -1), (8, 2, 9, True, -1),
                             (6, 2, 3, False, -1), (1, 1, 1, True, -2), (64, 2, 3, True, -2)):
        with pytest.raises(ckr.CkrError) as e:
            ctx.order_range(small["gkeys"], [ct], N, a, b, cmp, ind, tie)
        assert e.value.status == st, (N, a, b, tie)
    low = ctx.encrypt(small["gkeys"], np.linspace(0.1, 0.8, 8), 3, bytes(32))
    with pytest.raises(ckr.CkrError) as e:
        ctx.order_range(small["gkeys"], [low], 8, 4, 5, cmp, ind, True)
    assert e.value.status == -3


def test_median128_with_ties_matches_golden(p17o):
    """Tie-corrected median of N = 128 at n = 2^17 (window [64, 65]) against
    the oracle's digests."""
    ctx, ps = p17o
    gold = json.load(open(os.path.join(GOLD, "median128_p17o.json")))
    N = 128
    cmp, ind = W.ORDER_TIE_CMP[N]
    v, kseed, eseed = W.tied_workload(N, 3)
    assert gold["level"] == 44 and gold["window"] == [64, 65]
    say("[gpu] P17O median keygen")
    keys = ctx.keygen(kseed, gold["level"], [N], what=2)
    (oh, val), = ctx.median(keys, [ctx.encrypt(keys, v, gold["level"], eseed)], N, cmp, ind)
    say("[gpu] P17O median done")
    assert hashlib.sha256(oh.export().tobytes()).hexdigest() == gold["sha256"][0]
    assert hashlib.sha256(val.export().tobytes()).hexdigest() == gold["sha256"][1]
    assert np.array_equal(np.round(ctx.decrypt(keys, oh, N)), _window_mask(v, 64, 65))
    tol = VB.tolerance(v, 64, 65, cmp, ind, True, 17)
    assert tol < 2.0 ** -11
    assert abs(ctx.decrypt(keys, val, 1)[0] - np.median(v)) <= tol


def test_median101_padded_full_size_matches_golden():
    """Tie-corrected median of N = 101 values (rank 51) zero-padded to the 128
    layout at n = 2^17 against the oracle's digests."""
    import paper_2412_15126_amd as ckr
    gold = json.load(open(os.path.join(GOLD, "median101_p17s.json")))
    N = 101
    cmp, ind = W.ORDER_TIE_CMP[128]
    assert ckr.median_window(N) == tuple(gold["window"]) == (51, 51)
    level = ckr.order_range_depth(N, 51, 51, cmp, ind, True)
    assert level == gold["level"]
    v, kseed, eseed = W.tied_workload(N, 4)
    ctx = ckr.Context(W.PSETS["P17S"])
    say("[gpu] P17S padded median keygen")
    keys = ctx.keygen(kseed, level, [N], what=2)
    (oh, val), = ctx.median(keys, [ctx.encrypt(keys, v, level, eseed)], N, cmp, ind)
    say("[gpu] P17S padded median done")
    assert hashlib.sha256(oh.export().tobytes()).hexdigest() == gold["sha256"][0]
    assert hashlib.sha256(val.export().tobytes()).hexdigest() == gold["sha256"][1]
    assert np.array_equal(np.round(ctx.decrypt(keys, oh, N)), _window_mask(v, 51, 51))
    tol = VB.tolerance(v, 51, 51, cmp, ind, True, 17)
    assert tol < 2.0 ** -11
    assert abs(ctx.decrypt(keys, val, 1)[0] - np.median(v)) <= tol


def test_multi_ciphertext_rank2048_full_size_matches_golden():
    """N = 2048 values (gap 2^-12) in 16 blocks of 128 at n = 2^16 (136 block
    pairs in batched comparator passes of 32) against oracle digests; every
    rank exact; the device high-water mark is reported."""
    import paper_2412_15126_amd as ckr
    gold = json.load(open(os.path.join(GOLD, "rank2048_p16d_multi.json")))
    ps = W.PSETS["P16D"]
    N, b = 2048, 128
    cmp = W.MULTI_RANK_CMP[N]
    level = ckr.rank_multi_depth(cmp)
    assert level == gold["level"] == 24
    v, kseed, eseed = W.rank_workload(N, W.MULTI_GAP[N], 0)
    ctx = ckr.Context(ps)
    say("[gpu] P16D multi-ciphertext keys")
    keys = ctx.keygen(kseed, level, [b], what=4)
    blocks = [ctx.encrypt(keys, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    say("[gpu] P16D multi-ciphertext rank of 2048")
    R = ctx.rank_multi(keys, blocks, b, cmp)
    assert [hashlib.sha256(r.export().tobytes()).hexdigest() for r in R] == gold["sha256"]
    got = np.concatenate([ctx.decrypt(keys, r, b) for r in R])
    assert np.array_equal(np.round(got), np.argsort(np.argsort(v)) + 1)
    say(f"[gpu] rank-2048: max error {np.max(np.abs(got - (np.argsort(np.argsort(v)) + 1))):.3f}, "
        f"device high-water {ctx.memory()[1] / 2 ** 30:.1f} GiB")


def test_multi_ciphertext_sort1024_full_size_matches_golden():
    """N = 1024 values (gap 2^-11) in 4 blocks of 256 at n = 2^17 against
    oracle digests (the L^2 indicators in batched passes of 32)."""
    import paper_2412_15126_amd as ckr
    gold = json.load(open(os.path.join(GOLD, "sort1024_p17s_multi.json")))
    ps = W.PSETS["P17S"]
    N, b = 1024, 256
    cmp, ind = W.MULTI_SORT_CMP[N]
    level = ckr.sort_multi_depth(cmp, ind)
    assert level == gold["level"] == 47
    v, kseed, eseed = W.rank_workload(N, W.MULTI_GAP[N], 0)
    ctx = ckr.Context(ps)
    say("[gpu] P17S multi-ciphertext keys (1024)")
    keys = ctx.keygen(kseed, level, [b], what=4)
    blocks = [ctx.encrypt(keys, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    say("[gpu] P17S multi-ciphertext sort of 1024")
    S = ctx.sort_multi(keys, blocks, b, cmp, ind)
    assert [hashlib.sha256(s.export().tobytes()).hexdigest() for s in S] == gold["sha256"]
    got = np.concatenate([ctx.decrypt(keys, s, b) for s in S])
    assert np.max(np.abs(got - np.sort(v))) <= VB.sort_tolerance(v, cmp, ind)
