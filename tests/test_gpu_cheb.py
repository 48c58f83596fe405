"""GPU parity of the Chebyshev comparator (section 2.2): the batched
Paterson-Stockmeyer evaluation, rank, order statistics and sorting with it,
element by element against the oracle on the same seeded inputs."""
import sys

import numpy as np
import pytest

from paper_2412_15126_amd import workloads as W

import value_bound as VB


pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ckr():
    import paper_2412_15126_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def t10(ora, ckr):
    ps = W.PSETS["T10"]
    P = ora.Params(**ps)
    seed = bytes(range(5, 37))
    say("[gpu] T10 relinearisation keys")
    ctx = ckr.Context(ps)
    return dict(P=P, okeys=ora.Keys(P, seed, P.L, []), ctx=ctx, gkeys=ctx.keygen(seed, P.L, []))


@pytest.mark.parametrize("deg1", [2, 4, 8, 16, 32, 64])
def test_cheb_eval_bit_exact(ora, t10, deg1):
    """Every shape of the evaluation (no giant step; one; several; the
    largest baby-step set the ring's 7 levels allow) with random
    coefficients, a third of them exactly zero."""
    P, ctx = t10["P"], t10["ctx"]
    rng = np.random.default_rng(100 + deg1)
    c = rng.uniform(-1.0, 1.0, deg1)
    c[rng.random(deg1) < 0.3] = 0.0
    x = rng.uniform(-1.0, 1.0, 64)
    seed = bytes([deg1]) * 32
    say(f"[gpu] cheb_eval deg1={deg1}")
    o = ora.cheb_eval(t10["okeys"], ora.encrypt(t10["okeys"], x, P.L, seed), c)
    g = ctx.cheb_eval(t10["gkeys"], ctx.encrypt(t10["gkeys"], x, P.L, seed), c)
    assert np.array_equal(o.export(), g.export())
    from numpy.polynomial import chebyshev as Ch
    got = ctx.decrypt(t10["gkeys"], g, 64)
    assert np.max(np.abs(got - Ch.chebval(x, c))) < 1e-5 * np.sum(np.abs(c))


def test_cheb_eval_rejects_bad_lengths_and_depth(ckr, t10):
    ctx = t10["ctx"]
    ct = ctx.encrypt(t10["gkeys"], np.zeros(4), 2, bytes(32))
    with pytest.raises(ckr.CkrError) as e:
        ctx.cheb_eval(t10["gkeys"], ct, np.ones(6))
    assert e.value.status == -1
    with pytest.raises(ckr.CkrError) as e:
        ctx.cheb_eval(t10["gkeys"], ct, np.ones(8))      # needs 4 levels, has 2
    assert e.value.status == -3


@pytest.fixture(scope="module")
def small(ora, ckr):
    ps = W.PSETS["T12D"]
    P = ora.Params(**ps)
    seed = bytes(range(32))
    say("[gpu] T12D keys")
    okeys = ora.Keys(P, seed, P.L, P.circuit_galois(8, 6))
    ctx = ckr.Context(ps)
    return dict(P=P, okeys=okeys, ctx=ctx, gkeys=ctx.keygen(seed, P.L, [8], what=6), ckr=ckr)


@pytest.mark.parametrize("seed", [0, 1])
def test_rank8_chebyshev_bit_exact(ora, small, seed):
    P, ctx = small["P"], small["ctx"]
    N, cmp = 8, W.CHEB_CMP[8]
    v, _, eseed = W.rank_workload(N, 0.01, seed)
    level = ora.rank_depth(*cmp)
    say(f"[gpu] rank8 chebyshev seed {seed}")
    o = ora.rank(small["okeys"], ora.encrypt(small["okeys"], v, level, eseed), N, *cmp)
    g = ctx.rank(small["gkeys"], ctx.encrypt(small["gkeys"], v, level, eseed), N, cmp)
    assert np.array_equal(o.export(), g.export())
    assert np.array_equal(np.round(ctx.decrypt(small["gkeys"], g, N)), np.argsort(np.argsort(v)) + 1)


def test_rank8_chebyshev_batch_and_graph_equal_single(ora, small):
    """A batch of 3 (first call eager, then captured, then replayed) gives the
    single-query ciphertexts."""
    P, ctx = small["P"], small["ctx"]
    N, cmp = 8, W.CHEB_CMP[8]
    level = ora.rank_depth(*cmp)
    qs = [W.rank_workload(N, 0.01, 10 + i) for i in range(3)]
    cts = [ctx.encrypt(small["gkeys"], v, level, es) for v, _, es in qs]
    singles = [ctx.rank(small["gkeys"], c, N, cmp).export() for c in cts]
    for rep in range(3):
        say(f"[gpu] rank8 chebyshev batch replay {rep}")
        outs = ctx.run_batch(small["gkeys"], "rank", cts, N, cmp)
        for a, b in zip(outs, singles):
            assert np.array_equal(a.export(), b)


@pytest.mark.parametrize("k,tie", [(1, True), (3, False), (8, False)])
def test_order_statistic_chebyshev_bit_exact(ora, small, k, tie):
    P, ctx = small["P"], small["ctx"]
    N = 8
    cmp = ind = W.CHEB_CMP[N]
    v, _, eseed = (W.tied_workload(N, 3, 0.01) if tie else W.rank_workload(N, 0.01, 3))
    level = ora.order_stat_depth(N, k, cmp, ind, tie)
    assert level == small["ckr"].order_stat_depth(N, k, cmp, ind, tie)
    say(f"[gpu] order statistic chebyshev k={k} tie={tie}")
    ooh, oval = ora.order_stat(small["okeys"], ora.encrypt(small["okeys"], v, level, eseed), N, k, cmp, ind, tie)
    goh, gval = ctx.order_stat(small["gkeys"], ctx.encrypt(small["gkeys"], v, level, eseed), N, k, cmp, ind, tie)
    assert np.array_equal(ooh.export(), goh.export()) and np.array_equal(oval.export(), gval.export())
    j = np.argsort(v, kind="stable")[k - 1]
    assert np.array_equal(np.round(ctx.decrypt(small["gkeys"], goh, N)), np.eye(N)[j])


def test_sort8_chebyshev_rank_bit_exact(ora, small):
    """Sorting with the Chebyshev comparator in its rank and the f/g window
    indicator (the interpolant's oscillation near its jump leaves the window
    product 0.1 off at this degree; the paper sorts with f/g)."""
    P, ctx = small["P"], small["ctx"]
    N = 8
    cmp, ind = W.CHEB_CMP[N], W.SORT_CMP[N][1]
    v, _, eseed = W.rank_workload(N, 0.01, 5)
    level = ora.sort_depth(cmp, ind)
    say("[gpu] sort8 chebyshev")
    o = ora.sort(small["okeys"], ora.encrypt(small["okeys"], v, level, eseed), N, cmp, ind)
    g = ctx.sort(small["gkeys"], ctx.encrypt(small["gkeys"], v, level, eseed), N, cmp, ind)
    assert np.array_equal(o.export(), g.export())
    assert np.max(np.abs(ctx.decrypt(small["gkeys"], g, N) - np.sort(v))) <= VB.sort_tolerance(v, cmp, ind)
