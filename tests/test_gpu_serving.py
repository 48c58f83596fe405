"""Serving: continuous batching over two rings (rank at n = 2^12; argmin and
sort at a deep n = 2^12 ring), requests arriving while batches run.  Every
result must equal the same query run alone, bit for bit; the HBM budget must
reject a request whose working set does not fit."""
import sys
import time

import numpy as np
import pytest

from paper_2412_15126_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rings():
    import paper_2412_15126_amd as ckr
    say("[gpu] serving rings")
    p12, t12d = W.PSETS["P12"], W.PSETS["T12D"]
    a = ckr.Context(p12)
    ka = a.keygen(bytes(range(32)), p12["L"], [8])
    b = ckr.Context(t12d)
    kb = b.keygen(bytes(range(1, 33)), t12d["L"], [8], what=6)
    return ckr, (a, ka, p12), (b, kb, t12d)


def _queries(rings):
    ckr, (a, ka, p12), (b, kb, t12d) = rings
    qs = []
    for s in range(10):
        v, _, e = W.rank_workload(8, 0.01, 300 + s)
        qs.append(("rank", a, ka, a.encrypt(ka, v, p12["L"], e), W.RANK_CMP[8], (0, 0)))
    for s in range(5):
        v, _, e = W.tied_workload(8, 400 + s, 0.01)
        qs.append(("argmin", b, kb, b.encrypt(kb, v, t12d["L"], e), *W.ARGMIN_CMP[8]))
    for s in range(5):
        v, _, e = W.rank_workload(8, 0.01, 500 + s)
        qs.append(("sort", b, kb, b.encrypt(kb, v, t12d["L"], e), *W.SORT_CMP[8]))
    order = np.random.default_rng(7).permutation(len(qs))
    return [qs[i] for i in order]


def _alone(q):
    kind, ctx, keys, ct, cmp, ind = q
    if kind == "rank":
        return [ctx.rank(keys, ct, 8, cmp).export()]
    if kind == "argmin":
        return [x.export() for x in ctx.argmin(keys, ct, 8, cmp, ind)]
    return [ctx.sort(keys, ct, 8, cmp, ind).export()]


def test_served_results_equal_alone(rings):
    ckr = rings[0]
    qs = _queries(rings)
    alone = [_alone(q) for q in qs]
    srv = ckr.Server(hbm_budget=0, max_batch=4)
    (a, ka, _), (b, kb, _) = rings[1], rings[2]
    srv.add_route("rank", 8, a, ka, W.RANK_CMP[8])
    srv.add_route("argmin", 8, b, kb, *W.ARGMIN_CMP[8])
    srv.add_route("sort", 8, b, kb, *W.SORT_CMP[8])
    rng = np.random.default_rng(3)
    tickets = []
    say("[gpu] serving: submitting")
    for q in qs:
        tickets.append(srv.submit(q[0], 8, q[3]))
        time.sleep(float(rng.exponential(0.002)))
    lats, batches = [], []
    for t, want in zip(tickets, alone):
        outs, (lat, queue, batch) = srv.wait(t, 60000)
        assert len(outs) == len(want)
        for o, w in zip(outs, want):
            assert np.array_equal(o.export(), w)
        lats.append(lat)
        batches.append(batch)
    st = srv.stats()
    say(f"[gpu] served {st}; p50 {np.percentile(lats, 50):.2f} ms p99 {np.percentile(lats, 99):.2f} ms")
    assert st["completed"] == len(qs)
    assert st["batches"] < len(qs) and max(batches) > 1     # requests were batched
    assert min(lats) > 0
    srv.close()


def test_budget_rejects_oversized_request(rings):
    ckr = rings[0]
    a, ka, p12 = rings[1]
    srv = ckr.Server(hbm_budget=1 << 20, max_batch=4)      # 1 MiB: less than one query's working set
    srv.add_route("rank", 8, a, ka, W.RANK_CMP[8])
    v, _, e = W.rank_workload(8, 0.01, 900)
    ct = a.encrypt(ka, v, p12["L"], e)
    # the first batch of a route runs alone and measures its working set
    outs, _ = srv.wait(srv.submit("rank", 8, ct), 60000)
    assert np.array_equal(outs[0].export(), a.rank(ka, ct, 8, W.RANK_CMP[8]).export())
    with pytest.raises(ckr.CkrError) as e:
        srv.wait(srv.submit("rank", 8, ct), 60000)
    assert e.value.status == -4
    srv.close()
