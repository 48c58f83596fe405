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
    assert st["overlap_high"] >= 2                           # batches of one context overlapped
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


def test_served_mix_full_size_matches_oracle_digests():
    """The served configuration at full size: rank-128 at n = 2^16 and sort /
    argmin at n = 2^17 arriving interleaved (Poisson gaps) through the server,
    batched as they come.  The rank-128 and sort-128 queries of the stored
    oracle digests (tests/golden/rank128_p16.json, sort128_p17.json: workload
    seed 0, the same key seed) must reproduce those digests in the mix; every
    other request must equal the same query run alone, bit for bit."""
    import hashlib
    import json
    import os
    import paper_2412_15126_amd as ckr
    gold_dir = os.path.join(os.path.dirname(__file__), "golden")
    g_rank = json.load(open(os.path.join(gold_dir, "rank128_p16.json")))
    g_sort = json.load(open(os.path.join(gold_dir, "sort128_p17.json")))
    p16, p17 = W.PSETS["P16"], W.PSETS["P17"]
    v0, kseed, e0 = W.rank_workload(128, 2.0 ** -10, 0)
    say("[gpu] served full size: keys")
    a = ckr.Context(p16)
    ka = a.keygen(kseed, 17, [128])
    b = ckr.Context(p17)
    kb = b.keygen(kseed, p17["L"], [64, 128], what=6)
    jobs = [("rank", 128, a, ka, a.encrypt(ka, v0, 17, e0), "gold"),
            ("sort", 128, b, kb, b.encrypt(kb, v0, p17["L"], e0), "gold")]
    for s in range(4):
        v, _, e = W.rank_workload(128, 2.0 ** -10, 700 + s)
        jobs.append(("rank", 128, a, ka, a.encrypt(ka, v, 17, e), None))
    for s in range(2):
        v, _, e = W.tied_workload(64, 710 + s)
        jobs.append(("argmin", 64, b, kb, b.encrypt(kb, v, p17["L"], e), None))
        v, _, e = W.rank_workload(64, 2.0 ** -10, 720 + s)
        jobs.append(("sort", 64, b, kb, b.encrypt(kb, v, p17["L"], e), None))
    order = np.random.default_rng(5).permutation(len(jobs))
    jobs = [jobs[i] for i in order]
    srv = ckr.Server(hbm_budget=64 << 30, max_batch=4)
    srv.add_route("rank", 128, a, ka, W.RANK_CMP[128])
    srv.add_route("argmin", 64, b, kb, *W.ARGMIN_CMP[64])
    srv.add_route("sort", 64, b, kb, *W.SORT_CMP[64])
    srv.add_route("sort", 128, b, kb, *W.SORT_CMP[128])
    rng = np.random.default_rng(9)
    say("[gpu] served full size: submitting")
    tickets = []
    for j in jobs:
        tickets.append(srv.submit(j[0], j[1], j[4]))
        time.sleep(float(rng.exponential(0.05)))
    outs = []
    for t in tickets:
        o, _ = srv.wait(t, 300000)
        outs.append(o)
    say(f"[gpu] served full size: {srv.stats()}")
    srv.close()
    for (kind, N, ctx, keys, ct, tag), o in zip(jobs, outs):
        if tag == "gold":
            want = g_rank["sha256"] if kind == "rank" else g_sort["sha256"]
            assert hashlib.sha256(o[0].export().tobytes()).hexdigest() == want, kind
            continue
        if kind == "rank":
            alone = [ctx.rank(keys, ct, N, W.RANK_CMP[N])]
        elif kind == "argmin":
            alone = list(ctx.argmin(keys, ct, N, *W.ARGMIN_CMP[N]))
        else:
            alone = [ctx.sort(keys, ct, N, *W.SORT_CMP[N])]
        assert all(np.array_equal(x.export(), y.export()) for x, y in zip(alone, o)), kind
