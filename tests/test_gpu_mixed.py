"""Batched execution of many independent queries at n = 2^16: 64 rank and
argmin queries (N drawn from {16, 32, 64, 128}, values min-gap uniform,
seed 7), each encrypted at the level its own circuit needs, run as one
graph-captured launch.  Every result must equal the query run alone, bit for
bit; ranks must be exact and every one-hot must mark the minimum; two of the
queries must match digests written by tests/golden/make_golden.py (oracle
only)."""
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


def mixed_queries(ckr, ctx, keys, qs):
    out = []
    for q in qs:
        N = q["N"]
        if q["kind"] == "rank":
            cmp, ind = W.RANK_CMP[N], (0, 0)
            d = dict(kind="rank", level=ckr.rank_depth(cmp))
        else:
            cmp, ind = W.ORDER_CMP[N]
            d = dict(kind="order", k=1, tie=False, level=ckr.order_stat_depth(N, 1, cmp, ind, False))
        d.update(N=N, cmp=cmp, ind=ind, v=q["v"], ct=ctx.encrypt(keys, q["v"], d["level"], q["eseed"]))
        out.append(d)
    return out


@pytest.fixture(scope="module")
def mix():
    import paper_2412_15126_amd as ckr
    ps = W.PSETS["P16D"]
    ctx = ckr.Context(ps)
    kseed, qs = W.mixed_workload(7, 64)
    say("[gpu] P16D keys for N in {16, 32, 64, 128}")
    keys = ctx.keygen(kseed, ps["L"], [16, 32, 64, 128], what=2)
    return ctx, keys, mixed_queries(ckr, ctx, keys, qs)


def _single(ctx, keys, q):
    if q["kind"] == "rank":
        return (ctx.rank(keys, q["ct"], q["N"], q["cmp"]),)
    return ctx.order_stat(keys, q["ct"], q["N"], 1, q["cmp"], q["ind"], False)


def test_mixed64_one_launch_equals_single_queries(mix):
    ctx, keys, qs = mix
    assert len({(q["kind"], q["N"]) for q in qs}) == 8 and len({q["level"] for q in qs}) >= 4
    say("[gpu] 64 single queries")
    singles = [[x.export() for x in _single(ctx, keys, q)] for q in qs]
    for rep in range(3):   # eager, captured, replayed
        say(f"[gpu] mixed batch of 64, call {rep}")
        outs = ctx.run_mixed(keys, qs)
        for i, (o, s) in enumerate(zip(outs, singles)):
            got = [x.export() for x in (o if isinstance(o, tuple) else (o,))]
            assert all(np.array_equal(a, b) for a, b in zip(got, s)), (rep, i)
    for q, o in zip(qs, outs):
        N, v = q["N"], q["v"]
        if q["kind"] == "rank":
            assert np.array_equal(np.round(ctx.decrypt(keys, o, N)), np.argsort(np.argsort(v)) + 1)
        else:
            assert np.array_equal(np.round(ctx.decrypt(keys, o[0], N)), np.eye(N)[int(np.argmin(v))])
            assert abs(ctx.decrypt(keys, o[1], 1)[0] - v.min()) <= VB.tolerance(v, 1, 1, q["cmp"], q["ind"], False, 16)


def test_mixed64_matches_oracle_digests(mix):
    ctx, keys, qs = mix
    gold = json.load(open(os.path.join(GOLD, "mixed_p16d.json")))
    outs = ctx.run_mixed(keys, qs)
    r = outs[gold["rank_index"]]
    assert qs[gold["rank_index"]]["level"] == gold["rank_level"]
    assert hashlib.sha256(r.export().tobytes()).hexdigest() == gold["rank_sha256"]
    oh, val = outs[gold["argmin_index"]]
    assert qs[gold["argmin_index"]]["level"] == gold["argmin_level"]
    assert hashlib.sha256(oh.export().tobytes()).hexdigest() == gold["argmin_sha256_onehot"]
    assert hashlib.sha256(val.export().tobytes()).hexdigest() == gold["argmin_sha256_value"]
