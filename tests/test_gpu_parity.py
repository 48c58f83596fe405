"""GPU parity: the HIP path against the CPU oracle, ciphertext for ciphertext.

Every comparison is on exported coefficient-domain limbs (canonical uint64),
so the two sides must agree bit for bit.  Inputs come from the seeded
generators in paper_2412_15126_amd.workloads; nothing the oracle sees comes
from the HIP path.
"""
import sys

import numpy as np
import pytest

from paper_2412_15126_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ckr():
    import paper_2412_15126_amd as m
    m.lib()
    return m


class Pair:
    """Same parameter set, keys and seeds on both sides."""

    def __init__(self, ora, ckr, name, lmax, shifts=(), Ns=(), seed=bytes(range(32))):
        self.ps = W.PSETS[name] if isinstance(name, str) else name
        self.P = ora.Params(**self.ps)
        self.ctx = ckr.Context(self.ps)
        self.ora = ora
        self.n = self.P.n
        gal = set(self.P.galois_left(k % (self.n // 2)) for k in shifts)
        for N in Ns:
            gal |= set(self.P.rank_galois(N))
        self.okeys = ora.Keys(self.P, seed, lmax, sorted(gal))
        self.gkeys = self.ctx.keygen(seed, lmax, Ns)
        if shifts:
            self.gkeys.add_rotations(shifts)

    def enc(self, v, level, seed):
        return self.ora.encrypt(self.okeys, v, level, seed), self.ctx.encrypt(self.gkeys, v, level, seed)


def same(o, g, what=""):
    a, b = o.export(), g.export()
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if not np.array_equal(a, b):
        bad = np.argwhere(a != b)
        raise AssertionError(f"{what}: {len(bad)} words differ, first at {bad[0].tolist()}")


@pytest.fixture(scope="module")
def t10(ora, ckr):
    say("[gpu] T10 pair")
    return Pair(ora, ckr, "T10", W.PSETS["T10"]["L"], shifts=(1, 3, -1, -5, 200))


def test_context_moduli_match_oracle(t10):
    assert np.array_equal(t10.ctx.moduli, t10.P.mods)
    assert np.array_equal(t10.ctx.scales.view(np.uint64), t10.P.scales.view(np.uint64))


def test_raw_ntt_roundtrip_on_device(ckr, t10):
    from paper_2412_15126_amd import hip
    say("[gpu] raw ntt roundtrip")
    n, nm = t10.n, len(t10.P.mods)
    rng = np.random.default_rng(0)
    host = np.stack([rng.integers(0, int(q), n, dtype=np.uint64) for q in t10.P.mods])
    dev = hip.DeviceArray(host)
    t10.ctx.ntt_device(dev.ptr.value, nm, 0, False)
    hip.synchronize()
    fwd = dev.numpy()
    assert not np.array_equal(fwd, host)
    assert np.all(fwd < t10.P.mods[:, None])
    t10.ctx.ntt_device(dev.ptr.value, nm, 0, True)
    hip.synchronize()
    assert np.array_equal(dev.numpy(), host)


@pytest.mark.parametrize("level", [0, 3, 7])
def test_encrypt_bit_exact(t10, level):
    v = np.random.default_rng(level).uniform(0, 1, 40)
    o, g = t10.enc(v, level, bytes([level + 1] * 32))
    same(o, g, "encrypt")
    assert np.max(np.abs(t10.ctx.decrypt(t10.gkeys, g, 40) - v)) < 1e-6


def test_import_export_roundtrip_and_range_check(ckr, t10):
    o, g = t10.enc(np.linspace(0, 1, 16), 4, bytes([9] * 32))
    arr = o.export()
    back = t10.ctx.import_ct(arr)
    assert np.array_equal(back.export(), arr)
    bad = arr.copy()
    bad[1, 2, 5] = t10.P.mods[2]
    with pytest.raises(ckr.CkrError) as e:
        t10.ctx.import_ct(bad)
    assert e.value.status == -1


@pytest.mark.parametrize("k", [1, 3, -1, -5, 200])
def test_rotate_bit_exact(t10, k):
    v = np.random.default_rng(abs(k)).uniform(0, 1, t10.n // 2)
    for level in (7, 2):
        o, g = t10.enc(v, level, bytes([k & 0xFF] * 32))
        same(t10.ora.rotate(t10.okeys, o, k), t10.ctx.rotate(t10.gkeys, g, k), f"rotate {k} at {level}")


def test_mul_rescale_cmul_const_plain_bit_exact(t10):
    ora, ctx = t10.ora, t10.ctx
    rng = np.random.default_rng(7)
    v1, v2 = rng.uniform(-1, 1, 300), rng.uniform(-1, 1, 300)
    for level in (7, 4, 1):
        (o1, g1), (o2, g2) = t10.enc(v1, level, bytes([1] * 32)), t10.enc(v2, level, bytes([2] * 32))
        same(ora.mul(t10.okeys, o1, o2), ctx.mul(t10.gkeys, g1, g2), f"mul at {level}")
        same(ora.mul(t10.okeys, o1, o1), ctx.mul(t10.gkeys, g1, g1), f"square at {level}")
        same(ora.rescale(o1), ctx.rescale(g1), "rescale")
        same(ora.add(o1, o2), ctx.add(g1, g2), "add")
        same(ora.sub(o1, o2), ctx.sub(g1, g2), "sub")
        same(ora.add_const(o1, -0.3125), ctx.add_const(g1, -0.3125), "add_const")
        for c, tgt in [(2.5, level - 1), (-16577 / 1024, 0), (1.0, max(level - 3, 0))]:
            same(ora.cmul_to(o1, c, tgt), ctx.cmul_to(g1, c, tgt), f"cmul_to {c} {tgt}")
        mask = (np.arange(400) % 7 == 0).astype(float)
        same(ora.mul_plain(o1, mask), ctx.mul_plain(g1, mask), "mul_plain")


def test_errors_reported(ckr, t10):
    o, g = t10.enc(np.zeros(4), 0, bytes([3] * 32))
    with pytest.raises(ckr.CkrError) as e:
        t10.ctx.rescale(g)
    assert e.value.status == -3
    with pytest.raises(ckr.CkrError) as e:
        t10.ctx.rotate(t10.gkeys, g, 77)       # no key for this shift
    assert e.value.status == -1
    with pytest.raises(ckr.CkrError) as e:
        t10.ctx.sort(t10.gkeys, g, 6, (2, 1), (2, 2))  # sort: N must be a power of two
    assert e.value.status == -2
    with pytest.raises(ckr.CkrError) as e:
        t10.ctx.rank(t10.gkeys, g, 17, (2, 1))  # rank pads 17 to 32: 32^2 > 512 slots
    assert e.value.status == -2
    with pytest.raises(ckr.CkrError) as e:
        t10.ctx.rank(t10.gkeys, g, 8, (2, 1))  # level 0: too shallow
    assert e.value.status == -3


@pytest.fixture(scope="module")
def p12(ora, ckr):
    say("[gpu] P12 pair")
    return Pair(ora, ckr, "P12", W.PSETS["P12"]["L"], Ns=(8,))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rank8_bit_exact_and_exact_ranks(p12, seed):
    N = 8
    cmp = W.RANK_CMP[N]
    v, kseed, eseed = W.rank_workload(N, 0.01, seed)
    o, g = p12.enc(v, p12.P.L, eseed)
    say(f"[gpu] rank8 seed {seed}")
    ro = p12.ora.rank(p12.okeys, o, N, *cmp)
    rg = p12.ctx.rank(p12.gkeys, g, N, cmp)
    same(ro, rg, "rank8")
    dec = p12.ctx.decrypt(p12.gkeys, rg, N)
    assert np.array_equal(np.round(dec), np.argsort(np.argsort(v)) + 1)


def test_rank8_batch_equals_single(p12):
    N, cmp = 8, W.RANK_CMP[8]
    cts = []
    singles = []
    for seed in range(3):
        v, _, eseed = W.rank_workload(N, 0.01, 10 + seed)
        g = p12.ctx.encrypt(p12.gkeys, v, p12.P.L, eseed)
        cts.append(g)
        singles.append(p12.ctx.rank(p12.gkeys, g, N, cmp).export())
    outs = p12.ctx.rank_batch(p12.gkeys, cts, N, cmp)
    for s, b in zip(singles, outs):
        assert np.array_equal(s, b.export())


def test_rank8_hundred_seeds_batched_bit_exact(ora, p12):
    """Rank of N = 8 (gap 0.01) over seeds 0..99: one batch of 100 rank-8 queries
    (one graph-captured circuit after the eager first call) against the
    oracle's rank of each query alone, bit for bit, and exact ranks."""
    N, cmp = 8, W.RANK_CMP[8]
    vals, gcts, want = [], [], []
    for seed in range(100):
        v, _, eseed = W.rank_workload(N, 0.01, seed)
        vals.append(v)
        o, g = p12.enc(v, p12.P.L, eseed)
        gcts.append(g)
        want.append(ora.rank(p12.okeys, o, N, *cmp).export())
    say("[gpu] rank-8 batch of 100 (eager, captured)")
    for rep in range(2):
        outs = p12.ctx.rank_batch(p12.gkeys, gcts, N, cmp)
        for i, (o, w) in enumerate(zip(outs, want)):
            assert np.array_equal(o.export(), w), (rep, i)
    for o, v in zip(outs, vals):
        assert np.array_equal(np.round(p12.ctx.decrypt(p12.gkeys, o, N)), np.argsort(np.argsort(v)) + 1)


def test_rank8_graph_replays_equal_eager(p12):
    """Batched rank through hipGraph capture: call 1 runs eagerly, call 2 captures
    and replays, calls 3-4 replay; eager single calls run in between.  Every
    replay must equal the eager single-query results."""
    N, cmp = 8, W.RANK_CMP[8]
    cts, singles = [], []
    for seed in range(4):
        v, _, eseed = W.rank_workload(N, 0.01, 40 + seed)
        g = p12.ctx.encrypt(p12.gkeys, v, p12.P.L, eseed)
        cts.append(g)
        singles.append(p12.ctx.rank(p12.gkeys, g, N, cmp).export())
    for rep in range(4):
        outs = p12.ctx.run_batch(p12.gkeys, "rank", cts, N, cmp)
        for s, b in zip(singles, outs):
            assert np.array_equal(s, b.export()), f"replay {rep}"
        # eager work between replays
        p12.ctx.rank(p12.gkeys, cts[rep], N, cmp)


def test_graph_plan_cache_evicts_and_stays_exact(p12):
    """Captured plans are cached per (slot, circuit, batch size) and each keeps
    its temporaries; past 16 plans on a slot the least recently replayed one
    is destroyed.  Batches of 1..20 queries, three passes (eager, captured with
    evictions from the 17th size on, then re-captured after eviction): every
    result equals the same query ranked alone."""
    N, cmp = 8, W.RANK_CMP[8]
    cts, singles = [], []
    for seed in range(20):
        v, _, eseed = W.rank_workload(N, 0.01, 600 + seed)
        g = p12.ctx.encrypt(p12.gkeys, v, p12.P.L, eseed)
        cts.append(g)
        singles.append(p12.ctx.rank(p12.gkeys, g, N, cmp).export())
    for rep in range(3):
        say(f"[gpu] rank-8 batches of 1..20, pass {rep}")
        for B in range(1, 21):
            outs = p12.ctx.run_batch(p12.gkeys, "rank", cts[:B], N, cmp)
            for i, o in enumerate(outs):
                assert np.array_equal(o.export(), singles[i]), (rep, B, i)


@pytest.mark.parametrize("name", ["T10", "P12", "P16", "P17"])
def test_ntt_tile_variants_bit_identical(ckr, name):
    """Every NTT tile variant the autotuner may pick computes the same transform."""
    from paper_2412_15126_amd import hip
    ps = W.PSETS[name]
    ctx = ckr.Context(ps)
    n, nm = 1 << ps["logn"], len(ctx.moduli)
    limbs = min(nm, 6)
    rng = np.random.default_rng(1)
    host = np.stack([rng.integers(0, int(q), n, dtype=np.uint64) for q in ctx.moduli[:limbs]])
    ref = None
    for v in range(5):
        for inv in (0, 1):
            for ps_ in (0, 1):
                ctx.ntt_variant(inv, ps_, v)
        dev = hip.DeviceArray(host)
        ctx.ntt_device(dev.ptr.value, limbs, 0, False)
        hip.synchronize()
        fwd = dev.numpy()
        ctx.ntt_device(dev.ptr.value, limbs, 0, True)
        hip.synchronize()
        assert np.array_equal(dev.numpy(), host), f"variant {v} roundtrip"
        if ref is None:
            ref = fwd
        assert np.array_equal(fwd, ref), f"variant {v} forward differs"
    table = ctx.autotune(limbs * 4, 2)
    assert table.shape == (2, 2, 5) and np.all(table > 0)


@pytest.mark.parametrize("logn", [11, 13, 14, 15])
def test_keyswitch_other_ring_sizes_bit_exact(ora, ckr, logn):
    """Rotation and relinearisation (ModUp, fused row pass + inner product,
    ModDown) at the ring sizes whose transforms use 5-, 6- and 7-bit rows."""
    ps = dict(logn=logn, L=5, q0_bits=44, log_scale=36, K=3, p_bits=46, dnum=3)
    say(f"[gpu] key switch at n=2^{logn}")
    pr = Pair(ora, ckr, ps, ps["L"], shifts=(1, -7))
    v = np.random.default_rng(logn).uniform(0, 1, pr.n // 2)
    for level in (ps["L"], 2):
        o, g = pr.enc(v, level, bytes([logn] * 32))
        same(o, g, "encrypt")
        same(ora.rotate(pr.okeys, o, 1), pr.ctx.rotate(pr.gkeys, g, 1), f"rotate level {level}")
        same(ora.rotate(pr.okeys, o, -7), pr.ctx.rotate(pr.gkeys, g, -7), f"rotate -7 level {level}")
        same(ora.mul(pr.okeys, o, o), pr.ctx.mul(pr.gkeys, g, g), f"mul level {level}")


def test_keyswitch_many_digits_bit_exact(ora, ckr):
    """One prime per digit and the library's largest digit count, 8 at the
    top level: the inner product accumulates its 8 products unreduced before
    reducing."""
    ps = dict(logn=10, L=7, q0_bits=44, log_scale=36, K=1, p_bits=46, dnum=8)
    say("[gpu] key switch with 8 digits")
    pr = Pair(ora, ckr, ps, ps["L"], shifts=(3,))
    v = np.random.default_rng(12).uniform(0, 1, pr.n // 2)
    for level in (ps["L"], 5, 2):
        o, g = pr.enc(v, level, bytes([level] * 32))
        same(ora.rotate(pr.okeys, o, 3), pr.ctx.rotate(pr.gkeys, g, 3), f"rotate level {level}")
        same(ora.mul(pr.okeys, o, o), pr.ctx.mul(pr.gkeys, g, g), f"mul level {level}")


def test_row_ip_tile_variants_bit_identical(ckr):
    """Every tile of the fused row pass + inner product gives the same
    relinearised product at n = 2^16 (rows of 2^8 points)."""
    ps = W.PSETS["P16"]
    ctx = ckr.Context(ps)
    keys = ctx.keygen(bytes(range(9, 41)), 9, [])
    v = np.random.default_rng(5).uniform(0, 1, 1 << 15)
    cts = [ctx.encrypt(keys, v, lv, bytes([lv] * 32)) for lv in (9, 4)]
    ref = None
    for var in range(8):
        say(f"[gpu] row_ip variant {var}")
        ctx.row_ip_variant(var)
        got = [ctx.mul(keys, c, c).export() for c in cts]
        if ref is None:
            ref = got
        assert all(np.array_equal(a, b) for a, b in zip(ref, got)), f"variant {var}"
    ms = ctx.autotune_row_ip(4, 2)
    assert ms.shape == (8,) and np.all(ms > 0)


def test_rank8_ntt_chunking_bit_identical(p12):
    """Cache-chunked transforms give the same ciphertexts as whole dispatches."""
    N, cmp = 8, W.RANK_CMP[8]
    cts = [p12.ctx.encrypt(p12.gkeys, W.rank_workload(N, 0.01, 60 + s)[0], p12.P.L, bytes([s] * 32)) for s in range(3)]
    p12.ctx.set_graphs(False)
    try:
        ref = [o.export() for o in p12.ctx.run_batch(p12.gkeys, "rank", cts, N, cmp)]
        for chunk in (1, 5, 24):
            p12.ctx.set_ntt_chunk(chunk)
            got = [o.export() for o in p12.ctx.run_batch(p12.gkeys, "rank", cts, N, cmp)]
            assert all(np.array_equal(a, b) for a, b in zip(ref, got)), chunk
    finally:
        p12.ctx.set_ntt_chunk(0)
        p12.ctx.set_graphs(True)


def test_rank8_tuning_changes_between_replays(p12):
    """A captured batch replayed, then run again after each tile or chunk
    change (each makes the next run capture its graph again): every run
    gives the eager result bit for bit."""
    N, cmp = 8, W.RANK_CMP[8]
    ctx = p12.ctx
    cts = [ctx.encrypt(p12.gkeys, W.rank_workload(N, 0.01, 80 + s)[0], p12.P.L, bytes([s + 7] * 32)) for s in range(4)]
    run = lambda: [o.export() for o in ctx.run_batch(p12.gkeys, "rank", cts, N, cmp)]
    ref = run()            # eager
    changes = [lambda: ctx.ntt_variant(1, 0, 4), lambda: ctx.ntt_variant(0, 1, 3), lambda: ctx.set_ntt_chunk(5),
               lambda: ctx.row_ip_variant(6), lambda: ctx.autotune(8, 1)]
    try:
        for i, change in enumerate([None] + changes):
            if change:
                say(f"[gpu] tuning change {i}")
                change()
            for _ in range(2):     # capture (or re-capture), then replay
                got = run()
                assert all(np.array_equal(a, b) for a, b in zip(ref, got)), i
    finally:
        for inv in (0, 1):
            for ps_ in (0, 1):
                ctx.ntt_variant(inv, ps_, 0)
        ctx.set_ntt_chunk(0)
        ctx.row_ip_variant(7)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_minimax_comparator_bit_exact(ora, ckr, k):
    """k stages of the minimax composite on ciphertexts (the constants of
    stage 0 reach 126) against the oracle, bit for bit, at n = 2^12, and rank
    of 8 values with four stages."""
    ps = W.PSETS["T12D"]
    say(f"[gpu] minimax comparator, {k} stages")
    pr = Pair(ora, ckr, ps, 16, Ns=(8,))
    v = np.random.default_rng(30 + k).uniform(-1, 1, pr.n // 2)
    o, g = pr.enc(v, 16, bytes([k] * 32))
    same(ora.cmp_sign(pr.okeys, o, 0, 0, 0, k), pr.ctx.cmp_sign(pr.gkeys, g, (0, 0, 0, k)), f"minimax {k}")
    if k == 3:
        w, _, eseed = W.rank_workload(8, 0.01, 77)
        o, g = pr.enc(w, 14, eseed)
        same(ora.rank(pr.okeys, o, 8, 0, 0, 0, 4), pr.ctx.rank(pr.gkeys, g, 8, (0, 0, 0, 4)), "rank-8 minimax")

