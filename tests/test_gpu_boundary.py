"""The C ABI's hooks for PyTorch-style interop (include/ckr.h): an external
allocator (ckr_context_set_allocator), an external stream
(ckr_context_set_stream) and allocation failure.  Every result must equal the
default context's bit for bit; every block the allocator hands out must come
back to it, also after a failed call."""
import gc
import sys

import numpy as np
import pytest

from paper_2412_15126_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class CountingAllocator:
    """hipMalloc / hipFree through the HIP runtime the library links, with
    counts, live bytes and an optional failure after `fail_after` blocks"""

    def __init__(self):
        self.allocs = self.frees = self.live = self.peak = 0
        self.sizes = {}
        self.fail_after = None
        self.refused = 0

    def alloc(self, nbytes):
        import ctypes as C
        from paper_2412_15126_amd import hip
        if self.fail_after is not None and self.allocs >= self.fail_after:
            self.refused += 1
            return 0
        p = C.c_void_p()
        if hip.rt().hipMalloc(C.byref(p), nbytes) != 0 or not p.value:
            return 0
        self.allocs += 1
        self.sizes[p.value] = nbytes
        self.live += nbytes
        self.peak = max(self.peak, self.live)
        return p.value

    def free(self, ptr):
        from paper_2412_15126_amd import hip
        assert ptr in self.sizes, "freed a block the allocator never handed out"
        self.live -= self.sizes.pop(ptr)
        self.frees += 1
        hip.rt().hipFree(ptr)


def _rank8(ctx, seed=0):
    ps = W.PSETS["P12"]
    v, kseed, eseed = W.rank_workload(8, 0.01, seed)
    keys = ctx.keygen(kseed, ps["L"], [8])
    ct = ctx.encrypt(keys, v, ps["L"], eseed)
    return keys, ct, v


def test_allocator_hook_bit_identical_and_balanced():
    import paper_2412_15126_amd as ckr
    ps = W.PSETS["P12"]
    ref_ctx = ckr.Context(ps)
    keys, ct, v = _rank8(ref_ctx)
    want = ref_ctx.rank(keys, ct, 8, W.RANK_CMP[8]).export()

    al = CountingAllocator()
    ctx = ckr.Context(ps)
    ctx.set_allocator(al.alloc, al.free)
    say("[gpu] rank-8 through the counting allocator")
    k2, c2, _ = _rank8(ctx)
    got = ctx.rank(k2, c2, 8, W.RANK_CMP[8])
    assert np.array_equal(got.export(), want)
    assert np.array_equal(np.round(ctx.decrypt(k2, got, 8)), np.argsort(np.argsort(v)) + 1)
    in_use, high = ctx.memory()
    assert al.allocs > 0 and al.live >= in_use > 0 and al.peak >= high
    # too late: blocks exist
    with pytest.raises(ckr.CkrError) as e:
        ctx.set_allocator(al.alloc, al.free)
    assert e.value.status == -1
    del got, c2, k2
    gc.collect()
    ctx.close()
    assert al.live == 0 and al.allocs == al.frees


def _failing_rank(ps, k, want):
    """rank-8 on a fresh context whose allocator refuses every block after the
    k-th one past key generation and encryption; then the same call with the
    allocator healthy again"""
    import paper_2412_15126_amd as ckr
    al = CountingAllocator()
    ctx = ckr.Context(ps)
    ctx.set_allocator(al.alloc, al.free)

    def run():
        keys, ct, _ = _rank8(ctx)
        al.fail_after = al.allocs + k
        with pytest.raises(ckr.CkrError) as e:
            ctx.rank(keys, ct, 8, W.RANK_CMP[8])
        assert e.value.status == -4          # CKR_E_NOMEM
        assert al.refused == 1
        al.fail_after = None
        got = ctx.rank(keys, ct, 8, W.RANK_CMP[8])    # the context still works
        assert np.array_equal(got.export(), want)

    run()
    gc.collect()
    ctx.close()
    assert al.live == 0 and al.allocs == al.frees    # no block lost on the failure path


def test_allocator_failure_injection_no_leak():
    import paper_2412_15126_amd as ckr
    ps = W.PSETS["P12"]
    ref = ckr.Context(ps)
    rk, rc, _ = _rank8(ref)
    want = ref.rank(rk, rc, 8, W.RANK_CMP[8]).export()
    for k in (0, 1, 3, 7):
        say(f"[gpu] rank-8 with the allocator failing after {k} more blocks")
        _failing_rank(ps, k, want)


def test_external_stream_bit_identical():
    import paper_2412_15126_amd as ckr
    from paper_2412_15126_amd import hip
    ps = W.PSETS["P12"]
    ref = ckr.Context(ps)
    rk, rc, _ = _rank8(ref, 3)
    want = ref.rank(rk, rc, 8, W.RANK_CMP[8]).export()
    s = hip.Stream()
    ctx = ckr.Context(ps)
    ctx.set_stream(s.h.value)
    say("[gpu] rank-8 on an external stream (eager, captured, replayed)")
    keys, ct, _ = _rank8(ctx, 3)
    assert np.array_equal(ctx.rank(keys, ct, 8, W.RANK_CMP[8]).export(), want)
    for rep in range(3):
        outs = ctx.rank_batch(keys, [ct, ct], 8, W.RANK_CMP[8])
        s.synchronize()
        assert all(np.array_equal(o.export(), want) for o in outs), rep
    ctx.close()
