"""The allocation-free rotation (ckr_op_rotate_into): its key switch runs on
the library's file-scope device scratch array and takes nothing from the
context's allocator or pool.  Two calls in a row, the second on a smaller
input (fewer limbs), must equal ckr_op_rotate bit for bit; sizes beyond the
scratch array are rejected.  (Named to run last: it must pass alone in a
fresh process and after every other test.)"""
import gc
import sys

import numpy as np
import pytest

from paper_2412_15126_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Counting:
    def __init__(self):
        self.allocs = self.frees = 0
        self.sizes = {}

    def alloc(self, nbytes):
        import ctypes as C
        from paper_2412_15126_amd import hip
        p = C.c_void_p()
        if hip.rt().hipMalloc(C.byref(p), nbytes) != 0:
            return 0
        self.allocs += 1
        self.sizes[p.value] = nbytes
        return p.value

    def free(self, ptr):
        from paper_2412_15126_amd import hip
        self.sizes.pop(ptr)
        self.frees += 1
        hip.rt().hipFree(ptr)


def _rotations(ckr, ctx, al, pname):
    ps = W.PSETS[pname]
    N = 8 if pname == "P12" else 128
    lv = 11 if pname == "P12" else 17
    v, kseed, eseed = W.rank_workload(N, 0.01 if N == 8 else 2.0 ** -10, 5)
    keys = ctx.keygen(kseed, lv, [N])
    shifts = [N, -1]                                        # SumR's and ReplC's first rotations
    big = ctx.encrypt(keys, v, lv, eseed)
    small = ctx.encrypt(keys, v, lv - 4, eseed)
    wants = [[ctx.rotate(keys, c, k).export() for k in shifts] for c in (big, small)]
    outs = [[[ctx.encrypt(keys, np.zeros(N), c.level, eseed) for _ in shifts] for c in (big, small)]
            for _ in range(2)]
    ctx.synchronize()
    mem, calls = ctx.memory(), (al.allocs, al.frees)
    say(f"[gpu] {pname}: allocation-free rotations at levels {lv} and {lv - 4}")
    for rep in range(2):
        for c, os_ in zip((big, small), outs[rep]):      # the second call has fewer limbs
            for k, o in zip(shifts, os_):
                ctx.rotate_into(keys, c, k, o)
    ctx.synchronize()
    assert ctx.memory() == mem and (al.allocs, al.frees) == calls
    for rep in range(2):
        for os_, w in zip(outs[rep], wants):
            for o, wk in zip(os_, w):
                assert np.array_equal(o.export(), wk), (rep, o.level)
    o0, o1 = outs[0][0]
    # a rotation by a multiple of n/2 is the identity (a copy)
    ctx.rotate_into(keys, big, ctx.n // 2, o0)
    assert np.array_equal(o0.export(), big.export())
    # out must be at the input's level and must not be the input
    with pytest.raises(ckr.CkrError) as e:
        ctx.rotate_into(keys, small, N, o1)
    assert e.value.status == -1
    with pytest.raises(ckr.CkrError) as e:
        ctx.rotate_into(keys, big, N, big)
    assert e.value.status == -1


@pytest.mark.parametrize("pname", ["P12", "P16"])
def test_rotate_into_allocates_nothing_and_equals_rotate(pname):
    import paper_2412_15126_amd as ckr
    al = Counting()
    ctx = ckr.Context(W.PSETS[pname])
    ctx.set_allocator(al.alloc, al.free)
    _rotations(ckr, ctx, al, pname)
    gc.collect()
    ctx.close()
    assert al.allocs == al.frees


def test_rotate_into_rejects_beyond_scratch():
    """n = 2^17 at level 20 with 5 special primes and 3 digits needs
    (21 + 3*26 + 2*26 + 2*21) limbs of 1 MiB = 193 MiB > 128 MiB"""
    import paper_2412_15126_amd as ckr
    ps = dict(logn=17, L=20, q0_bits=50, log_scale=40, K=5, p_bits=50, dnum=3)
    ctx = ckr.Context(ps)
    v, kseed, eseed = W.rank_workload(8, 0.01, 6)
    keys = ctx.keygen(kseed, ps["L"], [8])
    a = ctx.encrypt(keys, v, ps["L"], eseed)
    o = ctx.encrypt(keys, v, ps["L"], eseed)
    before = o.export()
    with pytest.raises(ckr.CkrError) as e:
        ctx.rotate_into(keys, a, 1, o)
    assert e.value.status == -4 and "scratch" in str(e.value)
    assert np.array_equal(o.export(), before)
