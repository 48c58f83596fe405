"""Python binding of libckr.so (include/ckr.h): argument marshalling only.

Every homomorphic step runs in the library's HIP kernels.  Importing this
module loads the built library and raises if it is missing; there is no
fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libckr.so")

STATUS = {0: "ok", -1: "invalid", -2: "range", -3: "depth", -4: "nomem", -5: "device", -6: "busy"}


class CkrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("log_n", C.c_uint32), ("n_q", C.c_uint32), ("q0_bits", C.c_uint32), ("log_scale", C.c_uint32),
                ("n_p", C.c_uint32), ("p_bits", C.c_uint32), ("dnum", C.c_uint32)]

    @staticmethod
    def of(pset):
        return Params(pset["logn"], pset["L"] + 1, pset["q0_bits"], pset["log_scale"], pset["K"], pset["p_bits"],
                      pset["dnum"])


class Sign(C.Structure):
    _fields_ = [("d_g", C.c_uint8), ("d_f", C.c_uint8), ("cheb", C.c_uint8), ("minimax", C.c_uint8)]


class Query(C.Structure):
    _fields_ = [("kind", C.c_int), ("N", C.c_uint32), ("k", C.c_uint32), ("tie_correct", C.c_int),
                ("cmp", Sign), ("ind", Sign), ("v", C.c_void_p)]


vp = C.c_void_p
u64p = C.POINTER(C.c_uint64)
i64p = C.POINTER(C.c_int64)
dblp = C.POINTER(C.c_double)
u32p = C.POINTER(C.c_uint32)

_SIGS = {
    "ckr_last_error": (C.c_char_p, []),
    "ckr_context_create": (C.c_int, [C.POINTER(Params), C.c_int, C.c_size_t, C.POINTER(vp)]),
    "ckr_context_free": (None, [vp]),
    "ckr_context_set_stream": (C.c_int, [vp, vp]),
    "ckr_context_set_allocator": (C.c_int, [vp, vp, vp, vp]),
    "ckr_context_info": (C.c_int, [vp, u64p, dblp]),
    "ckr_params_derive": (C.c_int, [C.POINTER(Params), u64p, dblp]),
    "ckr_encode": (C.c_int, [C.c_uint32, dblp, C.c_uint32, C.c_double, i64p]),
    "ckr_sample": (C.c_int, [C.c_char_p, C.c_uint32, C.c_uint64, C.c_int, C.c_uint64, C.c_size_t, i64p]),
    "ckr_context_memory": (C.c_int, [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "ckr_keygen": (C.c_int, [vp, C.c_char_p, C.c_uint32, u32p, C.c_size_t, C.c_uint32, C.POINTER(vp)]),
    "ckr_keys_free": (None, [vp]),
    "ckr_keys_add_rotations": (C.c_int, [vp, vp, i64p, C.c_size_t]),
    "ckr_encrypt": (C.c_int, [vp, vp, dblp, C.c_uint32, C.c_uint32, C.c_char_p, C.POINTER(vp)]),
    "ckr_decrypt": (C.c_int, [vp, vp, vp, dblp, C.c_uint32]),
    "ckr_rank": (C.c_int, [vp, vp, vp, C.c_uint32, Sign, C.c_int, C.POINTER(vp)]),
    "ckr_rank_depth": (C.c_uint32, [Sign, C.c_int]),
    "ckr_rank_depth_n": (C.c_uint32, [C.c_uint32, Sign, C.c_int]),
    "ckr_argmin_depth": (C.c_uint32, [Sign, Sign]),
    "ckr_order_stat_depth": (C.c_uint32, [C.c_uint32, C.c_uint32, Sign, Sign, C.c_int]),
    "ckr_order_stat": (C.c_int, [vp, vp, vp, C.c_uint32, C.c_uint32, Sign, Sign, C.c_int, C.POINTER(vp),
                                 C.POINTER(vp)]),
    "ckr_run_mixed": (C.c_int, [vp, vp, C.POINTER(Query), C.c_size_t, C.POINTER(vp)]),
    "ckr_rank_multi": (C.c_int, [vp, vp, C.POINTER(vp), C.c_uint32, C.c_uint32, Sign, C.POINTER(vp)]),
    "ckr_rank_multi_depth": (C.c_uint32, [Sign]),
    "ckr_sort_multi": (C.c_int, [vp, vp, C.POINTER(vp), C.c_uint32, C.c_uint32, Sign, Sign, C.POINTER(vp)]),
    "ckr_sort_multi_depth": (C.c_uint32, [Sign, Sign]),
    "ckr_sort_depth": (C.c_uint32, [Sign, Sign]),
    "ckr_argmin": (C.c_int, [vp, vp, vp, C.c_uint32, Sign, Sign, C.POINTER(vp), C.POINTER(vp)]),
    "ckr_sort": (C.c_int, [vp, vp, vp, C.c_uint32, Sign, Sign, C.POINTER(vp)]),
    "ckr_sort_col": (C.c_int, [vp, vp, vp, C.c_uint32, Sign, Sign, C.POINTER(vp)]),
    "ckr_sort_col_depth": (C.c_uint32, [Sign, Sign]),
    "ckr_order_stat_div": (C.c_int, [vp, vp, C.POINTER(vp), C.c_size_t, C.c_uint32, C.c_uint32, Sign, Sign,
                                     C.c_uint32, C.POINTER(vp), C.POINTER(vp)]),
    "ckr_order_stat_div_depth": (C.c_uint32, [C.c_uint32, C.c_uint32, Sign, Sign, C.c_uint32]),
    "ckr_order_range": (C.c_int, [vp, vp, C.POINTER(vp), C.c_size_t, C.c_uint32, C.c_uint32, C.c_uint32, Sign, Sign,
                                  C.c_int, C.POINTER(vp), C.POINTER(vp)]),
    "ckr_order_range_depth": (C.c_uint32, [C.c_uint32, C.c_uint32, C.c_uint32, Sign, Sign, C.c_int]),
    "ckr_rank_batch": (C.c_int, [vp, vp, C.POINTER(vp), C.c_size_t, C.c_uint32, Sign, C.POINTER(vp)]),
    "ckr_ct_level": (C.c_uint32, [vp]),
    "ckr_ct_scale": (C.c_double, [vp]),
    "ckr_ct_export": (C.c_int, [vp, vp, u64p, C.c_size_t]),
    "ckr_ct_import": (C.c_int, [vp, u64p, C.c_size_t, C.c_uint32, C.POINTER(vp)]),
    "ckr_ct_free": (None, [vp]),
    "ckr_op_rotate": (C.c_int, [vp, vp, vp, C.c_int64, C.POINTER(vp)]),
    "ckr_op_rotate_into": (C.c_int, [vp, vp, vp, C.c_int64, vp]),
    "ckr_op_mul": (C.c_int, [vp, vp, vp, vp, C.POINTER(vp)]),
    "ckr_op_cheb_eval": (C.c_int, [vp, vp, vp, dblp, C.c_uint32, C.POINTER(vp)]),
    "ckr_op_cmp_sign": (C.c_int, [vp, vp, vp, Sign, C.POINTER(vp)]),
    "ckr_op_add": (C.c_int, [vp, vp, vp, C.POINTER(vp)]),
    "ckr_op_sub": (C.c_int, [vp, vp, vp, C.POINTER(vp)]),
    "ckr_op_rescale": (C.c_int, [vp, vp, C.POINTER(vp)]),
    "ckr_op_cmul_to": (C.c_int, [vp, vp, C.c_double, C.c_uint32, C.POINTER(vp)]),
    "ckr_op_add_const": (C.c_int, [vp, vp, C.c_double, C.POINTER(vp)]),
    "ckr_op_mul_plain": (C.c_int, [vp, vp, dblp, C.c_uint32, C.POINTER(vp)]),
    "ckr_ntt_device": (C.c_int, [vp, vp, C.c_uint32, C.c_uint32, C.c_int]),
    "ckr_set_profiling": (C.c_int, [vp, C.c_int]),
    "ckr_profile_reset": (C.c_int, [vp]),
    "ckr_profile_read": (C.c_int, [vp, C.c_int, C.POINTER(C.c_uint64), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ckr_profile_name": (C.c_char_p, [C.c_int]),
    "ckr_synchronize": (C.c_int, [vp]),
    "ckr_run_batch": (C.c_int, [vp, vp, C.c_int, C.c_uint32, Sign, Sign, C.POINTER(vp), C.c_size_t, C.POINTER(vp)]),
    "ckr_context_set_graphs": (C.c_int, [vp, C.c_int]),
    "ckr_autotune": (C.c_int, [vp, C.c_uint32, C.c_uint32, C.POINTER(C.c_float)]),
    "ckr_server_create": (C.c_int, [C.c_size_t, C.c_uint32, C.POINTER(vp)]),
    "ckr_server_add_route": (C.c_int, [vp, C.c_int, C.c_uint32, vp, vp, Sign, Sign]),
    "ckr_server_submit": (C.c_int, [vp, C.c_int, C.c_uint32, vp, C.POINTER(C.c_uint64)]),
    "ckr_server_wait": (C.c_int, [vp, C.c_uint64, C.c_int, C.POINTER(vp), C.c_size_t, C.POINTER(C.c_double)]),
    "ckr_server_stats": (C.c_int, [vp, C.POINTER(C.c_double)]),
    "ckr_server_free": (None, [vp]),
    "ckr_ntt_variant": (C.c_int, [vp, C.c_int, C.c_int, C.c_int]),
    "ckr_autotune_row_ip": (C.c_int, [vp, C.c_uint32, C.c_uint32, C.POINTER(C.c_float)]),
    "ckr_row_ip_variant": (C.c_int, [vp, C.c_int]),
    "ckr_set_ntt_chunk": (C.c_int, [vp, C.c_uint32]),
}

_lib = None


def lib():
    """Load libckr.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2412_15126_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ok(st):
    if st != 0:
        raise CkrError(st, lib().ckr_last_error().decode())


def _p(a, t):
    return a.ctypes.data_as(t)


def sign(cmp):
    """(d_g, d_f) for the f/g composite, (0, 0, D) for the Chebyshev comparator
    of D levels, (0, 0, 0, k) for k stages of the minimax composite"""
    c = tuple(int(x) for x in cmp) + (0, 0)
    return Sign(c[0], c[1], c[2], c[3])


# ---- host-only helpers ------------------------------------------------------
def derive_params(pset):
    nq, K = pset["L"] + 1, pset["K"]
    mods = np.zeros(nq + K, np.uint64)
    scales = np.zeros(nq, np.float64)
    _ok(lib().ckr_params_derive(C.byref(Params.of(pset)), _p(mods, u64p), _p(scales, dblp)))
    return mods, scales


def encode(log_n, z, scale):
    z = np.ascontiguousarray(z, np.float64)
    m = np.zeros(1 << log_n, np.int64)
    _ok(lib().ckr_encode(log_n, _p(z, dblp), len(z), scale, _p(m, i64p)))
    return m


def sample(seed, purpose, oid, kind, q, count):
    out = np.zeros(count, np.int64)
    _ok(lib().ckr_sample(bytes(seed), purpose, oid, kind, q, count, _p(out, i64p)))
    return out


def rank_depth(cmp, tie=False):
    return int(lib().ckr_rank_depth(sign(cmp), int(tie)))


def rank_depth_n(N, cmp, tie=False):
    """levels of rank on N values (one more when N is not a power of two)"""
    return int(lib().ckr_rank_depth_n(N, sign(cmp), int(tie)))


def rank_multi_depth(cmp):
    return int(lib().ckr_rank_multi_depth(sign(cmp)))


def sort_multi_depth(cmp, ind):
    return int(lib().ckr_sort_multi_depth(sign(cmp), sign(ind)))


def order_stat_depth(N, k, cmp, ind, tie):
    return int(lib().ckr_order_stat_depth(N, k, sign(cmp), sign(ind), int(tie)))


def argmin_depth(cmp, ind):
    return int(lib().ckr_argmin_depth(sign(cmp), sign(ind)))


def sort_depth(cmp, ind):
    return int(lib().ckr_sort_depth(sign(cmp), sign(ind)))


def order_stat_div_depth(N, k, cmp, ind, iters):
    return int(lib().ckr_order_stat_div_depth(N, k, sign(cmp), sign(ind), iters))


def sort_col_depth(cmp, ind):
    return int(lib().ckr_sort_col_depth(sign(cmp), sign(ind)))


def order_range_depth(N, a, b, cmp, ind, tie):
    return int(lib().ckr_order_range_depth(N, a, b, sign(cmp), sign(ind), int(tie)))


def median_window(N):
    """the rank window of the median: [N/2, N/2 + 1] for an even N, the middle rank for an odd N"""
    return (N // 2, N // 2 + 1) if N % 2 == 0 else ((N + 1) // 2, (N + 1) // 2)


# ---- device objects -----------------------------------------------------------
class Context:
    def __init__(self, pset, device=0, hbm_budget=0):
        self.pset = dict(pset)
        self.n = 1 << pset["logn"]
        self.L = pset["L"]
        h = vp()
        _ok(lib().ckr_context_create(C.byref(Params.of(pset)), device, hbm_budget, C.byref(h)))
        self.h = h
        nq, K = pset["L"] + 1, pset["K"]
        self.moduli = np.zeros(nq + K, np.uint64)
        self.scales = np.zeros(nq, np.float64)
        _ok(lib().ckr_context_info(self.h, _p(self.moduli, u64p), _p(self.scales, dblp)))

    def close(self):
        if getattr(self, "h", None):
            lib().ckr_context_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def set_stream(self, stream_ptr):
        _ok(lib().ckr_context_set_stream(self.h, vp(stream_ptr)))

    def set_allocator(self, alloc, free):
        """Route the context's device allocations through alloc(nbytes) -> device
        pointer (int; 0 or None fails the allocation) and free(ptr); must come
        before any key or ciphertext exists.  The callbacks stay referenced by
        the context."""
        AF = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
        FF = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
        cbs = (AF(lambda nbytes, user: alloc(nbytes) or None), FF(lambda ptr, user: free(ptr)))
        _ok(lib().ckr_context_set_allocator(self.h, C.cast(cbs[0], vp), C.cast(cbs[1], vp), None))
        self._allocator = cbs

    def memory(self):
        a, b = C.c_size_t(), C.c_size_t()
        _ok(lib().ckr_context_memory(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    # -- keys and ciphertexts
    def keygen(self, seed, max_level, Ns=(), what=1):
        Ns = np.array(list(Ns), np.uint32)
        h = vp()
        _ok(lib().ckr_keygen(self.h, bytes(seed), max_level, _p(Ns, u32p), len(Ns), what, C.byref(h)))
        return Keys(self, h)

    def encrypt(self, keys, v, level, seed):
        v = np.ascontiguousarray(v, np.float64)
        h = vp()
        _ok(lib().ckr_encrypt(self.h, keys.h, _p(v, dblp), len(v), level, bytes(seed), C.byref(h)))
        return Ct(self, h)

    def decrypt(self, keys, ct, count):
        out = np.zeros(count, np.float64)
        _ok(lib().ckr_decrypt(self.h, keys.h, ct.h, _p(out, dblp), count))
        return out

    def import_ct(self, arr):
        arr = np.ascontiguousarray(arr, np.uint64)
        h = vp()
        _ok(lib().ckr_ct_import(self.h, _p(arr, u64p), arr.size, arr.shape[1] - 1, C.byref(h)))
        return Ct(self, h)

    # -- circuits
    def rank(self, keys, ct, N, cmp, tie=False):
        h = vp()
        _ok(lib().ckr_rank(self.h, keys.h, ct.h, N, sign(cmp), int(tie), C.byref(h)))
        return Ct(self, h)

    def rank_multi(self, keys, blocks, b, cmp):
        """Multi-ciphertext ranking: blocks of b values -> one rank block per input block."""
        arr = (vp * len(blocks))(*[x.h for x in blocks])
        out = (vp * len(blocks))()
        _ok(lib().ckr_rank_multi(self.h, keys.h, arr, len(blocks), b, sign(cmp), out))
        return [Ct(self, vp(o)) for o in out]

    def sort_multi(self, keys, blocks, b, cmp, ind):
        """Multi-ciphertext sorting: blocks of b distinct values -> the sorted vector, block by block."""
        arr = (vp * len(blocks))(*[x.h for x in blocks])
        out = (vp * len(blocks))()
        _ok(lib().ckr_sort_multi(self.h, keys.h, arr, len(blocks), b, sign(cmp), sign(ind), out))
        return [Ct(self, vp(o)) for o in out]

    def order_stat(self, keys, ct, N, k, cmp, ind, tie):
        """(onehot, value) of the k-th smallest element."""
        oh, val = vp(), vp()
        _ok(lib().ckr_order_stat(self.h, keys.h, ct.h, N, k, sign(cmp), sign(ind), int(tie), C.byref(oh),
                                 C.byref(val)))
        return Ct(self, oh), Ct(self, val)

    def argmin(self, keys, ct, N, cmp, ind):
        oh, val = vp(), vp()
        _ok(lib().ckr_argmin(self.h, keys.h, ct.h, N, sign(cmp), sign(ind), C.byref(oh), C.byref(val)))
        return Ct(self, oh), Ct(self, val)

    def sort(self, keys, ct, N, cmp, ind):
        h = vp()
        _ok(lib().ckr_sort(self.h, keys.h, ct.h, N, sign(cmp), sign(ind), C.byref(h)))
        return Ct(self, h)

    def order_stat_div(self, keys, cts, N, k, cmp, ind, iters):
        """[(mask, value)] per input: order statistic k without tie-correction, value by Goldschmidt division"""
        arr = (vp * len(cts))(*[c.h for c in cts])
        oh, val = (vp * len(cts))(), (vp * len(cts))()
        _ok(lib().ckr_order_stat_div(self.h, keys.h, arr, len(cts), N, k, sign(cmp), sign(ind), iters, oh, val))
        return [(Ct(self, vp(oh[i])), Ct(self, vp(val[i]))) for i in range(len(cts))]

    def order_range(self, keys, cts, N, a, b, cmp, ind, tie):
        """[(mask, value)] per input: the elements of rank a..b and the mean of the order statistics a..b"""
        arr = (vp * len(cts))(*[c.h for c in cts])
        oh, val = (vp * len(cts))(), (vp * len(cts))()
        _ok(lib().ckr_order_range(self.h, keys.h, arr, len(cts), N, a, b, sign(cmp), sign(ind), int(tie), oh, val))
        return [(Ct(self, vp(oh[i])), Ct(self, vp(val[i]))) for i in range(len(cts))]

    def median(self, keys, cts, N, cmp, ind, tie=True):
        """[(mask, value)] per input: the median (section 4) as the rank window of median_window(N)"""
        return self.order_range(keys, cts, N, *median_window(N), cmp, ind, tie)

    def sort_col(self, keys, ct, N, cmp, ind):
        """column-form sort: no final transposition, one level fewer"""
        h = vp()
        _ok(lib().ckr_sort_col(self.h, keys.h, ct.h, N, sign(cmp), sign(ind), C.byref(h)))
        return Ct(self, h)

    def autotune(self, limbs, iters=5):
        """Pick the fastest NTT tile per (direction, pass); returns the timing table [inv][pass][variant] in ms."""
        ms = (C.c_float * 20)()
        _ok(lib().ckr_autotune(self.h, limbs, iters, ms))
        return np.array(ms[:], dtype=np.float64).reshape(2, 2, 5)

    def autotune_row_ip(self, batch, iters=3):
        """Pick the fastest tile of the fused row pass + key-switch inner product; returns ms per variant."""
        ms = (C.c_float * 8)()
        _ok(lib().ckr_autotune_row_ip(self.h, int(batch), int(iters), ms))
        return np.array(ms[:], dtype=np.float64)

    def set_ntt_chunk(self, limbs):
        _ok(lib().ckr_set_ntt_chunk(self.h, int(limbs)))

    def ntt_variant(self, inverse, pass_, variant):
        _ok(lib().ckr_ntt_variant(self.h, int(inverse), int(pass_), int(variant)))

    def row_ip_variant(self, variant):
        _ok(lib().ckr_row_ip_variant(self.h, int(variant)))

    def set_graphs(self, on):
        _ok(lib().ckr_context_set_graphs(self.h, int(on)))

    def run_batch(self, keys, kind, cts, N, cmp, ind=(0, 0)):
        """kind: 'rank', 'argmin' (returns (onehot, value) pairs) or 'sort'."""
        k = {"rank": 1, "argmin": 2, "sort": 3, "sort_col": 5}[kind]
        per = 2 if kind == "argmin" else 1
        arr = (vp * len(cts))(*[c.h for c in cts])
        out = (vp * (per * len(cts)))()
        _ok(lib().ckr_run_batch(self.h, keys.h, k, N, sign(cmp), sign(ind), arr, len(cts), out))
        res = [Ct(self, vp(o)) for o in out]
        return [tuple(res[2 * i:2 * i + 2]) for i in range(len(cts))] if per == 2 else res

    def run_mixed(self, keys, queries):
        """queries: dicts with kind ('rank', 'argmin', 'sort', 'order'), N, ct, cmp and, as
        needed, ind, k, tie.  Returns per query a Ct or an (onehot, value) pair."""
        kinds = {"rank": 1, "argmin": 2, "sort": 3, "order": 4, "sort_col": 5}
        arr = (Query * len(queries))()
        for a, q in zip(arr, queries):
            a.kind, a.N, a.k, a.tie_correct = kinds[q["kind"]], q["N"], q.get("k", 1), int(q.get("tie", False))
            a.cmp, a.ind, a.v = sign(q["cmp"]), sign(q.get("ind", (0, 0))), q["ct"].h.value
        out = (vp * (2 * len(queries)))()
        _ok(lib().ckr_run_mixed(self.h, keys.h, arr, len(queries), out))
        res = []
        for i in range(len(queries)):
            a, b = out[2 * i], out[2 * i + 1]
            res.append((Ct(self, vp(a)), Ct(self, vp(b))) if b else Ct(self, vp(a)))
        return res

    def rank_batch(self, keys, cts, N, cmp):
        arr = (vp * len(cts))(*[c.h for c in cts])
        out = (vp * len(cts))()
        _ok(lib().ckr_rank_batch(self.h, keys.h, arr, len(cts), N, sign(cmp), out))
        return [Ct(self, vp(o)) for o in out]

    # -- single operations
    def _unary(self, fn, *args):
        h = vp()
        _ok(fn(self.h, *args, C.byref(h)))
        return Ct(self, h)

    def rotate(self, keys, a, k):
        return self._unary(lib().ckr_op_rotate, keys.h, a.h, int(k))

    def rotate_into(self, keys, a, k, out):
        """the rotation of ckr_op_rotate written into the existing ciphertext
        `out` (a's level), allocating no device memory"""
        _ok(lib().ckr_op_rotate_into(self.h, keys.h, a.h, int(k), out.h))
        return out

    def cmp_sign(self, keys, a, cmp):
        """Cmp on a ciphertext of differences (section 2.2) under the comparator spec cmp"""
        return self._unary(lib().ckr_op_cmp_sign, keys.h, a.h, sign(cmp))

    def mul(self, keys, a, b):
        return self._unary(lib().ckr_op_mul, keys.h, a.h, b.h)

    def cheb_eval(self, keys, a, coeffs):
        """sum_i coeffs[i] T_i(a) by Paterson-Stockmeyer (len(coeffs) a power of two)"""
        c = np.ascontiguousarray(coeffs, np.float64)
        return self._unary(lib().ckr_op_cheb_eval, keys.h, a.h, _p(c, dblp), len(c))

    def add(self, a, b):
        return self._unary(lib().ckr_op_add, a.h, b.h)

    def sub(self, a, b):
        return self._unary(lib().ckr_op_sub, a.h, b.h)

    def rescale(self, a):
        return self._unary(lib().ckr_op_rescale, a.h)

    def cmul_to(self, a, c, target):
        return self._unary(lib().ckr_op_cmul_to, a.h, float(c), int(target))

    def add_const(self, a, c):
        return self._unary(lib().ckr_op_add_const, a.h, float(c))

    def mul_plain(self, a, z):
        z = np.ascontiguousarray(z, np.float64)
        return self._unary(lib().ckr_op_mul_plain, a.h, _p(z, dblp), len(z))

    def synchronize(self):
        _ok(lib().ckr_synchronize(self.h))

    def set_profiling(self, on):
        _ok(lib().ckr_set_profiling(self.h, int(on)))

    def profile_reset(self):
        _ok(lib().ckr_profile_reset(self.h))

    def profile(self):
        """{category: (launches, total_ms, bytes)} since the last reset."""
        out = {}
        c = 0
        while True:
            name = lib().ckr_profile_name(c)
            if name is None:
                return out
            a, b, d = C.c_uint64(), C.c_double(), C.c_double()
            _ok(lib().ckr_profile_read(self.h, c, C.byref(a), C.byref(b), C.byref(d)))
            out[name.decode()] = (a.value, b.value, d.value)
            c += 1

    def ntt_device(self, ptr, limbs, first_mod, inverse):
        _ok(lib().ckr_ntt_device(self.h, vp(ptr), limbs, first_mod, int(inverse)))


class Keys:
    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def add_rotations(self, shifts):
        s = np.array(list(shifts), np.int64)
        _ok(lib().ckr_keys_add_rotations(self.ctx.h, self.h, _p(s, i64p), len(s)))

    def __del__(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            lib().ckr_keys_free(self.h)
            self.h = None


class Ct:
    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    @property
    def level(self):
        return int(lib().ckr_ct_level(self.h))

    @property
    def scale(self):
        return float(lib().ckr_ct_scale(self.h))

    def export(self):
        out = np.zeros((2, self.level + 1, self.ctx.n), np.uint64)
        _ok(lib().ckr_ct_export(self.ctx.h, self.h, _p(out, u64p), out.size))
        return out

    def __del__(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            lib().ckr_ct_free(self.h)
            self.h = None


KINDS = {"rank": 1, "argmin": 2, "sort": 3}


class Server:
    """Continuous-batching request server over one or more contexts (ckr_server_*)."""

    def __init__(self, hbm_budget=0, max_batch=8):
        h = vp()
        _ok(lib().ckr_server_create(hbm_budget, max_batch, C.byref(h)))
        self.h = h
        self.ctx_of = {}
        self._alive = {}

    def add_route(self, kind, N, ctx, keys, cmp, ind=(0, 0)):
        _ok(lib().ckr_server_add_route(self.h, KINDS[kind], N, ctx.h, keys.h, sign(cmp), sign(ind)))
        self.ctx_of[(kind, N)] = ctx
        self._routes = getattr(self, "_routes", [])
        self._routes.append((ctx, keys))     # the route's context and keys outlive the server

    def submit(self, kind, N, ct):
        t = C.c_uint64()
        _ok(lib().ckr_server_submit(self.h, KINDS[kind], N, ct.h, C.byref(t)))
        self._alive[t.value] = ct          # the input must outlive the request
        self._kind = getattr(self, "_kind", {})
        self._kind[t.value] = (kind, N)
        return t.value

    def wait(self, ticket, timeout_ms=-1):
        """(outputs, (latency_ms, queue_ms, batch))"""
        kind, N = self._kind[ticket]
        per = 2 if kind == "argmin" else 1
        outs = (vp * per)()
        lat = (C.c_double * 3)()
        st = lib().ckr_server_wait(self.h, ticket, timeout_ms, outs, per, lat)
        if st == -6:
            raise TimeoutError("ticket not finished")
        self._alive.pop(ticket, None)
        self._kind.pop(ticket, None)
        _ok(st)
        ctx = self.ctx_of[(kind, N)]
        return [Ct(ctx, vp(o)) for o in outs], (lat[0], lat[1], int(lat[2]))

    def stats(self):
        st = (C.c_double * 5)()
        _ok(lib().ckr_server_stats(self.h, st))
        return {"completed": int(st[0]), "batches": int(st[1]), "inflight_high_bytes": int(st[2]),
                "pending": int(st[3]), "overlap_high": int(st[4])}

    def close(self):
        if getattr(self, "h", None):
            lib().ckr_server_free(self.h)
            self.h = None

    def __del__(self):
        self.close()
