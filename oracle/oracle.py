"""ctypes view of the CPU oracle (oracle/ora.c) -- test infrastructure only.

Only tests/, the smoke check and bench.py's cpu_baseline leg use this module.
The product library never imports it.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ora.c")
_LIB = os.path.join(_HERE, "libora.so")

u64p = C.POINTER(C.c_uint64)
i64p = C.POINTER(C.c_int64)
dblp = C.POINTER(C.c_double)
u32p = C.POINTER(C.c_uint32)
intp = C.POINTER(C.c_int)

STATUS = {0: "ok", -1: "invalid", -2: "range", -3: "depth"}


def build(force=False):
    """Compile ora.c with gcc (plain C, OpenMP over limbs, binary128 encoder)."""
    if os.path.exists(_LIB) and not force:
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wno-unused-function", "-Wno-maybe-uninitialized", "-o", tmp, _SRC, "-lquadmath", "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


class OraCmp(C.Structure):
    """comparator: (d_g, d_f) of the f/g composite, cheb = D levels of the
    Chebyshev interpolant, or mm stages of the minimax composite"""
    _fields_ = [("dg", C.c_int), ("df", C.c_int), ("cheb", C.c_int), ("mm", C.c_int)]


def _cmp(spec):
    """(d_g, d_f), (0, 0, D) or (0, 0, 0, k) -> OraCmp"""
    spec = tuple(int(x) for x in spec) + (0, 0)
    return OraCmp(spec[0], spec[1], spec[2], spec[3])


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        sig = {
            "ora_params_new": (vp, [C.c_int] * 7),
            "ora_params_free": (None, [vp]),
            "ora_params_info": (None, [vp, u64p, dblp, u64p, intp]),
            "ora_set_threads": (None, [C.c_int]),
            "ora_negacyclic_mul": (None, [C.c_uint64, C.c_uint64, C.c_uint64, u64p, u64p, u64p]),
            "ora_ntt_forward": (None, [C.c_uint64, C.c_uint64, C.c_uint64, u64p]),
            "ora_chacha20_block": (None, [C.c_char_p, C.c_uint32, C.c_char_p, u32p]),
            "ora_sample": (None, [C.c_char_p, C.c_uint32, C.c_uint64, C.c_int, C.c_uint64, C.c_uint64, i64p]),
            "ora_encode": (C.c_int, [vp, dblp, C.c_uint32, C.c_double, i64p]),
            "ora_decode": (None, [vp, i64p, C.c_double, C.c_uint32, dblp]),
            "ora_automorphism": (None, [C.c_uint64, C.c_uint64, C.c_uint64, u64p, u64p]),
            "ora_bconv": (None, [u64p, u64p, C.c_int, C.c_uint64, C.c_uint64, u64p]),
            "ora_moddown": (None, [vp, C.c_int, u64p, u64p]),
            "ora_rescale_poly": (None, [vp, u64p, C.c_int, u64p]),
            "ora_keygen": (vp, [vp, C.c_char_p, C.c_int, u32p, C.c_int]),
            "ora_keys_free": (None, [vp]),
            "ora_keys_secret": (None, [vp, i64p]),
            "ora_encrypt": (vp, [vp, dblp, C.c_uint32, C.c_int, C.c_char_p, intp]),
            "ora_decrypt": (None, [vp, vp, dblp, C.c_uint32]),
            "ora_decrypt_coeffs": (None, [vp, vp, i64p]),
            "ora_ct_free": (None, [vp]),
            "ora_ct_level": (C.c_int, [vp]),
            "ora_ct_scale": (C.c_double, [vp]),
            "ora_ct_export": (None, [vp, u64p]),
            "ora_ct_import": (vp, [vp, C.c_int, u64p]),
            "ora_rescale": (vp, [vp]),
            "ora_drop": (vp, [vp, C.c_int]),
            "ora_add": (vp, [vp, vp]),
            "ora_sub": (vp, [vp, vp]),
            "ora_add_const": (vp, [vp, C.c_double]),
            "ora_cmul_to": (vp, [vp, C.c_double, C.c_int, intp]),
            "ora_mul_plain": (vp, [vp, dblp, C.c_uint32, intp]),
            "ora_add_plain": (vp, [vp, dblp, C.c_uint32, intp]),
            "ora_mul": (vp, [vp, vp, vp, intp]),
            "ora_apply_galois": (vp, [vp, vp, C.c_uint32, intp]),
            "ora_rotate": (vp, [vp, vp, C.c_int64, intp]),
            "ora_trans_r": (vp, [vp, vp, C.c_uint32, intp]),
            "ora_trans_c": (vp, [vp, vp, C.c_uint32, intp]),
            "ora_sum_r": (vp, [vp, vp, C.c_uint32, intp]),
            "ora_sum_c": (vp, [vp, vp, C.c_uint32, intp]),
            "ora_repl_r": (vp, [vp, vp, C.c_uint32, intp]),
            "ora_repl_c": (vp, [vp, vp, C.c_uint32, intp]),
            "ora_poly7": (vp, [vp, vp, dblp, intp]),
            "ora_cmp_sign": (vp, [vp, vp, OraCmp, intp]),
            "ora_cmp_matrix": (vp, [vp, vp, C.c_uint32, OraCmp, intp]),
            "ora_rank": (vp, [vp, vp, C.c_uint32, OraCmp, intp]),
            "ora_rank_depth": (C.c_int, [OraCmp]),
            "ora_rank_galois": (C.c_int, [vp, C.c_uint32, u32p]),
            "ora_galois_left": (C.c_uint32, [vp, C.c_uint64]),
            "ora_mul_int": (vp, [vp, C.c_int64]),
            "ora_argmin_depth": (C.c_int, [OraCmp, OraCmp]),
            "ora_argmin": (C.c_int, [vp, vp, C.c_uint32, OraCmp, OraCmp, C.POINTER(vp), C.POINTER(vp)]),
            "ora_rank_multi_depth": (C.c_int, [OraCmp]),
            "ora_rank_multi": (C.c_int, [vp, C.POINTER(vp), C.c_uint32, C.c_uint32, OraCmp, C.POINTER(vp)]),
            "ora_sort_multi_depth": (C.c_int, [OraCmp, OraCmp]),
            "ora_sort_multi": (C.c_int, [vp, C.POINTER(vp), C.c_uint32, C.c_uint32, OraCmp, OraCmp, C.POINTER(vp)]),
            "ora_rank_tie": (vp, [vp, vp, C.c_uint32, OraCmp, intp]),
            "ora_order_stat_depth": (C.c_int, [C.c_uint32, C.c_uint32, OraCmp, OraCmp, C.c_int]),
            "ora_order_stat": (C.c_int, [vp, vp, C.c_uint32, C.c_uint32, OraCmp, OraCmp, C.c_int, C.POINTER(vp),
                                         C.POINTER(vp)]),
            "ora_order_range_depth": (C.c_int, [C.c_uint32, C.c_uint32, C.c_uint32, OraCmp, OraCmp, C.c_int]),
            "ora_order_range": (C.c_int, [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, OraCmp, OraCmp, C.c_int,
                                          C.POINTER(vp), C.POINTER(vp)]),
            "ora_sort_depth": (C.c_int, [OraCmp, OraCmp]),
            "ora_sort": (vp, [vp, vp, C.c_uint32, OraCmp, OraCmp, intp]),
            "ora_circuit_galois": (C.c_int, [vp, C.c_uint32, C.c_int, u32p]),
            "ora_cheb_step_coeffs": (None, [C.c_int, dblp]),
            "ora_sort_col_depth": (C.c_int, [OraCmp, OraCmp]),
            "ora_rank_depth_n": (C.c_int, [C.c_uint32, OraCmp, C.c_int]),
            "ora_order_stat_div_depth": (C.c_int, [C.c_uint32, C.c_uint32, OraCmp, OraCmp, C.c_int]),
            "ora_order_stat_div": (C.c_int, [vp, vp, C.c_uint32, C.c_uint32, OraCmp, OraCmp, C.c_int, C.POINTER(vp),
                                             C.POINTER(vp)]),
            "ora_sort_col": (vp, [vp, vp, C.c_uint32, OraCmp, OraCmp, intp]),
            "ora_cheb_depth": (C.c_int, [C.c_uint32]),
            "ora_cheb_eval": (vp, [vp, vp, dblp, C.c_uint32, intp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def set_threads(t):
    lib().ora_set_threads(int(t))


class OracleError(RuntimeError):
    pass


def _check(ptr, st, what):
    if not ptr:
        raise OracleError(f"{what}: status {STATUS.get(st.value, st.value)}")
    return ptr


class Params:
    """Oracle parameter set: prime chain, special primes, per-level scales."""

    def __init__(self, logn, L, q0_bits, log_scale, K, p_bits, dnum):
        self.ptr = lib().ora_params_new(logn, L, q0_bits, log_scale, K, p_bits, dnum)
        if not self.ptr:
            raise OracleError("bad parameters")
        self.logn, self.L, self.K, self.dnum = logn, L, K, dnum
        self.n = 1 << logn
        nm = L + 1 + K
        self.mods = np.zeros(nm, np.uint64)
        self.psi = np.zeros(nm, np.uint64)
        self.scales = np.zeros(L + 1, np.float64)
        dims = np.zeros(5, np.int32)
        lib().ora_params_info(self.ptr, _p(self.mods, u64p), _p(self.scales, dblp), _p(self.psi, u64p),
                              _p(dims, intp))
        self.alpha = int(dims[4])
        self.q = [int(x) for x in self.mods[:L + 1]]
        self.p = [int(x) for x in self.mods[L + 1:]]

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().ora_params_free(self.ptr)
            self.ptr = None

    def galois_left(self, k):
        return int(lib().ora_galois_left(self.ptr, k))

    def circuit_galois(self, N, what):
        out = np.zeros(256, np.uint32)
        c = lib().ora_circuit_galois(self.ptr, N, what, _p(out, u32p))
        return [int(x) for x in out[:c]]

    def rank_galois(self, N):
        out = np.zeros(256, np.uint32)
        c = lib().ora_rank_galois(self.ptr, N, _p(out, u32p))
        return [int(x) for x in out[:c]]


class Keys:
    def __init__(self, params, seed, lmax, galois):
        self.params = params
        gal = np.array(list(galois), np.uint32)
        self.ptr = lib().ora_keygen(params.ptr, bytes(seed), lmax, _p(gal, u32p), len(gal))
        if not self.ptr:
            raise OracleError("keygen failed")
        self.lmax = lmax
        self.galois = set(int(g) for g in gal)

    def need(self, N, what):
        """raise unless the keys hold every rotation the circuits `what` on N need
        (the C circuits do not check for a missing key)"""
        missing = set(self.params.circuit_galois(N, what)) - self.galois
        if missing:
            raise OracleError(f"keys lack {len(missing)} rotation keys needed for N={N}")

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().ora_keys_free(self.ptr)
            self.ptr = None

    def secret(self):
        s = np.zeros(self.params.n, np.int64)
        lib().ora_keys_secret(self.ptr, _p(s, i64p))
        return s


class Ct:
    def __init__(self, ptr, params):
        self.ptr = ptr
        self.params = params

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().ora_ct_free(self.ptr)
            self.ptr = None

    @property
    def level(self):
        return lib().ora_ct_level(self.ptr)

    @property
    def scale(self):
        return lib().ora_ct_scale(self.ptr)

    def export(self):
        out = np.zeros((2, self.level + 1, self.params.n), np.uint64)
        lib().ora_ct_export(self.ptr, _p(out, u64p))
        return out

    @staticmethod
    def from_array(params, arr):
        arr = np.ascontiguousarray(arr, np.uint64)
        level = arr.shape[1] - 1
        return Ct(lib().ora_ct_import(params.ptr, level, _p(arr, u64p)), params)


def _ct(fn, params, *args, what="op"):
    st = C.c_int(0)
    ptr = fn(*args, C.byref(st))
    return Ct(_check(ptr, st, what), params)


def encrypt(keys, z, level, seed):
    z = np.ascontiguousarray(z, np.float64)
    return _ct(lib().ora_encrypt, keys.params, keys.ptr, _p(z, dblp), len(z), level, bytes(seed), what="encrypt")


def decrypt(keys, ct, count):
    out = np.zeros(count, np.float64)
    lib().ora_decrypt(keys.ptr, ct.ptr, _p(out, dblp), count)
    return out


def decrypt_coeffs(keys, ct):
    out = np.zeros(keys.params.n, np.int64)
    lib().ora_decrypt_coeffs(keys.ptr, ct.ptr, _p(out, i64p))
    return out


def encode(params, z, scale):
    z = np.ascontiguousarray(z, np.float64)
    m = np.zeros(params.n, np.int64)
    st = lib().ora_encode(params.ptr, _p(z, dblp), len(z), scale, _p(m, i64p))
    if st != 0:
        raise OracleError(f"encode: {STATUS.get(st, st)}")
    return m


def decode(params, m, scale, count):
    m = np.ascontiguousarray(m, np.int64)
    z = np.zeros(count, np.float64)
    lib().ora_decode(params.ptr, _p(m, i64p), scale, count, _p(z, dblp))
    return z


def rescale(ct):
    return Ct(lib().ora_rescale(ct.ptr), ct.params)


def drop(ct, level):
    return Ct(lib().ora_drop(ct.ptr, level), ct.params)


def add(a, b):
    return Ct(lib().ora_add(a.ptr, b.ptr), a.params)


def sub(a, b):
    return Ct(lib().ora_sub(a.ptr, b.ptr), a.params)


def add_const(a, c):
    return Ct(lib().ora_add_const(a.ptr, float(c)), a.params)


def cmul_to(a, c, target):
    return _ct(lib().ora_cmul_to, a.params, a.ptr, float(c), target, what="cmul_to")


def mul_plain(a, z):
    z = np.ascontiguousarray(z, np.float64)
    return _ct(lib().ora_mul_plain, a.params, a.ptr, _p(z, dblp), len(z), what="mul_plain")


def add_plain(a, z):
    z = np.ascontiguousarray(z, np.float64)
    return _ct(lib().ora_add_plain, a.params, a.ptr, _p(z, dblp), len(z), what="add_plain")


def mul(keys, a, b):
    return _ct(lib().ora_mul, a.params, keys.ptr, a.ptr, b.ptr, what="mul")


def apply_galois(keys, a, g):
    return _ct(lib().ora_apply_galois, a.params, keys.ptr, a.ptr, g, what="galois")


def rotate(keys, a, k):
    return _ct(lib().ora_rotate, a.params, keys.ptr, a.ptr, int(k), what="rotate")


def _mat(fn, keys, a, N):
    return _ct(fn, a.params, keys.ptr, a.ptr, N, what=fn.__name__)


def trans_r(keys, a, N): return _mat(lib().ora_trans_r, keys, a, N)
def trans_c(keys, a, N): return _mat(lib().ora_trans_c, keys, a, N)
def sum_r(keys, a, N): return _mat(lib().ora_sum_r, keys, a, N)
def sum_c(keys, a, N): return _mat(lib().ora_sum_c, keys, a, N)
def repl_r(keys, a, N): return _mat(lib().ora_repl_r, keys, a, N)
def repl_c(keys, a, N): return _mat(lib().ora_repl_c, keys, a, N)


def poly7(keys, a, coeffs):
    c = np.ascontiguousarray(coeffs, np.float64)
    return _ct(lib().ora_poly7, a.params, keys.ptr, a.ptr, _p(c, dblp), what="poly7")


# A comparator is given as (d_g, d_f) for the f/g composite or (0, 0, D) for
# the Chebyshev interpolant taking D levels; the functions taking "dg, df"
# accept the Chebyshev depth as a third argument.
def cmp_sign(keys, a, dg, df, cheb=0, mm=0):
    return _ct(lib().ora_cmp_sign, a.params, keys.ptr, a.ptr, _cmp((dg, df, cheb, mm)), what="cmp_sign")


def cmp_matrix(keys, a, N, dg, df, cheb=0, mm=0):
    return _ct(lib().ora_cmp_matrix, a.params, keys.ptr, a.ptr, N, _cmp((dg, df, cheb, mm)), what="cmp_matrix")


def rank(keys, a, N, dg, df, cheb=0, mm=0):
    keys.need(N, 1)
    return _ct(lib().ora_rank, a.params, keys.ptr, a.ptr, N, _cmp((dg, df, cheb, mm)), what="rank")


def rank_depth(dg, df, cheb=0, mm=0):
    return lib().ora_rank_depth(_cmp((dg, df, cheb, mm)))


def rank_multi_depth(dg, df, cheb=0, mm=0):
    return lib().ora_rank_multi_depth(_cmp((dg, df, cheb, mm)))


def cheb_step_coeffs(D):
    """the oracle's Chebyshev coefficients of the comparison function (2^(D-1) of them)"""
    c = np.zeros(1 << (D - 1))
    lib().ora_cheb_step_coeffs(D, _p(c, dblp))
    return c


def cheb_depth(deg1):
    return lib().ora_cheb_depth(deg1)


def cheb_eval(keys, a, coeffs):
    """sum_i coeffs[i] T_i(x) (len(coeffs) a power of two) by Paterson-Stockmeyer"""
    c = np.ascontiguousarray(coeffs, np.float64)
    return _ct(lib().ora_cheb_eval, a.params, keys.ptr, a.ptr, _p(c, dblp), len(c), what="cheb_eval")


def rank_multi(keys, blocks, b, dg, df, cheb=0, mm=0):
    """Multi-ciphertext ranking of len(blocks) blocks of b values; returns the L rank blocks."""
    keys.need(b, 4)
    L = len(blocks)
    arr = (C.c_void_p * L)(*[x.ptr for x in blocks])
    out = (C.c_void_p * L)()
    st = lib().ora_rank_multi(keys.ptr, arr, L, b, _cmp((dg, df, cheb, mm)), out)
    if st != 0:
        raise OracleError(f"rank_multi: status {STATUS.get(st, st)}")
    return [Ct(out[i], blocks[0].params) for i in range(L)]


def sort_multi_depth(cmp, ind):
    return lib().ora_sort_multi_depth(_cmp(cmp), _cmp(ind))


def sort_multi(keys, blocks, b, cmp, ind):
    """Multi-ciphertext sorting of len(blocks) blocks of b distinct values; returns the L sorted blocks."""
    keys.need(b, 4)
    L = len(blocks)
    arr = (C.c_void_p * L)(*[x.ptr for x in blocks])
    out = (C.c_void_p * L)()
    st = lib().ora_sort_multi(keys.ptr, arr, L, b, _cmp(cmp), _cmp(ind), out)
    if st != 0:
        raise OracleError(f"sort_multi: status {STATUS.get(st, st)}")
    return [Ct(out[i], blocks[0].params) for i in range(L)]


def rank_tie(keys, a, N, dg, df, cheb=0, mm=0):
    """tie-corrected rank (rank plus the tie-correction offset): a permutation of 1..N"""
    keys.need(N, 1)
    return _ct(lib().ora_rank_tie, a.params, keys.ptr, a.ptr, N, _cmp((dg, df, cheb, mm)), what="rank_tie")


# ---- primitive pins -------------------------------------------------------

def negacyclic_mul(n, q, psi, a, b):
    a = np.ascontiguousarray(a, np.uint64)
    b = np.ascontiguousarray(b, np.uint64)
    c = np.zeros(n, np.uint64)
    lib().ora_negacyclic_mul(n, q, psi, _p(a, u64p), _p(b, u64p), _p(c, u64p))
    return c


def ntt_forward(n, q, psi, a):
    a = np.array(a, np.uint64)
    lib().ora_ntt_forward(n, q, psi, _p(a, u64p))
    return a


def chacha20_block(key, counter, nonce):
    out = np.zeros(16, np.uint32)
    lib().ora_chacha20_block(bytes(key), counter, bytes(nonce), _p(out, u32p))
    return out


def sample(key, purpose, oid, kind, q, count):
    out = np.zeros(count, np.int64)
    lib().ora_sample(bytes(key), purpose, oid, kind, q, count, _p(out, i64p))
    return out


def automorphism(n, q, g, a):
    a = np.ascontiguousarray(a, np.uint64)
    b = np.zeros(n, np.uint64)
    lib().ora_automorphism(n, q, g, _p(a, u64p), _p(b, u64p))
    return b


def bconv(x, src, t):
    x = np.ascontiguousarray(x, np.uint64)
    src = np.ascontiguousarray(src, np.uint64)
    n = x.shape[1]
    out = np.zeros(n, np.uint64)
    lib().ora_bconv(_p(x, u64p), _p(src, u64p), len(src), t, n, _p(out, u64p))
    return out


def moddown(params, level, x):
    x = np.ascontiguousarray(x, np.uint64)
    out = np.zeros((level + 1, params.n), np.uint64)
    lib().ora_moddown(params.ptr, level, _p(x, u64p), _p(out, u64p))
    return out


def rescale_poly(params, x, level):
    x = np.ascontiguousarray(x, np.uint64)
    out = np.zeros((level, params.n), np.uint64)
    lib().ora_rescale_poly(params.ptr, _p(x, u64p), level, _p(out, u64p))
    return out


def mul_int(a, K):
    return Ct(lib().ora_mul_int(a.ptr, int(K)), a.params)


def argmin_depth(cmp, ind):
    return lib().ora_argmin_depth(_cmp(cmp), _cmp(ind))


def argmin(keys, a, N, cmp, ind):
    """(onehot, value) ciphertexts of the tie-corrected minimum."""
    keys.need(N, 2)
    oh, val = C.c_void_p(), C.c_void_p()
    st = lib().ora_argmin(keys.ptr, a.ptr, N, _cmp(cmp), _cmp(ind), C.byref(oh), C.byref(val))
    if st != 0:
        raise OracleError(f"argmin: status {STATUS.get(st, st)}")
    return Ct(oh.value, a.params), Ct(val.value, a.params)


def order_stat_depth(N, k, cmp, ind, tie):
    return lib().ora_order_stat_depth(N, k, _cmp(cmp), _cmp(ind), int(tie))


def order_stat(keys, a, N, k, cmp, ind, tie):
    """(onehot, value) ciphertexts of the k-th smallest element (tie-corrected if tie)."""
    keys.need(N, 2)
    oh, val = C.c_void_p(), C.c_void_p()
    st = lib().ora_order_stat(keys.ptr, a.ptr, N, k, _cmp(cmp), _cmp(ind), int(tie), C.byref(oh), C.byref(val))
    if st != 0:
        raise OracleError(f"order_stat: status {STATUS.get(st, st)}")
    return Ct(oh.value, a.params), Ct(val.value, a.params)


def order_range_depth(N, a, b, cmp, ind, tie):
    return lib().ora_order_range_depth(N, a, b, _cmp(cmp), _cmp(ind), int(tie))


def order_range(keys, ct, N, a, b, cmp, ind, tie):
    """(mask, value): the mask of the elements of rank a..b and the mean of
    the order statistics a..b (the median for a = N/2, b = N/2 + 1); N need
    not be a power of two when tie-corrected"""
    keys.need(N, 2)
    oh, val = C.c_void_p(), C.c_void_p()
    st = lib().ora_order_range(keys.ptr, ct.ptr, N, a, b, _cmp(cmp), _cmp(ind), int(tie), C.byref(oh), C.byref(val))
    if st != 0:
        raise OracleError(f"order_range: status {STATUS.get(st, st)}")
    return Ct(oh.value, ct.params), Ct(val.value, ct.params)


def sort_depth(cmp, ind):
    return lib().ora_sort_depth(_cmp(cmp), _cmp(ind))


def sort(keys, a, N, cmp, ind):
    keys.need(N, 4)
    return _ct(lib().ora_sort, a.params, keys.ptr, a.ptr, N, _cmp(cmp), _cmp(ind), what="sort")


def sort_col_depth(cmp, ind):
    return lib().ora_sort_col_depth(_cmp(cmp), _cmp(ind))


def sort_col(keys, a, N, cmp, ind):
    """column-form sorting: swapped comparator operands, SumC ranks, no final transposition"""
    keys.need(N, 2)
    return _ct(lib().ora_sort_col, a.params, keys.ptr, a.ptr, N, _cmp(cmp), _cmp(ind), what="sort_col")


def order_stat_div_depth(N, k, cmp, ind, iters):
    return lib().ora_order_stat_div_depth(N, k, _cmp(cmp), _cmp(ind), iters)


def order_stat_div(keys, a, N, k, cmp, ind, iters):
    """(mask, value): order statistic k without tie-correction, value = SumC(O V) / SumC(O) by Goldschmidt"""
    keys.need(N, 2)
    oh, val = C.c_void_p(), C.c_void_p()
    st = lib().ora_order_stat_div(keys.ptr, a.ptr, N, k, _cmp(cmp), _cmp(ind), iters, C.byref(oh), C.byref(val))
    if st != 0:
        raise OracleError(f"order_stat_div: status {STATUS.get(st, st)}")
    return Ct(oh.value, a.params), Ct(val.value, a.params)


def rank_depth_n(N, cmp, tie=False):
    """levels of rank (tie-corrected if tie) on N values, one more when N is not a power of two"""
    return lib().ora_rank_depth_n(N, _cmp(cmp), int(tie))
