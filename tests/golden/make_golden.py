"""Writes the stored expected values under tests/golden/ by running the
oracle only (never the HIP path).  Usage: python tests/golden/make_golden.py"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2412_15126_amd import workloads as W  # noqa: E402


def rank128_p16():
    N, level = 128, 17
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P16"])
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    K = O.Keys(P, kseed, level, P.rank_galois(N))
    ct = O.encrypt(K, v, level, eseed)
    R = O.rank(K, ct, N, *W.RANK_CMP[N])
    arr = R.export()
    dec = O.decrypt(K, R, N)
    return {"_what": "oracle rank of N=128 at n=2^16 (P16), workload seed 0, encryption level 17, "
                     "comparator g^4 then f: sha256 of the exported output ciphertext and its decoded ranks",
            "sha256": hashlib.sha256(arr.tobytes()).hexdigest(),
            "decoded": [float(x) for x in dec],
            "exact": [int(x) for x in np.argsort(np.argsort(v)) + 1]}


def rank128_p16_mm():
    """rank of N = 128 at n = 2^16 with four stages of the minimax composite
    (12 levels), encrypted at the circuit's depth"""
    N, cmp = 128, (0, 0, 0, 4)
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P16"])
    level = O.rank_depth(*cmp)
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    K = O.Keys(P, kseed, level, P.rank_galois(N))
    R = O.rank(K, O.encrypt(K, v, level, eseed), N, *cmp)
    dec = O.decrypt(K, R, N)
    return {"_what": "oracle rank of N=128 at n=2^16 (P16), workload seed 0 (gap 2^-10), encryption level 14, "
                     "comparator: four stages of the minimax composite: sha256 of the exported output and its "
                     "decoded ranks",
            "level": level,
            "sha256": hashlib.sha256(R.export().tobytes()).hexdigest(),
            "decoded": [float(x) for x in dec],
            "exact": [int(x) for x in np.argsort(np.argsort(v)) + 1]}


def argmin128_p17o():
    N = 128
    cmp, ind = W.ARGMIN_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P17O"])
    level = O.argmin_depth(cmp, ind)
    v, kseed, eseed = W.tied_workload(N, 0)
    K = O.Keys(P, kseed, level, P.circuit_galois(N, 2))
    ct = O.encrypt(K, v, level, eseed)
    oh, val = O.argmin(K, ct, N, cmp, ind)
    a, b = oh.export(), val.export()
    return {"_what": "oracle tie-corrected argmin of N=128 at n=2^17 (P17O), tied workload seed 0 (96 distinct "
                     "values + 32 duplicates), encryption level 43 (the circuit's depth), comparator g^4 f^2, "
                     "indicator g^4 f^2: sha256 of the exported one-hot and value ciphertexts and their decoded slots",
            "level": level,
            "sha256_onehot": hashlib.sha256(a.tobytes()).hexdigest(),
            "sha256_value": hashlib.sha256(b.tobytes()).hexdigest(),
            "onehot": [float(x) for x in O.decrypt(K, oh, N)],
            "value": float(O.decrypt(K, val, 1)[0]),
            "argmin": int(np.argmin(v)), "min": float(v.min())}


def sort128_p17():
    N = 128
    cmp, ind = W.SORT_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P17"])
    level = P.L
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    K = O.Keys(P, kseed, level, P.circuit_galois(N, 4))
    ct = O.encrypt(K, v, level, eseed)
    S = O.sort(K, ct, N, cmp, ind)
    a = S.export()
    return {"_what": "oracle sort of N=128 at n=2^17 (P17), workload seed 0, encryption level 40, comparator g^4 f, "
                     "indicator g^4 f^2: sha256 of the exported output ciphertext and its decoded slots",
            "sha256": hashlib.sha256(a.tobytes()).hexdigest(),
            "decoded": [float(x) for x in O.decrypt(K, S, N)],
            "sorted": [float(x) for x in np.sort(v)]}


def mixed_p16d():
    """two queries of the mixed batch (seed 7): the first rank and the first
    argmin (order statistic k = 1, no tie-correction) of N = 128, each
    encrypted at the level its circuit needs, keys at the top level"""
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P16D"])
    kseed, qs = W.mixed_workload(7, 64)
    N = 128
    ir = next(i for i, q in enumerate(qs) if q["kind"] == "rank" and q["N"] == N)
    ia = next(i for i, q in enumerate(qs) if q["kind"] == "argmin" and q["N"] == N)
    gal = sorted(set(P.circuit_galois(N, 2)) | set(P.rank_galois(N)))
    K = O.Keys(P, kseed, P.L, gal)
    rc = W.RANK_CMP[N]
    ac, ai = W.ORDER_CMP[N]
    lr, la = O.rank_depth(*rc), O.order_stat_depth(N, 1, ac, ai, False)
    q = qs[ir]
    R = O.rank(K, O.encrypt(K, q["v"], lr, q["eseed"]), N, *rc)
    out = {"_what": "oracle results of two queries of the mixed rank/argmin batch (mixed_workload seed 7, 64 "
                    "queries) at n=2^16 (P16D, keys at level 36): the first rank query of N=128 (encrypted at "
                    "level 17, comparator g^4 f) and the first argmin query of N=128 (order statistic k=1 without "
                    "tie-correction, encrypted at level 36, comparator g^4 f, indicator g^4 f^2): sha256 of the "
                    "exported ciphertexts and decoded slots",
           "rank_index": ir, "rank_level": lr, "rank_sha256": hashlib.sha256(R.export().tobytes()).hexdigest(),
           "rank_decoded": [float(x) for x in O.decrypt(K, R, N)],
           "rank_exact": [int(x) for x in np.argsort(np.argsort(q["v"])) + 1]}
    q = qs[ia]
    oh, val = O.order_stat(K, O.encrypt(K, q["v"], la, q["eseed"]), N, 1, ac, ai, False)
    out.update({"argmin_index": ia, "argmin_level": la,
                "argmin_sha256_onehot": hashlib.sha256(oh.export().tobytes()).hexdigest(),
                "argmin_sha256_value": hashlib.sha256(val.export().tobytes()).hexdigest(),
                "argmin_onehot": [float(x) for x in O.decrypt(K, oh, N)],
                "argmin_value": float(O.decrypt(K, val, 1)[0]),
                "argmin": int(np.argmin(q["v"])), "min": float(q["v"].min())})
    return out


def argmax128_p17o():
    N, k = 128, 128
    cmp, ind = W.ORDER_TIE_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P17O"])
    level = P.L
    v, kseed, eseed = W.tied_workload(N, 0)
    K = O.Keys(P, kseed, level, P.circuit_galois(N, 2))
    ct = O.encrypt(K, v, level, eseed)
    oh, val = O.order_stat(K, ct, N, k, cmp, ind, True)
    top = int(np.flatnonzero(v == v.max())[-1])
    return {"_what": "oracle tie-corrected argmax (order statistic k=N) of N=128 at n=2^17 (P17O), tied workload "
                     "seed 0 (96 distinct values + 32 duplicates), encryption level 44, comparator g^4 f^2, indicator "
                     "g^4 f^2: sha256 of the exported one-hot and value ciphertexts and their decoded slots",
            "sha256_onehot": hashlib.sha256(oh.export().tobytes()).hexdigest(),
            "sha256_value": hashlib.sha256(val.export().tobytes()).hexdigest(),
            "onehot": [float(x) for x in O.decrypt(K, oh, N)],
            "value": float(O.decrypt(K, val, 1)[0]),
            "argmax": top, "max": float(v.max())}


def rank512_p16_multi():
    """multi-ciphertext ranking of N = 512 values in 4 blocks of 128 at n = 2^16"""
    N, b = 512, 128
    cmp = W.MULTI_RANK_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P16"])
    level = O.rank_multi_depth(*cmp)
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    K = O.Keys(P, kseed, level, P.circuit_galois(b, 4))
    blocks = [O.encrypt(K, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    R = O.rank_multi(K, blocks, b, *cmp)
    dec = np.concatenate([O.decrypt(K, r, b) for r in R])
    return {"_what": "oracle multi-ciphertext ranking (section 5) of N=512 values (workload seed 0, gap 2^-10) in 4 "
                     "blocks of 128 at n=2^16 (P16), blocks encrypted at level 21 with seeds (i, eseed[1:]), "
                     "comparator g^4 f^2: sha256 of each exported rank block and the decoded ranks",
            "level": level,
            "sha256": [hashlib.sha256(r.export().tobytes()).hexdigest() for r in R],
            "decoded": [float(x) for x in dec],
            "exact": [int(x) for x in np.argsort(np.argsort(v)) + 1]}


def rank2048_p16d_multi():
    """multi-ciphertext ranking of N = 2048 values in 16 blocks of 128 at n = 2^16 (136 block pairs)"""
    N, b = 2048, 128
    cmp = W.MULTI_RANK_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P16D"])
    level = O.rank_multi_depth(*cmp)
    v, kseed, eseed = W.rank_workload(N, W.MULTI_GAP[N], 0)
    K = O.Keys(P, kseed, level, P.circuit_galois(b, 4))
    blocks = [O.encrypt(K, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    R = O.rank_multi(K, blocks, b, *cmp)
    dec = np.concatenate([O.decrypt(K, r, b) for r in R])
    return {"_what": "oracle multi-ciphertext ranking (section 5) of N=2048 values (workload seed 0, gap 2^-12) in 16 "
                     "blocks of 128 at n=2^16 (P16D), blocks encrypted at level 24 with seeds (i, eseed[1:]), "
                     "comparator g^5 f^2: sha256 of each exported rank block and the decoded ranks",
            "level": level,
            "sha256": [hashlib.sha256(r.export().tobytes()).hexdigest() for r in R],
            "decoded": [float(x) for x in dec],
            "exact": [int(x) for x in np.argsort(np.argsort(v)) + 1]}


def sort512_p17s_multi():
    """multi-ciphertext sorting of N = 512 values in 2 blocks of 256 at n = 2^17"""
    N, b = 512, 256
    cmp, ind = W.MULTI_SORT_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P17S"])
    level = O.sort_multi_depth(cmp, ind)
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    K = O.Keys(P, kseed, level, P.circuit_galois(b, 4))
    blocks = [O.encrypt(K, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    out = O.sort_multi(K, blocks, b, cmp, ind)
    dec = np.concatenate([O.decrypt(K, o, b) for o in out])
    return {"_what": "oracle multi-ciphertext sorting (section 5) of N=512 values (workload seed 0, gap 2^-10) in 2 "
                     "blocks of 256 at n=2^17 (P17S), blocks encrypted at level 47 with seeds (i, eseed[1:]), "
                     "comparator g^4 f^2, indicator g^5 f^2: sha256 of each exported sorted block and the decoded "
                     "values",
            "level": level,
            "sha256": [hashlib.sha256(o.export().tobytes()).hexdigest() for o in out],
            "decoded": [float(x) for x in dec],
            "sorted": [float(x) for x in np.sort(v)]}


def sort1024_p17s_multi():
    """multi-ciphertext sorting of N = 1024 values in 4 blocks of 256 at n = 2^17"""
    N, b = 1024, 256
    cmp, ind = W.MULTI_SORT_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P17S"])
    level = O.sort_multi_depth(cmp, ind)
    v, kseed, eseed = W.rank_workload(N, W.MULTI_GAP[N], 0)
    K = O.Keys(P, kseed, level, P.circuit_galois(b, 4))
    blocks = [O.encrypt(K, v[i * b:(i + 1) * b], level, bytes([i]) + eseed[1:]) for i in range(N // b)]
    out = O.sort_multi(K, blocks, b, cmp, ind)
    dec = np.concatenate([O.decrypt(K, o, b) for o in out])
    return {"_what": "oracle multi-ciphertext sorting (section 5) of N=1024 values (workload seed 0, gap 2^-11) in 4 "
                     "blocks of 256 at n=2^17 (P17S), blocks encrypted at level 47 with seeds (i, eseed[1:]), "
                     "comparator g^4 f^2, indicator g^5 f^2: sha256 of each exported sorted block and the decoded "
                     "values",
            "level": level,
            "sha256": [hashlib.sha256(o.export().tobytes()).hexdigest() for o in out],
            "decoded": [float(x) for x in dec],
            "sorted": [float(x) for x in np.sort(v)]}


def rank128_p16_cheb():
    """rank of N = 128 at n = 2^16 with the Chebyshev comparator of 12 levels"""
    N = 128
    cmp = W.CHEB_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P16"])
    level = O.rank_depth(*cmp)
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    K = O.Keys(P, kseed, level, P.rank_galois(N))
    R = O.rank(K, O.encrypt(K, v, level, eseed), N, *cmp)
    return {"_what": "oracle rank of N=128 at n=2^16 (P16), workload seed 0, encryption level 14, Chebyshev "
                     "comparator of degree 2^11 - 1 (12 levels): sha256 of the exported output ciphertext and its "
                     "decoded ranks",
            "level": level,
            "sha256": hashlib.sha256(R.export().tobytes()).hexdigest(),
            "decoded": [float(x) for x in O.decrypt(K, R, N)],
            "exact": [int(x) for x in np.argsort(np.argsort(v)) + 1]}


def argmin128_p17_cheb():
    """tie-corrected argmin of N = 128 at n = 2^17, Chebyshev comparator and indicator of 12 levels each"""
    N = 128
    cmp = ind = W.CHEB_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P17"])
    level = O.order_stat_depth(N, 1, cmp, ind, True)
    v, kseed, eseed = W.tied_workload(N, 0)
    K = O.Keys(P, kseed, level, P.circuit_galois(N, 2))
    oh, val = O.order_stat(K, O.encrypt(K, v, level, eseed), N, 1, cmp, ind, True)
    return {"_what": "oracle tie-corrected argmin of N=128 (tied workload seed 0) at n=2^17 (P17), encryption level "
                     "31, Chebyshev comparator and indicator of degree 2^11 - 1: sha256 of the exported one-hot and "
                     "value ciphertexts and their decoded contents",
            "level": level,
            "sha256": [hashlib.sha256(oh.export().tobytes()).hexdigest(),
                       hashlib.sha256(val.export().tobytes()).hexdigest()],
            "onehot": [float(x) for x in O.decrypt(K, oh, N)],
            "value": float(O.decrypt(K, val, 1)[0]),
            "argmin": int(np.argsort(v, kind="stable")[0]), "min": float(v.min())}


def sort128_p17_col():
    """column-form sort of N = 128 at n = 2^17"""
    N = 128
    cmp, ind = W.SORT_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P17"])
    level = O.sort_col_depth(cmp, ind)
    v, kseed, eseed = W.rank_workload(N, 2.0 ** -10, 0)
    K = O.Keys(P, kseed, level, P.circuit_galois(N, 2))
    S = O.sort_col(K, O.encrypt(K, v, level, eseed), N, cmp, ind)
    return {"_what": "oracle column-form sort of N=128 (workload seed 0, gap 2^-10) at n=2^17 (P17), encryption "
                     "level 39, comparator g^4 f, indicator g^4 f^2: sha256 of the exported output and its decoded "
                     "values",
            "level": level,
            "sha256": hashlib.sha256(S.export().tobytes()).hexdigest(),
            "decoded": [float(x) for x in O.decrypt(K, S, N)],
            "sorted": [float(x) for x in np.sort(v)]}


def kth64_p17s_div():
    """order statistic with the value by division, N = 64 with four tripled values, at n = 2^17"""
    N, iters = 64, 8
    cmp, ind = W.ORDER_CMP[N]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS["P17S"])
    v, kseed, eseed = W.tripled_workload(N, 0, triples=4)
    u, c = np.unique(v, return_counts=True)
    t = float(u[c == 3].min())
    k = int(np.sum(v < t)) + 2
    level = O.order_stat_div_depth(N, k, cmp, ind, iters)
    K = O.Keys(P, kseed, level, P.circuit_galois(N, 2))
    oh, val = O.order_stat_div(K, O.encrypt(K, v, level, eseed), N, k, cmp, ind, iters)
    return {"_what": "oracle order statistic with the value by division (Goldschmidt, 8 steps) of N=64 values with "
                     "four tripled ones (tripled workload seed 0, gap 2^-10) at n=2^17 (P17S), k = the rank of the "
                     "smallest tripled value, comparator g^4 f, indicator g^4 f^2: sha256 of the exported mask and "
                     "value ciphertexts and their decoded contents",
            "level": level, "k": k, "iters": iters, "value_expected": t,
            "sha256": [hashlib.sha256(oh.export().tobytes()).hexdigest(),
                       hashlib.sha256(val.export().tobytes()).hexdigest()],
            "mask": [float(x) for x in O.decrypt(K, oh, N)],
            "value": float(O.decrypt(K, val, 1)[0])}


def _median_case(N, pset, seed):
    cmp, ind = W.ORDER_TIE_CMP[128]
    O.set_threads(min(16, os.cpu_count() or 1))
    P = O.Params(**W.PSETS[pset])
    a, b = (N // 2, N // 2 + 1) if N % 2 == 0 else ((N + 1) // 2, (N + 1) // 2)
    v, kseed, eseed = W.tied_workload(N, seed)
    level = O.order_range_depth(N, a, b, cmp, ind, True)
    K = O.Keys(P, kseed, level, P.circuit_galois(N, 2))
    oh, val = O.order_range(K, O.encrypt(K, v, level, eseed), N, a, b, cmp, ind, True)
    return {"level": level, "window": [a, b], "median": float(np.median(v)),
            "sha256": [hashlib.sha256(oh.export().tobytes()).hexdigest(),
                       hashlib.sha256(val.export().tobytes()).hexdigest()],
            "mask": [float(x) for x in O.decrypt(K, oh, N)],
            "value": float(O.decrypt(K, val, 1)[0])}


def median128_p17o():
    """tie-corrected median of N = 128 (window [64, 65]) at n = 2^17"""
    d = _median_case(128, "P17O", 3)
    d["_what"] = ("oracle tie-corrected median (rank window [64, 65], the mean of the two middle statistics) of "
                  "N=128 at n=2^17 (P17O), tied workload seed 3 (96 distinct values + 32 duplicates), comparator "
                  "and indicator g^4 f^2, encryption at the circuit's depth: sha256 of the exported mask and value "
                  "ciphertexts and their decoded contents")
    return d


def median101_p17s():
    """tie-corrected median of N = 101 values (rank 51), padded to the 128 layout, at n = 2^17"""
    d = _median_case(101, "P17S", 4)
    d["_what"] = ("oracle tie-corrected median (rank window [51, 51]) of N=101 values zero-padded to the 128 "
                  "layout at n=2^17 (P17S), tied workload seed 4 (76 distinct values + 25 duplicates), comparator "
                  "and indicator g^4 f^2, encryption at the circuit's depth: sha256 of the exported mask and value "
                  "ciphertexts and their decoded contents")
    return d


if __name__ == "__main__":
    which = sys.argv[1:] or ["rank128_p16", "argmin128_p17o", "sort128_p17", "mixed_p16d", "argmax128_p17o",
                             "rank512_p16_multi", "sort512_p17s_multi", "rank128_p16_cheb",
                             "argmin128_p17_cheb", "sort128_p17_col", "kth64_p17s_div", "median128_p17o",
                             "median101_p17s", "rank128_p16_mm", "rank2048_p16d_multi",
                             "sort1024_p17s_multi"]
    for name in which:
        json.dump(globals()[name](), open(os.path.join(HERE, name + ".json"), "w"), indent=1)
        print("wrote", name + ".json", flush=True)
