"""Seeded synthetic inputs and parameter-set descriptions.

This module holds no arithmetic of the method: it only draws input vectors,
seeds and names the parameter sets (ring size, prime sizes, digit count).
Both the HIP path and the CPU oracle are fed from here.

Input recipe (the paper draws values uniformly at random in a bounded
interval, section 6.1 "Experimental Setup"):
  * min_gap_uniform: N values in [0, 1) whose pairwise gap is at least `gap`,
    drawn exactly uniformly on that constrained set by sort-and-spread
    (u ~ U[0, 1 - (N-1) gap)^N, sort, add i*gap to the i-th smallest,
    shuffle).
  * tied_pool: `pool` distinct values (min_gap_uniform) plus N - pool draws
    with replacement from the pool, shuffled (25 % duplicates at N=128).
  * seeds: 32-byte key / encryption seeds from numpy's default_rng.
"""
import numpy as np

# Parameter sets.  logn: ring degree 2^logn; L: top level (q_0..q_L);
# q0_bits: size class of q_0; log_scale: log2 of the top-level scale (the
# rescale primes are picked near the running scale); K special primes of
# p_bits; dnum key-switching digits.
PSETS = {
    # toy ring for the N=8 rank (not secure)
    "P12": dict(logn=12, L=11, q0_bits=44, log_scale=36, K=4, p_bits=40, dnum=3),
    # rank on N = 128 at n = 2^15 with the Chebyshev comparator up to 11 levels
    # (13 levels, log QP ~ 820 bits)
    "P15": dict(logn=15, L=13, q0_bits=50, log_scale=40, K=5, p_bits=50, dnum=3),
    # rank on N <= 128 at n = 2^16 (log QP ~ 1320 bits)
    "P16": dict(logn=16, L=23, q0_bits=50, log_scale=40, K=7, p_bits=50, dnum=3),
    # tie-corrected argmin and sort on N <= 128 at n = 2^17 (40 levels, log QP ~ 2150 bits)
    "P17": dict(logn=17, L=40, q0_bits=50, log_scale=40, K=10, p_bits=50, dnum=4),
    # mixed rank / order-statistic batches at n = 2^16, each query encrypted at
    # the level its circuit needs (36 levels, log QP ~ 1740 bits)
    "P16D": dict(logn=16, L=36, q0_bits=50, log_scale=40, K=5, p_bits=50, dnum=8),
    # tie-corrected order statistics for any k on N <= 128 at n = 2^17
    # (44 levels, log QP ~ 2360 bits)
    "P17O": dict(logn=17, L=44, q0_bits=50, log_scale=40, K=11, p_bits=50, dnum=4),
    # multi-ciphertext sort of N = 512 in blocks of 256 at n = 2^17 (47 levels, log QP ~ 2530 bits)
    "P17S": dict(logn=17, L=47, q0_bits=50, log_scale=40, K=12, p_bits=50, dnum=4),
    # small rings used by the unit and parity tests
    "T12D": dict(logn=12, L=34, q0_bits=44, log_scale=36, K=9, p_bits=40, dnum=4),
    "T10": dict(logn=10, L=7, q0_bits=44, log_scale=36, K=3, p_bits=46, dnum=3),
    "T12E": dict(logn=12, L=46, q0_bits=44, log_scale=36, K=12, p_bits=40, dnum=4),
    "T13": dict(logn=13, L=11, q0_bits=44, log_scale=36, K=4, p_bits=40, dnum=3),
}

# Comparator compositions (d_g, d_f) per workload: g applied d_g times, then f d_f times.
RANK_CMP = {8: (2, 1), 16: (3, 1), 32: (3, 1), 64: (4, 1), 128: (4, 1)}
# rank of N = 128 at the 2^-10 gap with the degree-7 polynomial composed 4
# times: four stages of the minimax composite (0, 0, 0, 4) rank exactly, where
# every four-fold f/g split fails (g^4 f above takes five)
RANK128_MM = (0, 0, 0, 4)
# tie-corrected argmin: (comparator, one-sided indicator).  At N = 128 the
# indicator g^3 f^2 leaks up to 4.6e-2 of the second-smallest value into the
# minimum's value (its output at rank distance 1/2 over N); g^4 f^2 bounds the
# leakage of all 127 others together by 4.3e-6 (43 levels: n = 2^17, P17O)
ARGMIN_CMP = {8: ((3, 1), (2, 1)), 16: ((4, 1), (3, 2)), 32: ((4, 2), (3, 2)), 64: ((4, 2), (3, 2)),
              128: ((4, 2), (4, 2))}
# order statistic k without tie-correction (distinct values), any k:
# (comparator, indicator: one-sided for k = 1 and k = N, a window otherwise)
ORDER_CMP = {8: ((3, 1), (2, 2)), 16: ((4, 1), (3, 2)), 32: ((4, 1), (3, 2)), 64: ((4, 1), (4, 2)),
             128: ((4, 1), (4, 2))}
# tie-corrected order statistic for k > 1 (k = 1 uses ARGMIN_CMP)
ORDER_TIE_CMP = {8: ((3, 1), (2, 2)), 128: ((4, 2), (4, 2))}
# Chebyshev comparator (0, 0, D): the interpolant of the comparison function
# taking D levels (degree 2^(D-1) - 1), the paper's choice for rank and minimum
# at N <= 256 (up to degree 2^11, i.e. D = 12); per N, the depth whose ranks
# round exactly at the workload's minimum gap
CHEB_CMP = {8: (0, 0, 8), 128: (0, 0, 12)}
# multi-ciphertext rank (blocks of b values, N = L b): comparator per total N
MULTI_RANK_CMP = {64: (4, 1), 128: (4, 1), 256: (4, 2), 512: (4, 2), 1024: (4, 2), 2048: (5, 2), 4096: (5, 2),
                  8192: (6, 2), 16384: (6, 2)}
# the gap of the min-gap workload per total N: (N - 1) gap < 1
MULTI_GAP = {64: 2.0 ** -10, 128: 2.0 ** -10, 256: 2.0 ** -10, 512: 2.0 ** -10, 1024: 2.0 ** -11,
             2048: 2.0 ** -12, 4096: 2.0 ** -13, 8192: 2.0 ** -14, 16384: 2.0 ** -15}
# multi-ciphertext sort: (comparator, two-sided indicator) per total N
MULTI_SORT_CMP = {64: ((4, 2), (4, 2)), 128: ((4, 2), (4, 2)), 512: ((4, 2), (5, 2)), 1024: ((4, 2), (5, 2))}
# sort: (comparator, two-sided indicator)
SORT_CMP = {8: ((3, 1), (3, 2)), 16: ((4, 1), (3, 2)), 32: ((4, 1), (3, 2)), 64: ((4, 1), (4, 2)),
            128: ((4, 1), (4, 2))}


def min_gap_uniform(N, gap, rng):
    if (N - 1) * gap >= 1.0:
        raise ValueError("gap too large for N values in [0,1)")
    u = np.sort(rng.uniform(0.0, 1.0 - (N - 1) * gap, N))
    v = u + gap * np.arange(N)
    rng.shuffle(v)
    return v


def tied_pool(N, pool, gap, rng):
    base = min_gap_uniform(pool, gap, rng)
    extra = rng.choice(base, size=N - pool, replace=True)
    v = np.concatenate([base, extra])
    rng.shuffle(v)
    return v


def seed_bytes(rng):
    return bytes(rng.integers(0, 256, 32, dtype=np.uint8).tolist())


def tied_workload(N, seed, gap=2.0 ** -10):
    """(values, key seed, encryption seed) with 25 % duplicated values."""
    rng = np.random.default_rng(seed)
    v = tied_pool(N, N - N // 4, gap, rng)
    return v, seed_bytes(rng), seed_bytes(rng)


def tripled_workload(N, seed, triples=1, gap=2.0 ** -10):
    """(values, key seed, encryption seed): N - 2 triples distinct values (min gap), `triples` of them
    appearing three times, shuffled; a tripled value's fractional rank is an integer shared by three
    elements."""
    rng = np.random.default_rng(seed)
    base = min_gap_uniform(N - 2 * triples, gap, rng)
    v = np.concatenate([base, np.repeat(base[:triples], 2)])
    rng.shuffle(v)
    return v, seed_bytes(rng), seed_bytes(rng)


def rank_workload(N, gap, seed):
    """(values, key seed, encryption seed) of one seeded rank query."""
    rng = np.random.default_rng(seed)
    v = min_gap_uniform(N, gap, rng)
    return v, seed_bytes(rng), seed_bytes(rng)


def mixed_workload(seed=7, count=64, Ns=(16, 32, 64, 128)):
    """A batch of independent queries: kind "rank" or "argmin" with equal
    odds, N drawn uniformly from Ns, values min-gap uniform (gap 2^-10).
    Returns (key seed, [dict(kind, N, v, eseed)])."""
    rng = np.random.default_rng(seed)
    kseed = seed_bytes(rng)
    qs = []
    for _ in range(count):
        kind = "rank" if rng.random() < 0.5 else "argmin"
        N = int(rng.choice(Ns))
        v = min_gap_uniform(N, 2.0 ** -10, rng)
        qs.append(dict(kind=kind, N=N, v=v, eseed=seed_bytes(rng)))
    return kseed, qs
