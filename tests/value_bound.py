"""Error bound of an order statistic's value output (test infrastructure).

Algorithm Order Statistic (section 3.2) returns value = SumC(O * V): the
inner product of the indicator mask O with the input vector, which a window
of ranks [a, b] (section 4's median) divides by b - a + 1.  With ideal
indicators this is the mean of the order statistics a..b exactly; with the
approximate comparator the decoded value differs from it by

  |value - mean| <= ( sum_{j selected}   |1 - O_j| |v_j|
                    + sum_{j unselected} |O_j|     |v_j| ) / (b - a + 1)
                    + (CKKS noise of the N products) / (b - a + 1).

Each O_j is the indicator composition evaluated at the distance of the
element's rank k_j from the window's threshold(s), divided by N:
  - one-sided, a = 1:  O = Cmp(b + 1/2, k_j);
  - one-sided, b = N:  O = Cmp(k_j, a - 1/2);
  - two-sided:         O = Cmp(k_j, a - 1/2) (1 - Cmp(k_j, b + 1/2)).
k_j lies within delta of the element's integer rank r_j (the comparator's rank
error; tie-corrected ranks are a permutation of 1..N, equal values in index
order), so an element whose rank is r_j sits at least |r_j - t| - delta from
threshold t.  The indicator's leakage at distance x is

  L(x) = sup_{x <= y <= 1} max(|Cmp(-y)|, |1 - Cmp(y)|)      (per unit N),

taken over the whole tail because the composites are not monotone near 1.
A two-sided window's other factor is at most M = sup |Cmp| or sup |1 - Cmp|
on [-1, 1].  The CKKS term is bounded by eta * sum_j |v_j| for a per-slot noise bound eta
of the mask (checked on the decoded mask where the tests have it).
"""
import numpy as np

from oracle import shadow as S

_G = 1 << 18          # grid points on [0, 1]
_tabs = {}
# per-slot CKKS noise allowance of the mask and of the product/rotation steps
# after it: the decoded masks of the full-size circuits (n = 2^17, 43-44
# levels) deviate from their noiseless value by at most ~8e-7 per slot, and the
# SumC rotations with the exact ModDown add ~1e-8 each
ETA = 2e-6


def _cmp_vals(ind, x):
    """the indicator's Cmp on argument x (the shadow's comparator)"""
    return S.cmp_of(np.asarray(x, dtype=np.float64), tuple(ind))


def _table(ind):
    key = tuple(ind)
    if key not in _tabs:
        y = np.linspace(0.0, 1.0, _G + 1)
        e = np.maximum(np.abs(_cmp_vals(key, -y)), np.abs(1.0 - _cmp_vals(key, y)))
        sup_tail = np.maximum.accumulate(e[::-1])[::-1]
        full = np.linspace(-1.0, 1.0, 2 * _G + 1)
        c = _cmp_vals(key, full)
        M = float(max(np.max(np.abs(c)), np.max(np.abs(1.0 - c))))
        _tabs[key] = (sup_tail, M)
    return _tabs[key]


def leak(ind, x):
    """L(x): the largest deviation of the indicator from its ideal value at
    any argument of magnitude >= x (x <= 0 gives the worst over [0, 1])"""
    tab, _ = _table(ind)
    i = int(np.floor(min(max(x, 0.0), 1.0) * _G))   # floor: the supremum over a superset
    return float(tab[i])


def other_factor(ind):
    return _table(ind)[1]


def ranks_of(v):
    """tie-corrected ranks 1..N: equal values take consecutive ranks, lowest
    index first (section 4's offset)"""
    order = np.argsort(np.asarray(v), kind="stable")
    r = np.empty(len(v), dtype=np.int64)
    r[order] = np.arange(1, len(v) + 1)
    return r


def mask_bound(v, a, b, ind, delta):
    """per-element bound on |O_j - ideal_j| before noise (ideal: 1 for ranks
    in [a, b], 0 elsewhere), the indicator arguments divided by N = len(v)"""
    v = np.asarray(v, dtype=np.float64)
    N = len(v)
    r = ranks_of(v)
    lower, upper = a == 1, b == N
    M = other_factor(ind)
    L = lambda d: leak(ind, (d - delta) / N)  # noqa: E731
    out = np.empty(N)
    for j in range(N):
        rj = r[j]
        if lower:
            out[j] = L(abs(b + 0.5 - rj))
        elif upper:
            out[j] = L(abs(rj - (a - 0.5)))
        elif rj < a:
            out[j] = L(a - 0.5 - rj) * M
        elif rj > b:
            out[j] = M * L(rj - b - 0.5)
        else:
            out[j] = L(rj - (a - 0.5)) + M * L(b + 0.5 - rj)
    return out


def value_bound(v, a, b, ind, delta, eta):
    """Bound on |decoded value - mean of the order statistics a..b| of the
    values v: the mask deviations plus eta, weighted by |v_j|, over
    b - a + 1"""
    v = np.asarray(v, dtype=np.float64)
    return float(np.dot(mask_bound(v, a, b, ind, delta) + eta, np.abs(v))) / (b - a + 1)


def tolerance(v, a, b, cmp, ind, tie, logn):
    """value_bound with delta from the comparator's rank error on v (ring 2^logn)"""
    return value_bound(v, a, b, ind, rank_error(v, cmp, tie, 1 << (logn - 1)), ETA)


def rank_error(v, cmp, tie, slots, margin=0.01):
    """delta: the largest distance of the circuit's k_j from the integer ranks
    on this input under the comparator `cmp` (the slot-level shadow, which has
    no noise), plus `margin` for the CKKS noise"""
    v = np.asarray(v, dtype=np.float64)
    _, _, kv = S.order_range_circuit(v, slots, 1, 1, cmp, cmp, tie)
    return float(np.max(np.abs(kv[:len(v)] - ranks_of(v)))) + margin


def direct_rank_error(v, cmp, margin=0.01):
    """delta for circuits whose ranks are k_j = sum_i Cmp(v_j - v_i) + 1/2
    without tie-correction (sort, multi-ciphertext rank and sort): the largest
    distance of the noiseless k_j from the integer ranks, plus `margin`.  The
    all-pairs sum is the definition of the rank (Algorithm Rank; Equation (3)
    regroups the same terms by blocks), so it holds at any N, also where the
    single-ciphertext layout would not fit the ring."""
    v = np.asarray(v, dtype=np.float64)
    k = S.cmp_of(v[:, None] - v[None, :], tuple(cmp)).sum(axis=1) + 0.5
    return float(np.max(np.abs(k - ranks_of(v)))) + margin


def sort_bound(v, ind, delta, eta):
    """Bound on max_i |sorted slot i - i-th smallest value| for Algorithm
    Sorting (and its column and multi-ciphertext forms): slot i is
    sum_j Ind((k_j - i)/N) v_j with Ind(x) = Cmp(x + 1/(2N)) (1 - Cmp(x - 1/(2N))),
    the two-sided window [i, i] of value_bound, so element j at rank distance
    d = |r_j - i| deviates from its ideal weight by at most
    (1 + M) L((1/2 - delta)/N) for d = 0 and M L((d - 1/2 - delta)/N) otherwise."""
    v = np.asarray(v, dtype=np.float64)
    N = len(v)
    r = ranks_of(v)
    M = other_factor(ind)
    tab, _ = _table(ind)
    # deviation by rank distance d = 0..N-1
    d = np.arange(N, dtype=np.float64)
    x = np.where(d == 0, 0.5 - delta, d - 0.5 - delta) / N
    idx = np.floor(np.clip(x, 0.0, 1.0) * _G).astype(np.int64)
    dev = np.where(d == 0, (1.0 + M) * tab[idx], M * tab[idx])
    av = np.abs(v)
    i = np.arange(1, N + 1)
    D = np.abs(r[None, :] - i[:, None])          # [slot i][element j]
    per_slot = (dev[D] + eta) @ av
    return float(np.max(per_slot))


def sort_tolerance(v, cmp, ind, eta=ETA):
    return sort_bound(v, ind, direct_rank_error(v, cmp), eta)


def average_ranks(v):
    """ranks without tie-correction: equal values share the mean of their
    places, #smaller + (copies + 1)/2 (what sum_i Cmp(v_j - v_i) + 1/2 gives
    with Cmp(0) = 1/2)"""
    v = np.asarray(v, dtype=np.float64)
    less = (v[None, :] < v[:, None]).sum(axis=1)
    same = (v[None, :] == v[:, None]).sum(axis=1)
    return less + (same + 1) / 2.0


def division_bound(v, k, cmp, ind, iters, eta=ETA):
    """Bound on |value - ideal| for the order statistic with the value by
    division (section 3.2: SumC(O V) / SumC(O), Goldschmidt's inverse of
    x = s SumC(O), s = 2/(N + 1), over `iters` factors).  The ideal value is
    the value of rank k, or 0 when no element has rank k (ranks without
    tie-correction: c copies of a value share one rank).

    Goldschmidt's product is exactly (1 - b^(2^d)) / x with b = 1 - x, so
    value = (num / den) (1 - b^(2^d)).  With mask deviations e_j, |e_j| <= m_j
    (the window bound at [k, k] taken at the elements' rank distances, plus
    eta), num = c t + sum e_j v_j and den = c + sum e_j:
      c > 0:  |value - t| <= E + (|t| + E) max|b|^(2^d),
              E = sum m_j |v_j - t| / (c - sum m_j),
              b over s [c - sum m_j, c + sum m_j];
      c = 0:  |value| <= s |num| 2^d <= s 2^d sum m_j |v_j|  (|1 - b^(2^d)| / x <= 2^d for |b| <= 1).
    The products of the Goldschmidt chain add eta (d + 2) G (|t| + 1), G the
    largest value of the inverse on the count's range."""
    v = np.asarray(v, dtype=np.float64)
    N = len(v)
    r = average_ranks(v)
    kd = S.cmp_of(v[:, None] - v[None, :], tuple(cmp)).sum(axis=1) + 0.5
    delta = float(np.max(np.abs(kd - r))) + 0.01
    M = other_factor(ind)
    L = lambda d: leak(ind, (d - delta) / N)  # noqa: E731
    m = np.empty(N)
    for j in range(N):
        if k == 1:
            m[j] = L(abs(k + 0.5 - r[j]))
        elif k == N:
            m[j] = L(abs(r[j] - (k - 0.5)))
        elif r[j] < k - 0.25:
            m[j] = L(k - 0.5 - r[j]) * M
        elif r[j] > k + 0.25:
            m[j] = M * L(r[j] - k - 0.5)
        else:
            m[j] = L(r[j] - (k - 0.5)) + M * L(k + 0.5 - r[j])
    m = m + eta
    s = 2.0 / (N + 1.0)
    sel = np.abs(r - k) < 0.25
    c = int(np.sum(sel))
    d2 = 2 ** iters
    if c == 0:
        G = float(2 ** iters)
        return s * G * float(np.dot(m, np.abs(v))) + eta * (iters + 2) * G
    t = float(v[sel][0])
    Msum = float(np.sum(m))
    E = float(np.dot(m, np.abs(v - t))) / (c - Msum)
    bmax = max(abs(1.0 - s * (c - Msum)), abs(1.0 - s * (c + Msum)))
    G = 1.0 / (s * (c - Msum))
    return E + (abs(t) + E) * bmax ** d2 + eta * (iters + 2) * G * (abs(t) + 1.0)
