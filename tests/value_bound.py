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
