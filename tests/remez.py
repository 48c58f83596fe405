"""Remez exchange for the minimax composite comparator (test infrastructure).

Section 2.2 of the paper closes by pointing to composite polynomials built
from minimax approximations of the sign function (Lee et al.): the first
polynomial is the degree-d odd minimax approximation of sign(x) on [e, 1];
each later one is the minimax approximation on the interval the previous
one maps [e, 1] onto.  This module recomputes that construction in float64,
independently of the coefficient tables the oracle and the library carry, so
the pins can check those tables against it.
"""
import numpy as np
from scipy.optimize import minimize_scalar


def _powers(x, m):
    return np.stack([x ** (2 * k + 1) for k in range(m)], axis=-1)


def _extrema(err, xs):
    """indices of the largest |err| on each maximal run of constant sign"""
    s = np.sign(err)
    cuts = np.flatnonzero(s[1:] != s[:-1]) + 1
    starts = np.concatenate([[0], cuts])
    ends = np.concatenate([cuts, [len(xs)]])
    return np.array([a + int(np.argmax(np.abs(err[a:b]))) for a, b in zip(starts, ends)])


def minimax_odd_sign(a, b, deg=7, grid=400001, iters=100):
    """Odd polynomial p of degree deg minimising max |1 - p(x)| on [a, b]
    (0 < a < b): returns (coefficients of x, x^3, ..., the levelled error E,
    the alternation points)."""
    m = (deg + 1) // 2
    xs = np.linspace(a, b, grid)
    ref = (a + b) / 2 + (b - a) / 2 * np.cos(np.pi * np.arange(m + 1)[::-1] / m)
    c = E = None
    for _ in range(iters):
        A = np.concatenate([_powers(ref, m), ((-1.0) ** np.arange(m + 1))[:, None]], axis=1)
        sol = np.linalg.solve(A, np.ones(m + 1))
        c, E = sol[:m], sol[m]
        f = lambda x: 1.0 - _powers(np.asarray(x, float), m) @ c  # noqa: E731
        idx = _extrema(f(xs), xs)
        while len(idx) > m + 1:
            idx = idx[1:] if abs(f(xs[idx[0]])) < abs(f(xs[idx[-1]])) else idx[:-1]
        if len(idx) < m + 1:
            break
        new = []
        for i in idx:   # refine each extremum off the grid
            lo, hi = xs[max(i - 1, 0)], xs[min(i + 1, len(xs) - 1)]
            sgn = np.sign(f(xs[i]))
            if lo == hi or i in (0, len(xs) - 1):
                new.append(xs[i])
                continue
            r = minimize_scalar(lambda x: -sgn * f(x), bounds=(lo, hi), method="bounded",
                                options={"xatol": 1e-15 * max(1.0, hi)})
            new.append(r.x)
        new = np.array(new)
        if np.max(np.abs(new - ref)) < 1e-14 * b:
            ref = new
            break
        ref = new
    return c, abs(E), ref


def composite(e, stages, deg=7):
    """[(coefficients, interval)] of the greedy minimax composite designed on [e, 1]"""
    out, a, b = [], e, 1.0
    for _ in range(stages):
        c, _, _ = minimax_odd_sign(a, b, deg)
        xs = np.linspace(a, b, 400001)
        p = _powers(xs, len(c)) @ c
        out.append((c, (a, b)))
        a, b = float(p.min()), float(p.max())
    return out
