"""Host checks of the range arguments the HIP kernels' exact FP64 reductions
rest on (integer-valued doubles; every modulus is a prime below 2^50).

- A reduction of x, |x| < 2^53, takes k = rint(x * fl(1/q)) and forms x - k q
  with one FMA.  That value must lie in (-q, q): then it is an integer the FMA
  forms exactly, and one conditional add of q makes it canonical.
- The base conversion adds NS terms in (0, 2t) to a start in (-t, 0]: all of
  them before one reduction when t (2 NS + 1) <= 2^53, else 3 at a time from
  a start in (-t, t), so every partial sum stays an integer below 2^53.

The products are computed here the way the kernel computes them: IEEE double
multiplication and round-to-nearest-even, with the exact difference in Python
integers (the FMA's exact result, which is representable)."""
import numpy as np

from paper_2412_15126_amd import workloads as W


def _moduli():
    """the library's primes for the full-size parameter sets, plus extremes"""
    import paper_2412_15126_amd as ckr
    qs = set()
    for name in ("P12", "P16", "P17", "P17S"):
        qs.update(int(q) for q in ckr.derive_params(W.PSETS[name])[0])
    qs.update({(1 << 50) - 27, (1 << 49) + 69, (1 << 40) + 15, (1 << 30) + 3, 12289})
    return sorted(qs)


def _reduce(x, q):
    k = int(np.rint(np.float64(x) * (np.float64(1.0) / np.float64(q))))
    return x - k * q


def test_single_correction_reduction_range():
    rng = np.random.default_rng(3)
    lim = (1 << 53) - 1
    for q in _moduli():
        xs = [lim, -lim, 0, 1, -1, q, -q, q - 1, 1 - q]
        xs += [int(v) for v in rng.integers(-lim, lim, 400, dtype=np.int64)]
        # next to multiples of q and of q/2, where the quotient estimate is closest to a tie
        for m in rng.integers(1, lim // q, 60, dtype=np.int64):
            for base in (int(m) * q, int(m) * q + q // 2):
                xs += [base + d for d in (-2, -1, 0, 1, 2) if abs(base + d) <= lim]
        for x in xs:
            r = _reduce(x, q)
            assert -q < r < q, (q, x, r)
            assert (r + q if r < 0 else r) == x % q


def test_base_conversion_sums_stay_exact():
    for t in _moduli():
        assert 7 * t < (1 << 53), t          # 3 terms from a start in (-t, t)
        for ns in range(1, 17):
            if t * (2 * ns + 1) <= (1 << 53):
                assert 2 * ns * t < (1 << 53)  # all NS terms from a start in (-t, 0]
