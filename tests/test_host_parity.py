"""CPU-side checks of the product library (no GPU): the C ABI loads and exports
every declared entry point, and its host-side pieces (modulus chain, slot
encoder, ChaCha20 sampler) agree bit for bit with the oracle's independent
implementations."""
import os
import re

import numpy as np
import pytest

import paper_2412_15126_amd as ckr
from paper_2412_15126_amd import workloads as W

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ckr.h")


def declared_functions():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ckr_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = ckr.lib()
    names = declared_functions()
    assert len(names) > 30
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("name", sorted(W.PSETS))
def test_modulus_chain_matches_oracle(ora, name):
    mods, scales = ckr.derive_params(W.PSETS[name])
    P = ora.Params(**W.PSETS[name])
    assert np.array_equal(mods, P.mods)
    assert np.array_equal(scales.view(np.uint64), P.scales.view(np.uint64))


def test_bad_params_rejected():
    bad = dict(W.PSETS["T10"], q0_bits=55)
    with pytest.raises(ckr.CkrError) as e:
        ckr.derive_params(bad)
    assert e.value.status == -1


@pytest.mark.parametrize("logn", [10, 12, 13])
def test_encoder_matches_oracle_bit_for_bit(ora, logn):
    P = ora.Params(**dict(W.PSETS["T10"], logn=logn))
    rng = np.random.default_rng(logn)
    h = (1 << logn) // 2
    cases = [rng.uniform(-1, 1, h), rng.uniform(0, 1, 37), np.ones(h), np.zeros(5),
             np.where(np.arange(64) % 8 == 0, 1.0, 0.0), np.full(8, 0.5)]
    for z in cases:
        for scale in (2.0 ** 36, 68719476736.0 * (1 + 2 ** -20), P.scales[3]):
            a = ckr.encode(logn, z, scale)
            b = ora.encode(P, z, scale)
            assert np.array_equal(a, b)


def test_encoder_rejects_too_many_slots():
    with pytest.raises(ckr.CkrError) as e:
        ckr.encode(10, np.zeros(513), 2.0 ** 30)
    assert e.value.status == -2


def test_sampler_matches_oracle(ora):
    key = bytes(range(1, 33))
    for purpose, oid, kind, q in [(1, 0, 0, 0), (3, 0, 1, 0), (2, 5, 2, (1 << 44) + 7), (4, (97 << 32) | 3, 2, 12289)]:
        assert np.array_equal(ckr.sample(key, purpose, oid, kind, q, 5000), ora.sample(key, purpose, oid, kind, q, 5000))


def _rn(x):
    """round a Fraction to the nearest IEEE double (ties to even), as a Fraction"""
    from fractions import Fraction
    f = float(x)                     # Python's int/Fraction -> float conversion rounds to nearest even
    return Fraction(f)


def test_twiddle_recovered_from_its_quotient():
    """The row passes keep only wq = RN(w/q) per twiddle and recover
    w = RN(wq * q + 2^52) - 2^52 (one FMA, one subtraction).  For primes below
    2^50 this is exact: |wq q - w| <= w 2^-53 < 1/8.  Checked with exact
    rational arithmetic on the extreme and random cases."""
    from fractions import Fraction
    rng = np.random.default_rng(5)
    cases = []
    for q in (2**50 - 27, 2**49 + 9, 2**44 + 7, 1125899906826241, 65537):
        cases += [(w, q) for w in (1, 2, q - 1, q - 2, q // 2, q // 3)]
        cases += [(int(w), q) for w in rng.integers(1, q, 200)]
    for w, q in cases:
        wq = _rn(Fraction(w, q))
        assert wq == Fraction(float(w) / float(q))            # the table's value: IEEE division, correctly rounded
        rec = _rn(wq * q + 2**52) - 2**52                      # the FMA rounds the exact sum once
        assert rec == w, (w, q)
