"""CPU: the arithmetic behind the fused kernel's barycenter quotient.

The kernel forms the barycenter (2M + C) / (2C) of two exact integers N < 2^53, 0 < D < 2^27 as
y0 = estimate of 1/D (the hardware reciprocal), y = y0 + y0 (1 - D y0), q1 = N y,
r = N - D q1 (one fused multiply-add), q2 = q1 + r y, and rounds q2 to float. It must give the
same float as rounding the double quotient N / D (the oracle's form, paper §2: the centroid of
the cluster charge). Here every step is carried out in exact rational arithmetic with
round-to-nearest-even to double after each operation, for reciprocal estimates off by up to
2^-14, on random pairs and on pairs whose quotient is, or lies next to, a float midpoint.
"""
from fractions import Fraction

import numpy as np

RNG = np.random.default_rng(11489)


def _rn(x: Fraction) -> float:
    return float(x)   # int / int true division: correctly rounded to the nearest double


def _fma(a, b, c) -> float:
    return _rn(Fraction(a) * Fraction(b) + Fraction(c))


def _method(n: int, d: int, err: Fraction) -> np.float32:
    y0 = _rn(Fraction(1, d) * (1 + err))
    y = _fma(y0, _fma(-float(d), y0, 1.0), y0)
    q1 = _rn(Fraction(n) * Fraction(y))
    r = _fma(-float(d), q1, float(n))
    return np.float32(_fma(r, y, q1))


def _reference(n: int, d: int) -> np.float32:
    return np.float32(n / d)   # the correctly rounded double quotient, then to float


ERRS = [Fraction(0), Fraction(1, 2**22), Fraction(-1, 2**22), Fraction(1, 2**14),
        Fraction(-1, 2**14)]


def _cases():
    """(n, d, is_midpoint) triples."""
    out = []
    for _ in range(1500):                      # barycenters up to 800 strips
        d = int(RNG.integers(1, 2**27))
        out.append((int(RNG.integers(0, d * 1600)), d, False))
    for _ in range(1500):                      # exact float midpoints K 2^-e, K odd of 25 bits
        k = int(RNG.integers(2**23, 2**24)) * 2 + 1
        e = int(RNG.integers(15, 25))
        d = (int(RNG.integers(1, 2**27)) >> e << e) or (1 << e)
        n = k * (d >> e)
        out += [(n, d, True), (n + 1, d, False), (n - 1, d, False)]   # and right next to them
    out += [(0, 2, False), (1, 2, False), (3, 2, False), (2**53 - 1, 2**27 - 1, False),
            (2**27 - 1, 2**27 - 2, False)]
    return out


def test_quotient_method_rounds_like_the_double_quotient():
    for n, d, mid in _cases():
        ref = _reference(n, d)
        if mid:   # halfway between two floats: the tie rule decides
            assert Fraction(float(ref)) != Fraction(n, d)
        for err in ERRS:
            got = _method(n, d, err)
            assert got.view(np.uint32) == ref.view(np.uint32), (n, d, err, got, ref)
