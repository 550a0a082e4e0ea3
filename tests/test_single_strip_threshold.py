"""CPU: the identity behind the fused kernel's cluster test of a one-strip run.

For a run of one strip the cluster threshold (paper §2: the cluster charge against the cluster
threshold times the root of the summed noise squares) is (float)a >= t * sqrtf(fmaf(n, n, 0)).
The kernel tests (float)a >= t * n instead wherever 2^-60 <= n <= 2^60, which relies on
sqrtf(RN(n * n)) == n for such floats (radix 2, round to nearest; the square is normal and
finite). Squares and roots scale exactly by powers of 4 and 2, so two adjacent binades cover
every exponent in that range; both binades are checked for every float, and the range ends
float by float in a sample.
"""
import numpy as np


def _binade(lo: float) -> np.ndarray:
    start = np.float32(lo).view(np.uint32)
    stop = np.float32(2.0 * lo).view(np.uint32)
    return np.arange(start, stop, dtype=np.uint32).view(np.float32)


def _root_of_square(x: np.ndarray) -> np.ndarray:
    sq = np.multiply(x, x, dtype=np.float32)   # one rounding, as fmaf(n, n, 0)
    return np.sqrt(sq, dtype=np.float32)        # correctly rounded, as sqrtf


def test_root_of_rounded_square_is_exact_on_two_binades():
    for lo in (1.0, 2.0):
        x = _binade(lo)
        r = _root_of_square(x)
        assert np.array_equal(r.view(np.uint32), x.view(np.uint32)), lo


def test_range_ends():
    step = 997   # every 997th float of each binade at the two ends of the kernel's range
    for lo in (2.0 ** -60, 2.0 ** 59):
        x = _binade(lo)[::step]
        r = _root_of_square(x)
        assert np.array_equal(r, x), lo
    # below the range the square is subnormal and the identity fails: the bound is needed
    x = _binade(2.0 ** -66)[::step]
    assert not np.array_equal(_root_of_square(x), x)
