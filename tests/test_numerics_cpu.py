"""Host checks of arithmetic identities the kernels rely on (no GPU).

The gather forms the pixel-centre ndc coordinate (2 i + 1) / w as the rounded
reciprocal 1 / w, q0 = (2 i + 1) * (1 / w) and one Markstein correction
q = fma(fma(-q0, w, 2 i + 1), 1 / w, q0).  Here each step is evaluated with
exact rational arithmetic and a single rounding per float operation (what
the fused multiply-adds do), and q must equal the IEEE quotient for every
numerator at the widths in use and at the maximum size."""
from fractions import Fraction

import pytest


def _rn(x):
    return float(x)      # Fraction -> float rounds to nearest, ties to even


def _markstein(a, w):
    r = 1.0 / w                                   # IEEE division: the rounded reciprocal
    q0 = a * r                                    # IEEE product
    rem = _rn(Fraction(a) - Fraction(q0) * w)     # fma(-q0, w, a)
    return _rn(Fraction(rem) * Fraction(r) + Fraction(q0))   # fma(rem, r, q0)


@pytest.mark.parametrize("w", list(range(1, 65)) + [75, 96, 100, 200, 1003, 1080, 1920, 2048, 16384])
def test_markstein_pixel_centre_quotients(w):
    for i in range(w):
        a = 2.0 * (i + 0.5)
        assert _markstein(a, w) == a / w, (i, w)
