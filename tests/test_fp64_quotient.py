"""The FP64 kernels divide by constants (the 12 of the fourth-order difference,
the 3 of the pressure and the RK3 stage, the interface width W) as
q = RN(a y), r = fma(-b, q, a), q' = fma(r, y, q) with y = RN(1/b), which
Markstein's theorem makes the correctly rounded a / b for normal quotients;
the FP64 parity with the oracle's plain divisions rests on it.  Emulated here
exactly (rational arithmetic, one rounding per operation) against IEEE
division, on random operands over the whole exponent range and on structured
ones (small integers, significands next to 1 and 2, powers of two)."""

import random
from fractions import Fraction

import pytest


def _fma(x, y, z):
    return float(Fraction(x) * Fraction(y) + Fraction(z))


def _quotient(a, b, y):
    q = a * y
    r = _fma(-b, q, a)
    return _fma(r, y, q) if r != 0.0 else q


@pytest.mark.parametrize("b", [12.0, 3.0, 4.0, 3.7, 2.5, 5.0, 7.0])
def test_fma_corrected_quotient_is_correctly_rounded(b):
    y = 1.0 / b
    rng = random.Random(int(b * 10))
    cases = [rng.uniform(1, 2) * 2.0 ** rng.randint(-1000, 1000) for _ in range(4000)]
    cases += [float(i) for i in range(1, 3000)]
    cases += [1.0 + k * 2.0 ** -52 for k in range(1500)] + [2.0 - k * 2.0 ** -52 for k in range(1, 1500)]
    cases += [2.0 ** e for e in range(-1000, 1001, 7)]
    bad = [a for a in cases for s in (a, -a) if _quotient(s, b, y) != s / b]
    assert not bad, (b, bad[:5])


def test_a_planted_error_is_caught():
    """Without the correction step the plain product RN(a y) is not always the
    quotient: the check above would see it."""
    y = 1.0 / 12.0
    rng = random.Random(5)
    cases = [rng.uniform(1, 2) * 2.0 ** rng.randint(-50, 50) for _ in range(2000)]
    assert any(a * y != a / 12.0 for a in cases)
