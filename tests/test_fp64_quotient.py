"""The FP64 kernels divide by constants (the 12 of the fourth-order difference,
the 3 of the pressure and the RK3 stage, the interface width W) as
q = RN(a y), r = fma(-b, q, a), q' = fma(r, y, q) with y = RN(1/b), which
Markstein's theorem makes the correctly rounded a / b for normal quotients;
the FP64 parity with the oracle's plain divisions rests on it.  Emulated here
exactly (rational arithmetic, one rounding per operation) against IEEE
division, on random operands over the whole exponent range and on structured
ones (small integers, significands next to 1 and 2, powers of two).  The FP32
kernels divide sums by 3 the same way (binary32 with fmaf), pinned likewise."""

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


def _f32(x):
    import numpy as np
    return float(np.float32(x))


def _fma32(x, y, z):
    """fmaf: the exact x y + z rounded once to binary32 (Fraction to float64 is
    exact here: x y + z of binary32 operands has at most 49 significant bits
    within a small exponent range, so the float64 value rounds once to binary32)."""
    import numpy as np
    v = Fraction(x) * Fraction(y) + Fraction(z)
    d = float(v)
    assert Fraction(d) == v
    return float(np.float32(d))


def test_fp32_division_by_three_is_correctly_rounded():
    """The FP32 gather's p = c_s^2 sum g as q = RN(a RN(1/3)), r = fmaf(-3, q, a),
    q' = fmaf(r, RN(1/3), q): correctly rounded a / 3 (the plain product is off by
    an ulp with a bias, which a step carries forward)."""
    import numpy as np
    y = _f32(1.0 / 3.0)
    rng = random.Random(33)
    cases = [_f32(rng.uniform(1, 2) * 2.0 ** rng.randint(-60, 60)) for _ in range(6000)]
    cases += [_f32(1.0 + k * 2.0 ** -23) for k in range(2000)]
    cases += [_f32(2.0 - k * 2.0 ** -23) for k in range(1, 2000)]
    cases += [float(i) for i in range(1, 2000)]
    bad, plain_off = [], 0
    for a in cases:
        for s in (a, -a):
            q = _f32(s * y)
            r = _fma32(-3.0, q, s)
            out = _fma32(r, y, q)
            exact = float(np.float32(Fraction(s) / 3))
            if out != exact:
                bad.append(s)
            plain_off += q != exact
    assert not bad, bad[:5]
    assert plain_off > 0
