"""Pins of the multi-component input definition (oracle/codec_ref.py) against
things other than itself (no GPU needed):

* at p = 53 the rounded sum of finite doubles whose sum is a normal double
  is what ``math.fsum`` returns (a correctly rounded sum, library routine);
* with enough precision the conversion is exact: the stored value equals the
  components' sum;
* worked cases derived by hand: ties to even down and up, a far component
  breaking a tie, exact cancellation to +0, subnormal components, a sum
  beyond the largest double;
* an infinite or NaN component gives +0.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

from mpgen import EXP_ZERO, multi_double
from oracle import codec_ref
from oracle import fraction_ref as fr


def _one(vals, p):
    comps = np.array(vals, dtype=np.float64).reshape(len(vals), 1, 1)
    part = codec_ref.from_doubles_part(comps, p)
    return fr.decode(part, 0, 0, p), part


@pytest.mark.parametrize("kind", ["expansion", "random", "extreme"])
@pytest.mark.parametrize("ncomp", [2, 3, 4])
def test_p53_is_fsum(kind, ncomp):
    comps = multi_double(11, 0, ncomp, 9, 7, kind, exp_range=40)
    part = codec_ref.from_doubles_part(comps, 53)
    checked = 0
    for c in range(7):
        for r in range(9):
            vals = [float(v) for v in comps[:, c, r]]
            f = math.fsum(vals)
            if f != 0 and not (2.0 ** -1022 <= abs(f) < 2.0 ** 1023):
                continue  # fsum is subnormal or near overflow there: another format
            assert fr.decode(part, r, c, 53) == Fraction(f), (vals, f)
            checked += 1
    assert checked > 20


@pytest.mark.parametrize("ncomp", [2, 3, 4])
def test_exact_when_wide_enough(ncomp):
    comps = multi_double(12, 1, ncomp, 6, 5, "expansion", exp_range=20)

    def bits(x: Fraction) -> int:  # significant bits of a dyadic rational
        n = abs(x.numerator)
        return (n >> ((n & -n).bit_length() - 1)).bit_length() if n else 1
    p = max(2, max(bits(codec_ref.exact_sum(comps[:, c, r])) for c in range(5) for r in range(6)))
    assert p > 53 * (ncomp - 1)
    part = codec_ref.from_doubles_part(comps, p)
    for c in range(5):
        for r in range(6):
            assert fr.decode(part, r, c, p) == codec_ref.exact_sum(comps[:, c, r])


def test_worked_cases():
    two = Fraction(2)
    one = Fraction(1)
    # 1 + 2^-53 at p = 53: a tie, the even neighbour is 1
    assert _one([1.0, 2.0 ** -53], 53)[0] == one
    # (1 + 2^-52) + 2^-53: a tie from an odd significand, rounds up
    assert _one([1.0 + 2.0 ** -52, 2.0 ** -53], 53)[0] == one + two ** -51
    # a component far below breaks the tie upward
    assert _one([1.0, 2.0 ** -53, 2.0 ** -900], 53)[0] == one + two ** -52
    # ... and downward when negative
    assert _one([1.0 + 2.0 ** -52, 2.0 ** -53, -(2.0 ** -900)], 53)[0] == one + two ** -52
    # exact cancellation -> +0
    v, part = _one([0.75, -0.75, 2.0 ** -600, -(2.0 ** -600)], 64)
    assert v == 0 and part.exp[0, 0] == EXP_ZERO and part.sign[0, 0] == 0
    # subnormal components add exactly
    assert _one([5e-324, 5e-324], 2)[0] == two ** -1073
    # beyond the largest double (exact in the library's format)
    big = 2.0 ** 1023
    assert _one([big, big, big, big], 2)[0] == two ** 1025
    # negative value, rounding symmetric
    assert _one([-1.0, -(2.0 ** -53), -(2.0 ** -900)], 53)[0] == -(one + two ** -52)
    # carry out of the significand renormalises: 1 - 2^-60 at p = 53 -> 1
    assert _one([1.0, -(2.0 ** -60)], 53)[0] == one


def test_non_finite_gives_zero():
    for bad in (math.inf, -math.inf, math.nan):
        v, part = _one([1.0, bad], 64)
        assert v == 0 and part.exp[0, 0] == EXP_ZERO


def test_round_double_is_float_in_range():
    """The written-out IEEE rounding against Python's correctly rounded
    float(Fraction), including subnormals, ties and the underflow to -0."""
    rng = np.random.default_rng(31)
    cases = [Fraction(1) + Fraction(1, 2 ** 53), Fraction(3, 2 ** 1076), -Fraction(1, 2 ** 1075),
             Fraction(5, 2 ** 1076), -Fraction(2 ** 1024 - 2 ** 971), Fraction(1, 3), -Fraction(10 ** 30, 7)]
    for _ in range(3000):
        num = int(rng.integers(1, 2 ** 62)) * (1 if rng.random() < 0.5 else -1)
        sh = int(rng.integers(-1150, 960))  # |x| < 2^1022
        cases.append(Fraction(num) * Fraction(2) ** sh + Fraction(int(rng.integers(0, 3)), 2 ** 1100))
    for x in cases:
        v, overflow = codec_ref.round_double(x)
        assert not overflow
        f = float(x)
        assert (v == Fraction(f)) and (v != 0 or math.copysign(1.0, f) == (-1.0 if x < 0 else 1.0)), x


def test_round_double_overflow():
    assert codec_ref.round_double(Fraction(2 ** 1024 - 2 ** 970))[1]       # the tie rounds up to 2^1024
    assert not codec_ref.round_double(Fraction(2 ** 1024 - 2 ** 971))[0] == 0


@pytest.mark.parametrize("ncomp", [1, 2, 3, 4])
def test_to_doubles_round_trip(ncomp):
    """A normalised expansion converted exactly and back gives itself."""
    comps = multi_double(13, 2, ncomp, 7, 6, "expansion", exp_range=300)
    part = codec_ref.from_doubles_part(comps, 64 * 4 * ncomp)
    back = codec_ref.to_doubles_part(part, 64 * 4 * ncomp, ncomp)
    assert np.array_equal(back.view(np.uint64), comps.view(np.uint64))


def test_to_doubles_greedy_worked():
    """Greedy components derived by hand."""
    from tests.mp_util import part_from_values
    p = 200
    two = Fraction(2)
    vals = [[1 + two ** -60], [-(1 + two ** -53)], [1 + two ** -53 + two ** -150], [3 * two ** -1076],
            [two ** -1075]]
    part = part_from_values(vals, p)
    d = codec_ref.to_doubles_part(part, p, 3)
    # exact in two components, the third +0
    assert [d[i, 0, 0] for i in range(3)] == [1.0, 2.0 ** -60, 0.0]
    # a tie rounds to the even neighbour 1, the rest follows with the sign
    assert [d[i, 0, 1] for i in range(3)] == [-1.0, -(2.0 ** -53), 0.0]
    # above the tie: up to 1 + 2^-52; the remainder -2^-53 + 2^-150 needs 98
    # bits, so it splits into -2^-53 and 2^-150
    assert [d[i, 0, 2] for i in range(3)] == [1.0 + 2.0 ** -52, -(2.0 ** -53), 2.0 ** -150]
    # 1.5 * 2^-1075 rounds up to the smallest subnormal, leaving -2^-1076 (below half of it: -0)
    assert d[0, 0, 3] == 5e-324 and d[1, 0, 3] == 0.0 and math.copysign(1.0, d[1, 0, 3]) == -1.0
    # 2^-1075 exactly: a tie between 0 and 2^-1074 goes to +0, and stays for the next component
    assert d[0, 0, 4] == 0.0 and math.copysign(1.0, d[0, 0, 4]) == 1.0
