"""Plant plausible mistakes in a copy of the LU oracle (oracle/lu_ref.py) and
check that the pins of test_oracle_lu.py catch every one of them (CPU only)."""
from __future__ import annotations

import os
import types

import pytest

from oracle import lu_ref
from tests import test_oracle_lu as pins

SRC = lu_ref.__file__

MUTATIONS = {
    "pivot_last_of_equal_keys": ("if bv is None or v > bv:", "if bv is None or v >= bv:"),
    "reciprocal_without_conjugate": ("_store(x.im, -yi / d, prec_bits)", "_store(x.im, yi / d, prec_bits)"),
    "reciprocal_denominator_difference": ("    d = yr * yr + yi * yi\n", "    d = yr * yr - yi * yi\n"),
    "reciprocal_parts_swapped": ("_store(x.re, yr / d, prec_bits)", "_store(x.re, yi / d, prec_bits)"),
    "panel_update_sign": ("_sub(M, c + 1, mr - 1, c + 1, w), p, sign=-1))", "_sub(M, c + 1, mr - 1, c + 1, w), p, sign=+1))"),
    "no_u12_solve": ("for c in range(j, j + jb - 1):", "for c in range(j, j):"),
    "trailing_update_sign": ("_sub(M, j + jb, nr, j + jb, nr), p, sign=-1))", "_sub(M, j + jb, nr, j + jb, nr), p, sign=+1))"),
    "reciprocal_truncated": ("    sg, e, q = round_rne(value, prec_bits)\n",
                             "    sg, e, q = round_rne(value, prec_bits)\n    q = (q >> 1) << 1 if prec_bits > 2 else q\n"),
    "forward_skips_a_row": ("    for c in range(1, n):\n", "    for c in range(2, n):\n"),
    "info_zero_based": ("                info = c + 1\n", "                info = c\n"),
    "no_row_exchange": ("            _swap_rows(M, c, r)\n", "            pass\n"),
}


def _mutant(old: str, new: str):
    text = open(SRC).read()
    assert text.count(old) == 1, old
    mod = types.ModuleType("lu_ref_mutant")
    mod.__file__ = SRC
    exec(compile(text.replace(old, new), SRC, "exec"), mod.__dict__)
    return mod


def _pin_suite():
    """A compact run of the pins; returns the names of the pins that failed."""
    failed = []

    def attempt(name, fn, *args):
        try:
            fn(*args)
        except Exception:  # an assertion or a shape error: the pin caught it
            failed.append(name)

    attempt("reciprocal", pins.test_reciprocal_matches_mpmath, 256)
    attempt("reciprocal_ieee", pins.test_reciprocal_p53_real_and_imaginary_match_ieee_division)
    attempt("reciprocal_pow2", pins.test_reciprocal_of_powers_of_two_is_exact, 64)
    attempt("exact_7_3", pins.test_exact_factors, 7, 3)
    attempt("exact_12_5", pins.test_exact_factors, 12, 5)
    attempt("backward", pins.test_backward_error, 9, 4, 64)
    attempt("ties", pins.test_pivot_ties_take_the_first_row)
    attempt("zero_pivot", pins.test_zero_pivot_is_reported)
    return failed


def test_unmutated_oracle_passes_the_suite():
    assert _pin_suite() == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    old, new = MUTATIONS[name]
    monkeypatch.setattr(pins, "lu_ref", _mutant(old, new))
    assert _pin_suite(), f"mutation {name} survived every pin"
