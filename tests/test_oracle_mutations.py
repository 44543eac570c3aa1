"""Plant plausible mistakes in a copy of the oracle source and check that the
pins of test_oracle.py catch every one of them (CPU only)."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import fraction_ref as fr
from mpgen import random_cmat
from tests import test_oracle as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle_cgemm.c")

MUTATIONS = {
    "drop_imim_term": ("tm[nt++] = (term4){ai, bi, 1};", ""),
    "wrong_sign_imim": ("tm[nt++] = (term4){ai, bi, 1};", "tm[nt++] = (term4){ai, bi, 0};"),
    "swapped_operand_im": ("tm[nt++] = (term4){ar, bi, 0};", "tm[nt++] = (term4){ar, br, 0};"),
    "ties_away": ("round_up = rbit && (sticky || lsb);", "round_up = rbit;"),
    "truncate": ("round_up = rbit && (sticky || lsb);", "round_up = 0;"),
    "no_sticky": ("round_up = rbit && (sticky || lsb);", "round_up = rbit && lsb;"),
    "exponent_off_by_one": ("int64_t e_out = top + 1 + base;", "int64_t e_out = top + base;"),
    "wrong_row_index": ("int64_t ia = (int64_t)t * J->lda + i;",
                        "int64_t ia = (int64_t)t * J->lda + (J->m - 1 - i);"),
    "lost_roundup_carry": ("carry = (s < M[l]) ? 1 : 0;", "carry = 0;"),
    "reads_all_limb_bits": ("int drop = 64 * L - p; /* 0..63 */", "int drop = 0;"),
    "3m_sum_sign": ("acc_add_shifted(out->mag, n, r[t]->sig, L, r[t]->e - p - base, r[t]->neg);",
                    "acc_add_shifted(out->mag, n, r[t]->sig, L, r[t]->e - p - base, 0);"),
}


def _pin_suite():
    """A compact run of the pins; returns the names of the pins that failed."""
    failed = []

    def attempt(name, fn, *args):
        try:
            fn(*args)
        except AssertionError:
            failed.append(name)

    for trial in range(0, 60, 3):
        attempt(f"brute{trial}", pins.test_bruteforce_random, trial)
    attempt("exhaustive_p2", pins.test_exhaustive_1x1x1_p2)
    for case in pins._parse_golden()[::3]:
        attempt("worked", pins.test_worked_rounding_cases, *case)
    attempt("identity", pins.test_identity, 64)
    attempt("conj", pins.test_conjugate_transpose, 100)
    attempt("low_bits", pins.test_low_bits_below_precision_are_ignored)
    attempt("3m_eq_4m", pins.test_3m_form_equals_4m_form, 1)
    return failed


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def test_pins_pass_on_the_real_oracle():
    assert _pin_suite() == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, source, tmp_path):
    old, new = MUTATIONS[name]
    assert old in source, f"mutation anchor for {name} not found"
    mutated = source.replace(old, new)
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-fPIC", "-shared", "-pthread", "-o", str(so), str(c)],
                   check=True)
    with oracle.use_library(str(so)):
        failed = _pin_suite()
    assert failed, f"planted mistake {name} was not caught by any pin"


# ---------------------------------------------------------------------------
# the accumulating form (C := Cin + sign AB): mistakes in the addend's term
# ---------------------------------------------------------------------------
ACC_MUTATIONS = {
    "acc_addend_dropped": ("acc_add_shifted(acc, nacc, addend->sig, L, addend->e - p - base, addend->neg);", ""),
    "acc_addend_sign_ignored": ("acc_add_shifted(acc, nacc, addend->sig, L, addend->e - p - base, addend->neg);",
                                "acc_add_shifted(acc, nacc, addend->sig, L, addend->e - p - base, 0);"),
    "acc_addend_shifted_by_one": ("acc_add_shifted(acc, nacc, addend->sig, L, addend->e - p - base, addend->neg);",
                                  "acc_add_shifted(acc, nacc, addend->sig, L, addend->e - p - base + 1, addend->neg);"),
    "acc_product_sign_ignored": ("int neg = x->neg ^ y->neg ^ tm[q].negate ^ neg_prod;",
                                 "int neg = x->neg ^ y->neg ^ tm[q].negate;"),
}


def _acc_pin_suite():
    from tests import test_oracle_acc as apins
    failed = []

    def attempt(name, fn, *args):
        try:
            fn(*args)
        except AssertionError:
            failed.append(name)

    for trial in range(0, 48, 4):
        attempt(f"acc_brute{trial}", apins.test_acc_bruteforce_random, trial)
    attempt("acc_cancel", apins.test_acc_cancellation_against_fractions, 53)
    attempt("acc_zero_addend", apins.test_acc_zero_addend_is_the_product)
    attempt("acc_zero_product", apins.test_acc_zero_product_returns_addend)
    attempt("acc_symmetry", apins.test_acc_sign_symmetry, 64)
    return failed


def test_acc_pins_pass_on_the_real_oracle():
    assert _acc_pin_suite() == []


@pytest.mark.parametrize("name", sorted(ACC_MUTATIONS))
def test_planted_accumulate_mistake_is_caught(name, source, tmp_path):
    old, new = ACC_MUTATIONS[name]
    assert old in source, f"mutation anchor for {name} not found"
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(source.replace(old, new))
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-fPIC", "-shared", "-pthread", "-o", str(so), str(c)],
                   check=True)
    with oracle.use_library(str(so)):
        failed = _acc_pin_suite()
    assert failed, f"planted mistake {name} was not caught by any pin"
