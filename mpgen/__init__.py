"""Seeded synthetic multi-precision complex matrices.

This module only draws random inputs and lays them out; it performs none of
the multiplication, splitting or rounding arithmetic.  Both the device path
and the CPU oracle consume what it produces.

Storage of one real component (the Re or Im part of a matrix), column-major
with leading dimension ``ld``:

* ``sign`` uint8 ``[cols, ld]``: 0 for +, 1 for -.
* ``exp``  int32 ``[cols, ld]``: the value is ``(-1)^sign * M * 2^(exp - 64L)``;
  ``exp == EXP_ZERO`` (INT32_MIN) marks an exact zero.
* ``mant`` uint64 ``[L, cols, ld]`` (limb-planar): limb 0 is least significant,
  the top bit of limb L-1 is set for nonzero entries, and the ``64L - p`` bits
  below the precision are zero, so the significand ``M / 2^(64L)`` lies in
  ``[1/2, 1)`` as in MPFR.

The element distribution stands in for the paper's benchmark inputs (random
real and imaginary parts of moderate magnitude, Section IV-A): each real
component is ``+-u * 2^e`` with a fair sign, ``e`` uniform on ``[-R, R]`` and
``u`` a uniform random ``p``-bit significand in ``[1/2, 1)``.
"""
from __future__ import annotations

import dataclasses

import numpy as np

EXP_ZERO = np.iinfo(np.int32).min


def limbs_for(prec_bits: int) -> int:
    return (prec_bits + 63) // 64


@dataclasses.dataclass
class HostPart:
    """One real component, host memory, column-major."""

    rows: int
    cols: int
    ld: int
    L: int
    sign: np.ndarray  # uint8 [cols, ld]
    exp: np.ndarray  # int32 [cols, ld]
    mant: np.ndarray  # uint64 [L, cols, ld]

    def copy(self) -> "HostPart":
        return HostPart(self.rows, self.cols, self.ld, self.L, self.sign.copy(),
                        self.exp.copy(), self.mant.copy())


@dataclasses.dataclass
class HostCMat:
    re: HostPart
    im: HostPart

    @property
    def rows(self) -> int:
        return self.re.rows

    @property
    def cols(self) -> int:
        return self.re.cols

    @property
    def ld(self) -> int:
        return self.re.ld

    @property
    def L(self) -> int:
        return self.re.L

    def copy(self) -> "HostCMat":
        return HostCMat(self.re.copy(), self.im.copy())


def empty_part(rows: int, cols: int, prec_bits: int, ld: int | None = None) -> HostPart:
    """All-zero component (every entry flagged EXP_ZERO)."""
    ld = rows if ld is None else ld
    L = limbs_for(prec_bits)
    return HostPart(rows, cols, ld, L,
                    np.zeros((cols, ld), np.uint8),
                    np.full((cols, ld), EXP_ZERO, np.int32),
                    np.zeros((L, cols, ld), np.uint64))


def empty_cmat(rows: int, cols: int, prec_bits: int, ld: int | None = None) -> HostCMat:
    return HostCMat(empty_part(rows, cols, prec_bits, ld), empty_part(rows, cols, prec_bits, ld))


def _low_mask(prec_bits: int) -> np.uint64:
    L = limbs_for(prec_bits)
    drop = 64 * L - prec_bits  # bits of limb 0 below the precision
    return np.uint64(((1 << 64) - 1) ^ ((1 << drop) - 1))


def random_part(rng: np.random.Generator, rows: int, cols: int, prec_bits: int,
                exp_range: int, ld: int | None = None, zero_frac: float = 0.0) -> HostPart:
    """Random component: fair sign, exponent uniform on [-R, R], p-bit significand."""
    ld = rows if ld is None else ld
    L = limbs_for(prec_bits)
    sign = rng.integers(0, 2, size=(cols, ld), dtype=np.uint8)
    exp = rng.integers(-exp_range, exp_range + 1, size=(cols, ld), dtype=np.int32)
    mant = rng.integers(0, np.iinfo(np.uint64).max, size=(L, cols, ld), dtype=np.uint64,
                        endpoint=True)
    mant[L - 1] |= np.uint64(1 << 63)
    mant[0] &= _low_mask(prec_bits)
    if zero_frac > 0.0:
        z = rng.random(size=(cols, ld)) < zero_frac
        exp[z] = EXP_ZERO
        sign[z] = 0
        mant[:, z] = 0
    if ld > rows:  # padding rows are zero
        exp[:, rows:] = EXP_ZERO
        sign[:, rows:] = 0
        mant[:, :, rows:] = 0
    return HostPart(rows, cols, ld, L, sign, exp, mant)


def random_cmat(seed, which: int, rows: int, cols: int, prec_bits: int, exp_range: int,
                ld: int | None = None, zero_frac: float = 0.0) -> HostCMat:
    """Random complex matrix; Re and Im draw sign, exponent and significand independently."""
    rng = np.random.default_rng([int(s) for s in np.atleast_1d(seed)] + [int(which)])
    re = random_part(rng, rows, cols, prec_bits, exp_range, ld, zero_frac)
    im = random_part(rng, rows, cols, prec_bits, exp_range, ld, zero_frac)
    return HostCMat(re, im)


def scale_exponents(part: HostPart, rows=None, cols=None, shift: int = 0) -> None:
    """Add ``shift`` to the exponents of the selected nonzero entries (in place)."""
    sel = np.zeros((part.cols, part.ld), bool)
    if rows is not None:
        sel[:, rows] = True
    if cols is not None:
        sel[cols, :] = True
    sel[:, part.rows:] = False
    sel &= part.exp != EXP_ZERO
    part.exp[sel] += np.int32(shift)


# ---------------------------------------------------------------------------
# Workloads.  Square problems use the sizes of the benchmark families; the
# batched family draws its shapes from the same seed.
# ---------------------------------------------------------------------------

WORKLOADS = {
    # name: (m, n, k, prec_bits, exp_range, seed)
    "cgemm64_p256": (64, 64, 64, 256, 4, 1),
    "cgemm512_p512": (512, 512, 512, 512, 8, 2),
    "cgemm2048_p1024": (2048, 2048, 2048, 1024, 32, 3),
}


def workload_inputs(name: str):
    """Return (m, n, k, prec_bits, A, B) for a named square workload."""
    if name in WORKLOADS:
        m, n, k, p, R, seed = WORKLOADS[name]
        A = random_cmat(seed, 0, m, k, p, R)
        B = random_cmat(seed, 1, k, n, p, R)
        return m, n, k, p, A, B
    if name == "cgemm2048_p1024_im200":
        # every imaginary part 2^200 below the real parts (exponents in [-232, -168])
        m, n, k, p, R, _ = WORKLOADS["cgemm2048_p1024"]
        A = random_cmat(33, 0, m, k, p, R)
        B = random_cmat(33, 1, k, n, p, R)
        scale_exponents(A.im, rows=list(range(m)), shift=-200)
        scale_exponents(B.im, rows=list(range(k)), shift=-200)
        return m, n, k, p, A, B
    if name in ("cgemm2048_p1024_rowcol60", "cgemm2048_p1024_contract60"):
        m, n, k, p, R, _ = WORKLOADS["cgemm2048_p1024"]
        seed = 31 if name.endswith("rowcol60") else 32
        A = random_cmat(seed, 0, m, k, p, R)
        B = random_cmat(seed, 1, k, n, p, R)
        if name.endswith("rowcol60"):
            # one row of A and one column of B carry an extra factor 2^60
            for part in (A.re, A.im):
                scale_exponents(part, rows=[7], shift=60)
            for part in (B.re, B.im):
                scale_exponents(part, cols=[11], shift=60)
        else:
            # the same factor on one contraction index: column 7 of A, row 7 of B
            for part in (A.re, A.im):
                scale_exponents(part, cols=[7], shift=60)
            for part in (B.re, B.im):
                scale_exponents(part, rows=[7], shift=60)
        return m, n, k, p, A, B
    raise KeyError(name)


def batched_shapes(count: int = 256, seed: int = 4, lo: int = 16, hi: int = 768):
    """Shapes (m, n, k) of the uneven batched family, each uniform on [lo, hi]."""
    rng = np.random.default_rng(seed)
    return [tuple(int(x) for x in row) for row in rng.integers(lo, hi + 1, size=(count, 3))]


def batched_inputs(count: int = 256, seed: int = 4, prec_bits: int = 256, exp_range: int = 8):
    shapes = batched_shapes(count, seed)
    out = []
    for idx, (m, n, k) in enumerate(shapes):
        A = random_cmat([seed, idx], 0, m, k, prec_bits, exp_range)
        B = random_cmat([seed, idx], 1, k, n, prec_bits, exp_range)
        out.append((m, n, k, A, B))
    return out


def multi_double(seed, which: int, ncomp: int, rows: int, cols: int, kind: str = "expansion",
                 exp_range: int = 30) -> np.ndarray:
    """Multi-component inputs (double-double to quad-double): a float64 array
    (ncomp, cols, rows), entry (r, c) standing for the sum of its components.

    kind "expansion": the normalised form of multi-component arithmetic, each
    component at most half an ulp of the one before (random sign and
    significand), the leading one's exponent uniform on [-exp_range, exp_range];
    "random": independent doubles with exponents over [-exp_range, exp_range]
    (overlaps, gaps and sign changes); "extreme": subnormals, values near the
    largest double, zeros and exact cancellations mixed in."""
    rng = np.random.default_rng([seed, which, ncomp])
    shape = (cols, rows)
    if kind == "random":
        x = rng.uniform(-1.0, 1.0, size=(ncomp,) + shape)
        return np.ldexp(x, rng.integers(-exp_range, exp_range + 1, size=(ncomp,) + shape))
    out = np.zeros((ncomp,) + shape)
    lead = rng.uniform(0.5, 1.0, size=shape) * rng.choice([-1.0, 1.0], size=shape)
    out[0] = np.ldexp(lead, rng.integers(-exp_range, exp_range + 1, size=shape))
    for i in range(1, ncomp):
        # at most half an ulp of the previous component: |x| < 2^(e - 53) with
        # 2^(e-1) <= |prev| < 2^e, times a random fraction and sign
        _, e = np.frexp(out[i - 1])
        f = rng.uniform(-1.0, 1.0, size=shape)
        out[i] = np.where(out[i - 1] != 0, np.ldexp(f, e - 54), 0.0)
    if kind == "extreme":
        pick = rng.integers(0, 6, size=shape)
        tiny = np.ldexp(rng.uniform(0.0, 1.0, size=shape), -1060)  # subnormal range
        huge = np.ldexp(rng.uniform(0.5, 1.0, size=shape), 1023) * rng.choice([-1.0, 1.0], size=shape)
        for i in range(ncomp):
            out[i] = np.where(pick == 0, tiny * (i + 1), out[i])
            out[i] = np.where(pick == 1, huge if i == 0 else np.ldexp(out[i], -i * 300), out[i])
            out[i] = np.where((pick == 2) & (i % 2 == 1), 0.0, out[i])
        if ncomp >= 2:
            out[1] = np.where(pick == 3, -out[0], out[1])  # exact cancellation of the leading pair
        if ncomp >= 3:
            out[2] = np.where(pick == 4, np.ldexp(out[0], -700), out[2])  # a far gap
    return out
