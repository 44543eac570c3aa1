// Multi-component fixed-precision inputs (double-double, triple-double,
// quad-double: the multi-component arithmetic named as future work in the
// paper's concluding section) turned into the library's number format.
//
// Each entry of a real component is the exact sum of up to four doubles.  A
// thread forms that sum exactly in a two's-complement fixed-point
// accumulator on a grid whose bit 0 is 2^-1074 (the lowest subnormal bit):
// the largest finite double's top bit is bit 2097, so four of them stay
// below bit 2100, and 34 limbs (2176 bits) leave the top bit for the sign.
// Only the limbs the components touch (and one above) are used: a first
// pass holds them in an 8-limb row when they span at most 512 bits (every
// normalised expansion), a second pass takes the rest with the full row.
// The sum is then rounded once to prec_bits, to nearest with ties to even,
// exactly as the rounding kernel rounds a product: leading bit, p kept bits,
// round bit, sticky bit, renormalisation on carry-out.
#include "mpcg_internal.h"

namespace mpcg {

namespace {

constexpr int ACC_LIMBS = 34;
constexpr int NARROW_LIMBS = 8;  // the first pass: components within 512 bits of each other
constexpr int NARROW_STRIDE = 9; // its LDS row stride (odd, so that lanes spread over the banks)
constexpr int CODEC_THREADS = 128;
// an exponent no converted double sum can have (theirs lie in [-1073, 1027]):
// marks an entry the first pass leaves to the second
constexpr int32_t EXP_PENDING = INT32_MIN + 1;

__device__ inline uint64_t lowbits(int n) { return n <= 0 ? 0ull : (n >= 64 ? ~0ull : ((1ull << n) - 1ull)); }

// A += m * 2^off (neg = 0) or A -= m * 2^off (neg = 1) over the limbs up to
// `top`; m < 2^53, off <= 2045, (off >> 6) + 1 <= top.
__device__ inline void acc_add(uint64_t* A, int off, uint64_t m, int neg, int top) {
  const int li = off >> 6, sh = off & 63;
  const uint64_t lo = m << sh, hi = sh ? m >> (64 - sh) : 0ull;
  const uint64_t a0 = A[li], a1 = A[li + 1];
  if (!neg) {
    const uint64_t s0 = a0 + lo, c0 = s0 < a0;
    const uint64_t s1 = a1 + hi, s1c = s1 + c0;
    uint64_t c = (s1 < a1) | (s1c < s1);
    A[li] = s0;
    A[li + 1] = s1c;
    for (int l = li + 2; c && l <= top; ++l) {
      A[l] += 1;
      c = A[l] == 0;
    }
  } else {
    const uint64_t d0 = a0 - lo, b0 = a0 < lo;
    const uint64_t d1 = a1 - hi, d1b = d1 - b0;
    uint64_t b = (a1 < hi) | (d1 < b0);
    A[li] = d0;
    A[li + 1] = d1b;
    for (int l = li + 2; b && l <= top; ++l) {
      b = A[l] == 0;
      A[l] -= 1;
    }
  }
}

__device__ inline void from_doubles_entry(const double* __restrict__ src, int rows, int ncomp, int64_t ld,
                                          int64_t plane, DOutPart out, int64_t ldo, int prec, int L, int* status,
                                          int* pending, int64_t e, uint64_t* A, bool wide);

// The marks of one call: `pending` is set by the first pass when it leaves
// an entry to the second, cleared before the first pass.
__global__ void clear_flag_kernel(int* pending) { *pending = 0; }

// Two passes over the entries: the first (WIDE = false) gives each thread an
// LDS row of NARROW_LIMBS limbs, indexed from the lowest limb its components
// touch, and marks the entries whose components span more; the second (WIDE)
// converts only those, with a row over the whole double range.
template <bool WIDE>
__global__ __launch_bounds__(CODEC_THREADS) void from_doubles_kernel(const double* __restrict__ src, int rows,
                                                                    int cols, int ncomp, int64_t ld, int64_t plane,
                                                                    DOutPart out, int64_t ldo, int prec, int L,
                                                                    int* status, int* pending) {
  constexpr int ROW = WIDE ? ACC_LIMBS : NARROW_STRIDE;
  extern __shared__ uint64_t acc_all[];
  uint64_t* A = acc_all + (size_t)threadIdx.x * ROW;
  const int64_t n = (int64_t)rows * cols;
  if (!WIDE) {
    const int64_t e = (int64_t)blockIdx.x * CODEC_THREADS + threadIdx.x;
    if (e < n) from_doubles_entry(src, rows, ncomp, ld, plane, out, ldo, prec, L, status, pending, e, A, false);
    return;
  }
  // the second pass: a small grid walking all entries, only if any was marked
  if (*reinterpret_cast<volatile int*>(pending) == 0) return;
  for (int64_t e = (int64_t)blockIdx.x * CODEC_THREADS + threadIdx.x; e < n; e += (int64_t)gridDim.x * CODEC_THREADS) {
    const int r = (int)(e % rows), j = (int)(e / rows);
    if (out.exp[(int64_t)j * ldo + r] == EXP_PENDING)
      from_doubles_entry(src, rows, ncomp, ld, plane, out, ldo, prec, L, status, pending, e, A, true);
  }
}

// One entry (wide: a row over the whole double range; else NARROW_LIMBS limbs
// from the lowest touched one, the entry marked when its span is larger).
__device__ inline void from_doubles_entry(const double* __restrict__ src, int rows, int ncomp, int64_t ld,
                                          int64_t plane, DOutPart out, int64_t ldo, int prec, int L, int* status,
                                          int* pending, int64_t e, uint64_t* A, bool wide) {
  const int r = (int)(e % rows), j = (int)(e / rows);
  const int64_t o = (int64_t)j * ldo + r;

  // the components, and the limbs they touch: the sum is formed in two's
  // complement over limbs [lo, top] (one limb above the highest touched for
  // the carries and the sign; below lo and above top it is zero or the sign)
  uint64_t mm[4];
  int pos[4], sg[4];
  int nz = 0, bad = 0, lo = ACC_LIMBS, top = 0;
  for (int c = 0; c < ncomp; ++c) {
    const uint64_t b = (uint64_t)__double_as_longlong(src[c * plane + (int64_t)j * ld + r]);
    const int ex = (int)((b >> 52) & 0x7FF);
    const uint64_t frac = b & ((1ull << 52) - 1ull);
    if (ex == 0x7FF) {  // infinity or NaN
      bad = 1;
      continue;
    }
    if (ex == 0 && frac == 0) continue;  // +0 or -0
    // a normal double is (2^52 + frac) 2^(ex - 1075), a subnormal frac 2^-1074
    mm[nz] = ex ? (frac | (1ull << 52)) : frac;
    pos[nz] = ex ? ex - 1 : 0;
    sg[nz] = (int)(b >> 63);
    lo = min(lo, pos[nz] >> 6);
    top = max(top, (pos[nz] >> 6) + 2);
    ++nz;
  }
  auto write_zero = [&]() {
    out.sign[o] = 0;
    out.exp[o] = EXP_ZERO;
    for (int l = 0; l < L; ++l) out.mant[(int64_t)l * out.ls + o] = 0;
  };
  if (bad) {
    atomicOr(status, ST_NONFINITE);
    write_zero();
    return;
  }
  if (nz == 0) {
    write_zero();
    return;
  }
  // row limb i is grid limb b0 + i; from here on limbs and bits are counted
  // in the row (the grid has no set bits below limb lo)
  const int b0 = wide ? 0 : lo;
  if (!wide && top - b0 >= NARROW_LIMBS) {
    out.exp[o] = EXP_PENDING;
    *pending = 1;
    return;
  }
  lo -= b0;
  top -= b0;
  for (int l = lo; l <= top; ++l) A[l] = 0;
  for (int i = 0; i < nz; ++i) acc_add(A, pos[i] - 64 * b0, mm[i], sg[i], top);
  const int neg = (int)(A[top] >> 63);
  if (neg) {  // magnitude: the two's complement
    uint64_t c = 1;
    for (int l = lo; l <= top; ++l) {
      const uint64_t v = ~A[l] + c;
      c = c && v == 0;
      A[l] = v;
    }
  }
  int lead = -1;
  for (int l = top; l >= lo && lead < 0; --l)
    if (A[l]) lead = 64 * l + 63 - __builtin_clzll(A[l]);
  if (lead < 0) {  // exact cancellation (or all components zero) -> +0
    write_zero();
    return;
  }
  auto limb = [&](int l) -> uint64_t { return (l >= lo && l <= top) ? A[l] : 0ull; };
  auto bit = [&](int pos) -> int { return pos < 0 ? 0 : (int)((limb(pos >> 6) >> (pos & 63)) & 1ull); };
  // bits [pos, pos + 64) of the magnitude (zero below bit 0)
  auto field = [&](int pos) -> uint64_t {
    const int li = pos >> 6, sh = pos & 63;  // floor division, also for pos < 0
    const uint64_t a = limb(li), b = limb(li + 1);
    return sh ? (a >> sh) | (b << (64 - sh)) : a;
  };
  const int low = lead - prec + 1;  // lowest kept bit
  int round_up = 0;
  if (low > 0) {
    const int rb = low - 1;
    int sticky = (limb(rb >> 6) & lowbits(rb & 63)) != 0;
    for (int l = lo; l < (rb >> 6) && !sticky; ++l) sticky = A[l] != 0;
    round_up = bit(rb) && (sticky || bit(low));
  }
  const int keep_from = 64 * L - prec;  // 0..63
  uint64_t carry = round_up ? (1ull << keep_from) : 0ull;
  int64_t e_out = (int64_t)lead + 64 * b0 + 1 - 1074;
  const int off = lead + 1 - 64 * L;
  uint64_t limbs_hi = 0;
  for (int l = 0; l < L; ++l) {
    uint64_t f = field(off + 64 * l);
    if (l == 0) f &= ~lowbits(keep_from);
    const uint64_t s = f + carry;
    carry = s < f;
    limbs_hi = s;
    if (l < L - 1) out.mant[(int64_t)l * out.ls + o] = s;
  }
  if (carry) {  // the significand rounded up to 2^p
    limbs_hi = 1ull << 63;
    e_out += 1;
  }
  out.mant[(int64_t)(L - 1) * out.ls + o] = limbs_hi;
  out.sign[o] = (uint8_t)neg;
  out.exp[o] = (int32_t)e_out;
}

}  // namespace

hipError_t launch_from_doubles(const double* src, int rows, int cols, int ncomp, int64_t ld, int64_t plane,
                               DOutPart out, int64_t ldo, int prec, int L, int* status, int* pending,
                               hipStream_t stream) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + CODEC_THREADS - 1) / CODEC_THREADS);
  clear_flag_kernel<<<dim3(1), dim3(1), 0, stream>>>(pending);
  from_doubles_kernel<false><<<dim3(blocks), dim3(CODEC_THREADS), (size_t)CODEC_THREADS * NARROW_STRIDE * 8, stream>>>(
      src, rows, cols, ncomp, ld, plane, out, ldo, prec, L, status, pending);
  const unsigned wide_blocks = blocks < 1024u ? blocks : 1024u;
  from_doubles_kernel<true><<<dim3(wide_blocks), dim3(CODEC_THREADS), (size_t)CODEC_THREADS * ACC_LIMBS * 8, stream>>>(
      src, rows, cols, ncomp, ld, plane, out, ldo, prec, L, status, pending);
  return hipGetLastError();
}

}  // namespace mpcg

namespace mpcg {

namespace {

// The opposite conversion: each stored entry (p-bit significand, L limbs) as
// ncomp doubles, greedily: component i is the double nearest (ties to even,
// with gradual underflow) to what the components before it leave of the
// value.  The remainder is kept exactly as a magnitude over the entry's limbs
// (bit 0 = 2^(exp - 64 L)) and a sign; rounding a component up leaves a
// remainder of the opposite sign.  A component beyond the largest double is
// written as infinity and reported; what remains after the last component is
// dropped (zero when the components cover the significand).
__global__ __launch_bounds__(CODEC_THREADS) void to_doubles_kernel(DPart in, int rows, int cols, int64_t ldi,
                                                                  int prec, int L, int ncomp, double* __restrict__ dst,
                                                                  int64_t ld, int64_t plane, int* status) {
  extern __shared__ uint64_t rem_all[];
  uint64_t* R = rem_all + (size_t)threadIdx.x * L;
  const int64_t e = (int64_t)blockIdx.x * CODEC_THREADS + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;  // no barrier follows
  const int r = (int)(e % rows), j = (int)(e / rows);
  const int64_t o = (int64_t)j * ldi + r;
  double* out = dst + (int64_t)j * ld + r;

  const int32_t ex = in.exp[o];
  int sgn = in.sign[o] ? 1 : 0;
  int nonzero = ex != EXP_ZERO;
  const int keep_from = 64 * L - prec;
  for (int l = 0; l < L; ++l) {
    uint64_t v = nonzero ? in.mant[(int64_t)l * in.ls + o] : 0ull;
    if (l == 0) v &= ~lowbits(keep_from);  // only the top prec bits are the value
    R[l] = v;
  }
  const int64_t base = nonzero ? (int64_t)ex - 64 * L : 0;  // exponent of grid bit 0
  auto limb = [&](int l) -> uint64_t { return (l >= 0 && l < L) ? R[l] : 0ull; };
  // bits [pos, pos + 64) of the remainder (zero outside its limbs)
  auto field = [&](int pos) -> uint64_t {
    const int li = pos >> 6, sh = pos & 63;  // floor division, also for pos < 0
    const uint64_t x = limb(li), y = limb(li + 1);
    return sh ? (x >> sh) | (y << (64 - sh)) : x;
  };
  for (int c = 0; c < ncomp; ++c) {
    int lead = -1;
    for (int l = L - 1; l >= 0 && lead < 0 && nonzero; --l)
      if (R[l]) lead = 64 * l + 63 - __builtin_clzll(R[l]);
    if (lead < 0) {  // nothing left: +0
      out[c * plane] = 0.0;
      nonzero = 0;
      continue;
    }
    // kept bits [low, lead]: at most 53, none below 2^-1074 (gradual underflow);
    // a remainder below 2^-1075 rounds to zero
    const int64_t sub = -1074 - base;  // grid position of 2^-1074
    const int64_t low64 = max((int64_t)lead - 52, sub);
    int low, up = 0;
    uint64_t T = 0;
    if (low64 > lead + 1) {
      low = lead + 2;
    } else {
      low = (int)low64;  // >= lead - 52 >= -52 when rounding a nonzero remainder
      T = field(low) & lowbits(lead - low + 1);
      const int rb = low - 1;
      int sticky = 0;
      if (rb > 0) {
        sticky = (limb(rb >> 6) & lowbits(rb & 63)) != 0;
        for (int l = 0; l < (rb >> 6) && !sticky; ++l) sticky = R[l] != 0;
      }
      up = (rb >= 0 && ((limb(rb >> 6) >> (rb & 63)) & 1ull)) && (sticky || (T & 1ull));
    }
    const uint64_t q = T + (uint64_t)up;  // <= 2^53
    const int64_t qexp = base + low;        // the component is q 2^qexp
    double d = 0.0;
    if (q != 0) {
      if (qexp + 63 - __builtin_clzll(q) > 1023) {
        d = __builtin_huge_val();
        atomicOr(status, ST_OUT_RANGE);
      } else {
        d = ldexp((double)q, (int)qexp);
      }
    }
    out[c * plane] = sgn ? -d : d;
    // the remainder: its bits below `low`, or 2^low minus them (and the
    // opposite sign) when the component was rounded up
    if (low < 64 * L) {
      for (int l = max(low, 0) >> 6; l < L; ++l) {
        const int keep = low - 64 * l;  // bits of limb l below `low`
        R[l] &= keep >= 64 ? ~0ull : lowbits(keep);
      }
      if (up) {
        uint64_t borrow = 0;
        for (int l = 0; l < L; ++l) {
          const uint64_t v = R[l], t = 0ull - v - borrow;
          borrow = (v | borrow) != 0;
          const int keep = low - 64 * l;
          R[l] = t & (keep >= 64 ? ~0ull : lowbits(keep));
        }
        sgn ^= 1;
      }
    }
  }
}

}  // namespace

hipError_t launch_to_doubles(DPart in, int rows, int cols, int64_t ldi, int prec, int L, int ncomp, double* dst,
                             int64_t ld, int64_t plane, int* status, hipStream_t stream) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return hipSuccess;
  const size_t lds = (size_t)CODEC_THREADS * L * sizeof(uint64_t);
  const unsigned blocks = (unsigned)((n + CODEC_THREADS - 1) / CODEC_THREADS);
  to_doubles_kernel<<<dim3(blocks), dim3(CODEC_THREADS), lds, stream>>>(in, rows, cols, ldi, prec, L, ncomp, dst,
                                                                        ld, plane, status);
  return hipGetLastError();
}

}  // namespace mpcg
