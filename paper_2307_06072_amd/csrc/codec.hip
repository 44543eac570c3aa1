// Multi-component fixed-precision inputs (double-double, triple-double,
// quad-double: the multi-component arithmetic named as future work in the
// paper's concluding section) turned into the library's number format.
//
// Each entry of a real component is the exact sum of up to four doubles.  A
// thread forms that sum exactly in a two's-complement fixed-point
// accumulator spanning the whole double range: bit 0 is 2^-1074 (the lowest
// subnormal bit), the largest finite double's top bit is bit 2097, so four
// of them stay below bit 2100, and 34 limbs (2176 bits) leave the top bit
// for the sign.  The sum is then rounded once to prec_bits, to nearest with
// ties to even, exactly as the rounding kernel rounds a product: leading bit,
// p kept bits, round bit, sticky bit, renormalisation on carry-out.
#include "mpcg_internal.h"

namespace mpcg {

namespace {

constexpr int ACC_LIMBS = 34;
constexpr int CODEC_THREADS = 128;

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

__global__ __launch_bounds__(CODEC_THREADS) void from_doubles_kernel(const double* __restrict__ src, int rows,
                                                                    int cols, int ncomp, int64_t ld, int64_t plane,
                                                                    DOutPart out, int64_t ldo, int prec, int L,
                                                                    int* status) {
  extern __shared__ uint64_t acc_all[];
  uint64_t* A = acc_all + (size_t)threadIdx.x * ACC_LIMBS;
  const int64_t e = (int64_t)blockIdx.x * CODEC_THREADS + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;  // no barrier follows
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
  for (int l = lo; l <= top; ++l) A[l] = 0;
  for (int i = 0; i < nz; ++i) acc_add(A, pos[i], mm[i], sg[i], top);
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
  int64_t e_out = (int64_t)lead + 1 - 1074;
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
                               DOutPart out, int64_t ldo, int prec, int L, int* status, hipStream_t stream) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return hipSuccess;
  const size_t lds = (size_t)CODEC_THREADS * ACC_LIMBS * sizeof(uint64_t);
  const unsigned blocks = (unsigned)((n + CODEC_THREADS - 1) / CODEC_THREADS);
  from_doubles_kernel<<<dim3(blocks), dim3(CODEC_THREADS), lds, stream>>>(src, rows, cols, ncomp, ld, plane, out,
                                                                          ldo, prec, L, status);
  return hipGetLastError();
}

}  // namespace mpcg
