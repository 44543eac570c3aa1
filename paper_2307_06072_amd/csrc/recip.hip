// The reciprocal of a complex multi-precision number, correctly rounded in
// each component: for y = a + ib, 1/y = a/(a^2 + b^2) - i b/(a^2 + b^2), and
// each of the two real components is rounded once to p bits, to nearest, ties
// to even (the division of MPC arithmetic, Sec. II, used by the blocked LU of
// Sec. IV-B for its pivots).
//
// Each component is an exact quotient of integers.  With a = A 2^(ea - p),
// b = B 2^(eb - p) (A, B the p-bit significands as integers) and e = min(ea, eb):
//   a^2 + b^2 = 2^(2e - 2p) D,   D = A^2 2^(2(ea - e)) + B^2 2^(2(eb - e)),
//   Re(1/y) = +-A 2^(ea - 2e + p) / D,   Im(1/y) = -+B 2^(eb - 2e + p) / D.
// The quotient N 2^s / D is formed by long division (Knuth's Algorithm D on
// 32-bit words) with s chosen so that it has p + 2 or p + 3 bits; its low
// bits and the remainder decide the rounding exactly.
//
// When the exponents of a and b differ by Delta >= (3p + 6)/2, the smaller
// part's square is dropped: with a the larger, Re(1/y) = (1/a)(1 - eps) and
// Im(1/y) = -(b/a^2)(1 - eps) with 0 < eps < 2^(2 - 2 Delta) <= 2^(-3p-4).
// The quotient of the dropped form, Q + R/D, then moves by less than one unit
// of its last place (it is below 2^(p+3) and its denominator below 2^(2p)),
// and by less than R/D when R > 0; so the exact value lies in (Q, Q + 1)
// when R > 0 and in (Q - 1, Q) when R = 0, which fixes the rounding (the
// sticky bit is set either way).  This bounds D to 5p + 7 bits.
//
// One thread per real component (two per entry), the integers in that
// thread's part of LDS.
#include <algorithm>

#include "mpcg_internal.h"

namespace mpcg {
namespace recip {

// Words (32-bit) of one thread's workspace at precision p.
__host__ __device__ inline int words_d(int p) { return (5 * p + 7 + 31) / 32 + 1; }
__host__ __device__ inline int words_u(int p) { return (6 * p + 71 + 31) / 32 + 1; }
__host__ __device__ inline int words_q(int p) { return (p + 2 + 31) / 32 + 2; }
__host__ __device__ inline int words_total(int p) { return words_d(p) + words_u(p) + words_q(p); }

__host__ __device__ inline int bitlen(const uint32_t* x, int n) {
  for (int i = n - 1; i >= 0; --i)
    if (x[i]) return 32 * i + 32 - __builtin_clz(x[i]);
  return 0;
}

__host__ __device__ inline void zero_words(uint32_t* x, int n) {
  for (int i = 0; i < n; ++i) x[i] = 0;
}

// Bit i of x (n words); 0 outside.
__host__ __device__ inline uint32_t bit_at(const uint32_t* x, int n, int64_t i) {
  if (i < 0 || i >= 32 * (int64_t)n) return 0;
  return (x[i >> 5] >> (i & 31)) & 1u;
}

// 32 bits of x starting at bit pos (pos may be negative; bits outside x are 0).
__host__ __device__ inline uint32_t window32(const uint32_t* x, int n, int64_t pos) {
  const int64_t w = pos >> 5;  // floor division
  const int b = (int)(pos & 31);
  const uint32_t lo = (w >= 0 && w < n) ? x[w] : 0u;
  if (b == 0) return lo;
  const uint32_t hi = (w + 1 >= 0 && w + 1 < n) ? x[w + 1] : 0u;
  return (lo >> b) | (hi << (32 - b));
}

// x[0, nw) := the top p bits of the L-limb significand at mant[l * ls] (an
// integer below 2^p).
__host__ __device__ inline void load_top_bits(const uint64_t* mant, int64_t ls, int L, int p, uint32_t* x, int nw) {
  const int r = 64 * L - p;  // bits below the p kept ones
  for (int w = 0; w < nw; ++w) {
    const int pos = r + 32 * w;  // bit of the L-limb integer
    const int li = pos >> 6, off = pos & 63;
    const uint64_t lo = li < L ? mant[li * ls] : 0;
    const uint64_t hi = li + 1 < L ? mant[(li + 1) * ls] : 0;
    const uint64_t v = off ? (lo >> off) | (hi << (64 - off)) : lo;
    x[w] = (uint32_t)v;
  }
  // bits at or above p are zero: the significand has 64 L bits
}

// P[0, 2 nx) := X^2.
__host__ __device__ inline void square(const uint32_t* X, int nx, uint32_t* P) {
  zero_words(P, 2 * nx);
  for (int i = 0; i < nx; ++i) {
    uint64_t carry = 0;
    const uint64_t xi = X[i];
    for (int j = 0; j < nx; ++j) {
      const uint64_t t = xi * X[j] + P[i + j] + carry;
      P[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    P[i + nx] = (uint32_t)carry;
  }
}

// D[0, nd) += P[0, np) * 2^sh (the sum must fit nd words).
__host__ __device__ inline void add_shifted(uint32_t* D, int nd, const uint32_t* P, int np, int64_t sh) {
  const int64_t ws = sh >> 5;
  uint64_t carry = 0;
  for (int64_t k = ws; k < nd; ++k) {
    const uint32_t v = window32(P, np, 32 * (k - ws) - (sh & 31));
    if (v == 0 && carry == 0 && k > ws + np) break;
    const uint64_t t = (uint64_t)D[k] + v + carry;
    D[k] = (uint32_t)t;
    carry = t >> 32;
  }
}

// U[0, nu) := X[0, nx) * 2^sh.
__host__ __device__ inline void set_shifted(uint32_t* U, int nu, const uint32_t* X, int nx, int64_t sh) {
  for (int k = 0; k < nu; ++k) U[k] = window32(X, nx, 32 * (int64_t)k - sh);
}

// Knuth's Algorithm D: Q[0, nu - nv) := floor(U / V), U[0, nv) := the
// remainder (scaled by the normalising shift, which the caller applied to
// both).  Needs nv >= 2, V[nv-1] with its top bit set, U[nu-1] < V[nv-1].
__host__ __device__ inline void divide(uint32_t* U, int nu, const uint32_t* V, int nv, uint32_t* Q) {
  const uint64_t B = 1ull << 32;
  const uint64_t vt = V[nv - 1], vs = V[nv - 2];
  for (int j = nu - nv - 1; j >= 0; --j) {
    const uint64_t num = ((uint64_t)U[j + nv] << 32) | U[j + nv - 1];
    uint64_t qh = num / vt;
    uint64_t rh = num - qh * vt;
    while (qh >= B || qh * vs > ((rh << 32) | U[j + nv - 2])) {
      --qh;
      rh += vt;
      if (rh >= B) break;
    }
    // U[j, j + nv] -= qh * V
    uint64_t carry = 0;
    uint32_t borrow = 0;
    for (int i = 0; i < nv; ++i) {
      const uint64_t prod = qh * V[i] + carry;
      carry = prod >> 32;
      const uint32_t pl = (uint32_t)prod, ui = U[i + j];
      const uint32_t d1 = ui - pl;
      const uint32_t b1 = ui < pl;
      const uint32_t d2 = d1 - borrow;
      const uint32_t b2 = d1 < borrow;
      U[i + j] = d2;
      borrow = b1 + b2;
    }
    const uint64_t sub = carry + borrow;
    const uint64_t top = U[j + nv];
    U[j + nv] = (uint32_t)(top - sub);
    if (top < sub) {  // qh was one too large: add V back
      --qh;
      uint64_t c = 0;
      for (int i = 0; i < nv; ++i) {
        const uint64_t t = (uint64_t)U[i + j] + V[i] + c;
        U[i + j] = (uint32_t)t;
        c = t >> 32;
      }
      U[j + nv] += (uint32_t)c;
    }
    Q[j] = (uint32_t)qh;
  }
}

// D[0, nd) <<= sh (0 <= sh < 32), in place.
__host__ __device__ inline void shl_small(uint32_t* D, int nd, int sh) {
  if (sh == 0) return;
  for (int i = nd - 1; i > 0; --i) D[i] = (D[i] << sh) | (D[i - 1] >> (32 - sh));
  D[0] <<= sh;
}

// The rounding of (N 2^z / D)(1 - eps), eps = 0 (below = 0) or a positive
// amount too small to move the quotient by one unit (below = 1), to p bits.
// N[0, nn) and D[0, nd) hold the integers; U and Q are scratch of
// words_u(p) and words_q(p) words; D is scaled in place.  The p-bit
// significand is written into limbs[l * ls], l < L.
__host__ __device__ inline int64_t rne_quotient(const uint32_t* N, int nn, uint32_t* D, int nd, int64_t z,
                                                int below, int p, uint32_t* U, uint32_t* Q, uint64_t* limbs,
                                                int64_t ls, int L) {
  const int bn = bitlen(N, nn);
  const int bd = bitlen(D, nd);
  // N 2^s / D lies in [2^(p+1), 2^(p+3))
  const int64_t s = (int64_t)p + 2 + bd - bn;
  int nv = (bd + 31) / 32;
  int extra = 0;  // Algorithm D needs two divisor words
  if (nv < 2) {
    extra = 32;
    nv = 2;
  }
  const int norm = __builtin_clz(D[(bd - 1) / 32]) & 31;  // top bit of the top word set after the shift
  // D := D 2^(norm + extra)
  if (extra) {
    D[1] = D[0];
    D[0] = 0;
  }
  shl_small(D, nv, norm);
  const int64_t ubits = bn + s + norm + extra;
  const int nu = (int)((ubits + 31) / 32) + 1;
  set_shifted(U, nu, N, nn, s + norm + extra);
  const int nq = nu - nv;
  divide(U, nu, D, nv, Q);
  int rem = 0;
  for (int i = 0; i < nv; ++i) rem |= U[i] != 0;
  int sticky = rem;
  if (below && !rem) {  // the exact value lies just below the integer Q
    for (int i = 0; i < nq; ++i) {
      const uint32_t w = Q[i];
      Q[i] = w - 1;
      if (w != 0) break;
    }
    sticky = 1;
  }
  const int lq = bitlen(Q, nq);  // p + 1 .. p + 3
  const int k = lq - p;          // bits below the kept p
  const uint32_t rbit = bit_at(Q, nq, k - 1);
  for (int i = 0; i < k - 1 && !sticky; ++i) sticky |= bit_at(Q, nq, i);
  const uint32_t lsb = bit_at(Q, nq, k);
  // limbs := (Q >> k) << (64 L - p), the bits below p cleared
  const int64_t off = (int64_t)k - (64 * (int64_t)L - p);  // bit of Q at bit 0 of the limbs
  const int r = 64 * L - p;
  for (int l = 0; l < L; ++l) {
    uint64_t v = (uint64_t)window32(Q, nq, off + 64 * l) | ((uint64_t)window32(Q, nq, off + 64 * l + 32) << 32);
    const int lo = 64 * l;  // clear bits below r
    if (lo + 64 <= r) v = 0;
    else if (lo < r) v &= ~0ull << (r - lo);
    limbs[l * ls] = v;
  }
  int64_t e = (int64_t)lq + z - s;  // value = (Q / 2^lq) 2^e before rounding
  if (rbit && (sticky || lsb)) {
    // add one unit in the last place, 2^r in the limbs
    int carry = 1;
    uint64_t inc = 1ull << (r & 63);
    for (int l = r / 64; l < L; ++l) {
      const uint64_t v = limbs[l * ls];
      const uint64_t t = v + inc;
      limbs[l * ls] = t;
      if (t >= v) {
        carry = 0;
        break;
      }
      inc = 1;
    }
    if (carry) {  // carried out of the top: 2^p -> 2^(p-1), exponent + 1
      limbs[(L - 1) * ls] = 1ull << 63;
      e += 1;
    }
  }
  return e;
}

// One component (comp 0: Re, 1: Im) of the reciprocal of entry (yre, yim)
// at index yi, written to index xi of out.  W: this thread's workspace.
__host__ __device__ inline void component(DPart yre, DPart yim, int64_t yi, DOutPart out, int64_t xi, int comp, int p,
                                          int L, uint32_t* W) {
  uint32_t* D = W;
  uint32_t* U = D + words_d(p);
  uint32_t* Q = U + words_u(p);
  const int np = (p + 31) / 32;
  const int32_t ea0 = yre.exp[yi], eb0 = yim.exp[yi];
  // magnitudes as p-bit integers; a zero significand counts as zero
  int za = ea0 == EXP_ZERO, zb = eb0 == EXP_ZERO;
  if (!za) {
    load_top_bits(yre.mant + yi, yre.ls, L, p, Q, np);
    za = bitlen(Q, np) == 0;
  }
  if (!zb) {
    load_top_bits(yim.mant + yi, yim.ls, L, p, Q, np);
    zb = bitlen(Q, np) == 0;
  }
  const int64_t ea = ea0, eb = eb0;
  const int own_zero = comp == 0 ? za : zb;
  if (own_zero || (za && zb)) {  // Re(1/y) = 0 when a = 0, Im(1/y) = 0 when b = 0
    out.sign[xi] = 0;
    out.exp[xi] = EXP_ZERO;
    for (int l = 0; l < L; ++l) out.mant[l * out.ls + xi] = 0;
    return;
  }
  const uint32_t sgn = comp == 0 ? (yre.sign[yi] & 1u) : ((yim.sign[yi] & 1u) ^ 1u);
  zero_words(D, words_d(p));
  uint32_t* N = Q;  // the numerator sits in Q's words until the division reads it into U
  int nn = np;
  int64_t z;
  int below = 0;
  // the magnitude of the other part, if it matters
  const int64_t delta = ea - eb;
  const int other_zero = comp == 0 ? zb : za;
  const int64_t eown = comp == 0 ? ea : eb;
  const int64_t wide = 2 * (delta < 0 ? -delta : delta) >= 3 * (int64_t)p + 6;
  const DPart own = comp == 0 ? yre : yim, oth = comp == 0 ? yim : yre;
  if (other_zero || (wide && (comp == 0 ? delta > 0 : delta < 0))) {
    // 1/own, exactly (the other part is zero) or just below it
    load_top_bits(own.mant + yi, own.ls, L, p, D, np);  // D := own significand
    zero_words(N, words_q(p));
    N[0] = 1;
    nn = 1;
    z = p - eown;
    below = !other_zero;
  } else if (wide) {
    // own part far below the other: own / other^2, just below it
    load_top_bits(oth.mant + yi, oth.ls, L, p, Q, np);
    square(Q, np, U);  // other^2 into U's words
    for (int i = 0; i < 2 * np; ++i) D[i] = U[i];
    load_top_bits(own.mant + yi, own.ls, L, p, N, np);
    const int64_t eoth = comp == 0 ? eb : ea;
    z = eown - 2 * eoth + p;
    below = 1;
  } else {
    // exact: D = A^2 2^(2(ea - e)) + B^2 2^(2(eb - e)), e = min(ea, eb)
    const int64_t e = ea < eb ? ea : eb;
    load_top_bits(yre.mant + yi, yre.ls, L, p, Q, np);
    square(Q, np, U);
    add_shifted(D, words_d(p), U, 2 * np, 2 * (ea - e));
    load_top_bits(yim.mant + yi, yim.ls, L, p, Q, np);
    square(Q, np, U);
    add_shifted(D, words_d(p), U, 2 * np, 2 * (eb - e));
    load_top_bits(own.mant + yi, own.ls, L, p, N, np);
    z = eown - 2 * e + p;
  }
  // N (in Q's words) is read into U before the division writes Q
  const int nd = words_d(p);
  const int64_t e = rne_quotient(N, nn, D, nd, z, below, p, U, Q, out.mant + xi, out.ls, L);
  out.sign[xi] = (uint8_t)sgn;
  out.exp[xi] = (int32_t)e;
}

}  // namespace recip

namespace {

__global__ void recip_kernel(DPart yre, DPart yim, int64_t stride, DOutPart xre, DOutPart xim, int prec, int L,
                             int count, int per_block) {
  extern __shared__ uint32_t lds[];
  const int t = threadIdx.x;
  const int entry = blockIdx.x * per_block + t / 2;
  if (t >= 2 * per_block || entry >= count) return;
  const int comp = t & 1;
  uint32_t* W = lds + (size_t)t * recip::words_total(prec);
  recip::component(yre, yim, (int64_t)entry * stride, comp ? xim : xre, entry, comp, prec, L, W);
}

}  // namespace

hipError_t launch_lu_recip(DPart yre, DPart yim, int64_t stride, DOutPart xre, DOutPart xim, int prec, int L,
                           int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const size_t per_thread = 4 * (size_t)recip::words_total(prec);
  int per_block = (int)std::min<size_t>(32, (64 * 1024) / (2 * per_thread));
  if (per_block < 1) per_block = 1;
  const unsigned blocks = (unsigned)((count + per_block - 1) / per_block);
  const size_t lds = 2 * per_block * per_thread;
  recip_kernel<<<blocks, 64, lds, stream>>>(yre, yim, stride, xre, xim, prec, L, count, per_block);
  return hipGetLastError();
}

}  // namespace mpcg
