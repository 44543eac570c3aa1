// Exact accumulation tail and the single rounding.
//
// For every output component the slice GEMM leaves an exact integer
//     X = T * 2^(w*nd) + sum_{d=0}^{Dmax} n_d * 2^(w*(Dmax-d)),   0 <= n_d < 2^w,
// (T the signed final carry, nd = Dmax + 1) whose value is
// X * 2^(G_i + H_j - w(Dmax + 2)).  Algorithm 2 adds its slice products into an
// L-bit floating-point accumulator; here the sum is already exact, and this
// kernel rounds it once to prec_bits, to nearest with ties to even.
//
// If the contraction was cut into chunks, their streams are first added
// digit by digit with a carry (the sum is written back into chunk 0's digits).
//
// For negative X the magnitude is formed digit-wise without materialising it:
// with z = the lowest nonzero digit index (largest d),
//     |X| digits = 2^w - 1 - n_d above z,  2^w - n_z at z,  0 below z,
// and top part -T - 1 (or -T when all digits are zero).
// Sticky information needs only the position of the lowest set bit of X,
// which is the same for X and |X|.
#include <algorithm>
#include <cstring>

#include "mpcg_internal.h"

namespace mpcg {

namespace {

constexpr uint64_t DFULL = 1ull << I8_W;  // the INT8 digit base

template <typename DIG>
struct Stream {
  const DIG* base;  // digit d of this element: base[d * 512]
  int Dmax, w;
  int neg;
  int z;        // lowest nonzero digit index (largest d), -1 if none
  uint64_t U;   // magnitude of the top part
  __device__ inline uint64_t n(int d) const { return (uint64_t)base[(size_t)d * 512]; }
  __device__ inline uint64_t m(int d) const {  // magnitude digit
    if (!neg) return n(d);
    if (z < 0 || d > z) return 0;
    const uint64_t full = 1ull << w;
    return d == z ? full - n(d) : full - 1 - n(d);
  }
  // bits [pos, pos + 64) of |X|; bit 0 = lowest bit of digit Dmax
  __device__ uint64_t field(int64_t pos) const {
    const int64_t nbits = (int64_t)w * (Dmax + 1);
    uint64_t r = 0;
    const int64_t lo = pos < 0 ? 0 : pos;
    const int64_t hi = pos + 64;  // exclusive
    if (lo < nbits) {
      const int64_t q0 = lo / w;
      const int64_t q1 = min((hi - 1) / w, (int64_t)Dmax);
      for (int64_t q = q0; q <= q1; ++q) {
        const uint64_t v = m(Dmax - (int)q);
        const int64_t sh = (int64_t)w * q - pos;
        if (sh >= 0) {
          if (sh < 64) r |= v << sh;
        } else if (-sh < 64) {
          r |= v >> (-sh);
        }
      }
    }
    if (hi > nbits && U) {
      const int64_t sh = nbits - pos;
      if (sh >= 0) {
        if (sh < 64) r |= U << sh;
      } else if (-sh < 64) {
        r |= U >> (-sh);
      }
    }
    return r;
  }
  __device__ inline int bit(int64_t pos) const {
    if (pos < 0) return 0;
    const int64_t nbits = (int64_t)w * (Dmax + 1);
    if (pos >= nbits) {
      const int64_t s = pos - nbits;
      return s < 64 ? (int)((U >> s) & 1) : 0;
    }
    const int64_t q = pos / w;
    return (int)((m(Dmax - (int)q) >> (pos - q * w)) & 1);
  }
};

// Thread gid handles digit byte (gid mod 512) of tile gid / 512: lane
// (gid mod 512) / 8 and slot gid mod 8 of the slice GEMM's output order, so a
// wavefront reads 64 consecutive bytes of every digit row.
template <typename DIG>
__device__ inline void round_element(const RoundArgs& a, int64_t gid) {
  const int tiles = a.mt * a.nt;
  if (gid >= (int64_t)tiles * 512) return;
  const int tile = (int)(gid >> 9);
  const int lane = (int)(gid >> 3) & 63, slot = (int)gid & 7;
  const int comp = slot >> 2;
  const int jj = lane & 15;
  // INT8 order: lane = jj + 16 (ii / 4), slot = 4 comp + ii % 4;
  // FP64 order: lane = jj + 16 (ii % 4), slot = 4 comp + ii / 4
  const int ii = a.f64_layout ? (lane >> 4) + 4 * (slot & 3) : 4 * (lane >> 4) + (slot & 3);
  const int ti = tile % a.mt, tj = tile / a.mt;
  const int i = ti * 16 + ii, j = tj * 16 + jj;
  if (i >= a.m || j >= a.n) return;
  const int nd = a.Dmax + 1;
  const int w = a.w;

  DIG* digits = reinterpret_cast<DIG*>(const_cast<void*>(a.digits));
  DIG* d0 = digits + ((size_t)tile * nd * 64 + lane) * 8 + slot;
  const size_t tb0 = ((size_t)tile * 64 + lane) * 8 + slot;

  int64_t T;
  int z;
  if (a.ksplit == 1) {
    T = a.top[tb0];
    z = a.lnz[tb0];
  } else {
    // add the chunk streams exactly, least significant digit first
    const uint64_t dmask = (1ull << w) - 1;
    const size_t sstride = (size_t)tiles * nd * 64 * 8;
    int64_t c = 0;
    z = -1;
    for (int d = a.Dmax; d >= 0; --d) {
      int64_t s = c;
      for (int q = 0; q < a.ksplit; ++q) s += (int64_t)d0[q * sstride + (size_t)d * 512];
      const uint64_t nd_ = (uint64_t)s & dmask;
      c = s >> w;
      d0[(size_t)d * 512] = (DIG)nd_;
      if (nd_ && z < 0) z = d;
    }
    T = c;
    for (int q = 0; q < a.ksplit; ++q) T += a.top[(size_t)q * tiles * 64 * 8 + tb0];
  }

  DOutPart out = comp ? a.cim : a.cre;
  const int64_t o = (int64_t)j * a.ldc + i;
  const int L = a.L, p = a.prec;

  if (T == 0 && z < 0) {  // exact zero -> +0
    out.sign[o] = 0;
    out.exp[o] = EXP_ZERO;
    for (int l = 0; l < L; ++l) out.mant[(int64_t)l * out.ls + o] = 0;
    return;
  }

  Stream<DIG> st;
  st.base = d0;
  st.Dmax = a.Dmax;
  st.w = w;
  st.neg = T < 0;
  st.z = z;
  if (!st.neg)
    st.U = (uint64_t)T;
  else
    st.U = (z < 0) ? (uint64_t)(-T) : (uint64_t)(-T - 1);

  const int64_t nbits = (int64_t)w * nd;
  // leading bit of |X|
  int64_t lead;
  if (st.U) {
    lead = nbits + 63 - __builtin_clzll(st.U);
  } else {
    lead = -1;
    for (int d = 0; d <= a.Dmax; ++d) {
      const uint64_t v = st.m(d);
      if (v) {
        lead = (int64_t)w * (a.Dmax - d) + 63 - __builtin_clzll(v);
        break;
      }
    }
  }
  // lowest set bit of X (= of |X|)
  int64_t lowset;
  if (z >= 0)
    lowset = (int64_t)w * (a.Dmax - z) + __builtin_ctzll(st.n(z));
  else
    lowset = nbits + __builtin_ctzll((uint64_t)T);

  const int64_t low = lead - p + 1;  // lowest kept bit of |X|
  int round_up = 0;
  if (low > 0) {
    const int rbit = st.bit(low - 1);
    const int sticky = lowset < low - 1;
    const int lsb = st.bit(low);
    round_up = rbit && (sticky || lsb);
  }
  // significand limbs, least significant first, with the rounding increment
  const int64_t off = lead + 1 - 64ll * L;
  const int keep_from = 64 * L - p;  // 0..63
  uint64_t carry = round_up ? (1ull << keep_from) : 0;
  int64_t e_out = lead + 1 + (int64_t)a.G[i] + (int64_t)a.H[j] - (int64_t)w * (a.Dmax + 2);
  uint64_t limbs_hi = 0;
  bool overflow = false;
  // first pass decides nothing further; write limbs as we go
  for (int l = 0; l < L; ++l) {
    uint64_t f = st.field(off + 64ll * l);
    if (l == 0 && keep_from) f &= ~((1ull << keep_from) - 1ull);
    const uint64_t s = f + carry;
    carry = (s < f) ? 1 : 0;
    limbs_hi = s;
    if (l < L - 1) out.mant[(int64_t)l * out.ls + o] = s;
  }
  if (carry) {  // significand overflowed to 2^p: 2^(p-1) with exponent + 1
    overflow = true;
    limbs_hi = 1ull << 63;
    e_out += 1;
  }
  (void)overflow;
  if (e_out > INT32_MAX || e_out <= (int64_t)INT32_MIN) {
    atomicOr(a.status, ST_OUT_RANGE);
    out.sign[o] = 0;
    out.exp[o] = EXP_ZERO;
    for (int l = 0; l < L; ++l) out.mant[(int64_t)l * out.ls + o] = 0;
    return;
  }
  out.mant[(int64_t)(L - 1) * out.ls + o] = limbs_hi;
  out.sign[o] = (uint8_t)st.neg;
  out.exp[o] = (int32_t)e_out;
}

template <typename DIG>
__global__ __launch_bounds__(256) void round_kernel(RoundArgs a) {
  round_element<DIG>(a, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

__global__ void zero_kernel(DOutPart cre, DOutPart cim, int m, int n, int64_t ldc, int L) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)m * n * 2;
  if (gid >= total) return;
  const int i = (int)(gid % m);
  const int64_t rest = gid / m;
  const int j = (int)(rest % n);
  DOutPart out = (rest / n) ? cim : cre;
  const int64_t o = (int64_t)j * ldc + i;
  out.sign[o] = 0;
  out.exp[o] = EXP_ZERO;
  for (int l = 0; l < L; ++l) out.mant[(int64_t)l * out.ls + o] = 0;
}

__global__ void fill_zero_kernel(uint32_t* p, size_t n32) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n32) p[i] = 0;
}

// dst[0, w.n) := w.v[0, w.n): host data carried in the kernel's arguments
// (a graph keeps its own copy of them at capture).
__global__ void store_words_kernel(uint32_t* dst, StoreWords w) {
  for (uint32_t i = threadIdx.x; i < w.n; i += blockDim.x) dst[i] = w.v[i];
}

// ---- INT8 digits: chunked per component --------------------------------------
//
// Digit q = Dmax - d of a component lives at chunk q / 16, byte q % 16 of its
// own 16-byte words ([slot][chunk][lane][16], 1 KB per chunk and slot), so a
// thread reads its digits 16 at a time.  A block is one (tile, component):
// 256 threads, thread t holds element (ii, jj) = (t % 16, t / 16), so the
// stores of a wavefront cover 16 consecutive rows of 4 columns.  The bits
// the p-bit result depends on (one word below the lowest bit of limb 0 up to
// the leading bit) are packed from the digits into binary 64-bit words in the
// thread's part of LDS, and the limbs, round bit and tie bit are read there.

struct Win8 {
  const uint8_t* glob; // the component's stream (digit q at glob[(q >> 4) * 1024 + (q & 15)])
  int Dmax, neg, z;    // z: lowest nonzero digit as an index d (largest d), -1 if none
  uint64_t U;
  __device__ inline uint64_t gn(int q) const { return glob[(size_t)(q >> 4) * 1024 + (q & 15)]; }
  // bits [pos, pos + 64) of |X| read from the digit stream (any position):
  // the at most 10 digits come from at most two 16-digit chunks, loaded whole
  __device__ uint64_t fieldg(int64_t pos) const {
    const int64_t nbits = (int64_t)I8_W * (Dmax + 1);
    uint64_t r = 0;
    const int64_t lo = pos < 0 ? 0 : pos;
    const int64_t hi = pos + 64;
    if (lo < nbits) {
      const int q0 = (int)(lo / I8_W);
      const int q1 = (int)min((hi - 1) / I8_W, (int64_t)Dmax);
      const int c0 = q0 >> 4;
      const uint4 v0 = *reinterpret_cast<const uint4*>(glob + (size_t)c0 * 1024);
      const uint4 v1 = (q1 >> 4) != c0 ? *reinterpret_cast<const uint4*>(glob + (size_t)(c0 + 1) * 1024) : v0;
      for (int q = q0; q <= q1; ++q) {
        const uint4 cv = (q >> 4) == c0 ? v0 : v1;
        const int b = q & 15;
        const uint32_t w = b < 8 ? (b < 4 ? cv.x : cv.y) : (b < 12 ? cv.z : cv.w);
        const uint64_t raw = (w >> (8 * (b & 3))) & 255u;
        const int d = Dmax - q;
        const uint64_t v = !neg ? raw : ((z < 0 || d > z) ? 0ull : (d == z ? DFULL - raw : DFULL - 1 - raw));
        const int64_t sh = (int64_t)I8_W * q - pos;
        if (sh >= 0) {
          if (sh < 64) r |= v << sh;
        } else if (-sh < 64) {
          r |= v >> (-sh);
        }
      }
    }
    if (hi > nbits && U) {
      const int64_t sh = nbits - pos;
      if (sh >= 0) {
        if (sh < 64) r |= U << sh;
      } else if (-sh < 64) {
        r |= U >> (-sh);
      }
    }
    return r;
  }
};

__device__ inline uint64_t lowmask(int64_t n) { return n <= 0 ? 0ull : (n >= 64 ? ~0ull : ((1ull << n) - 1ull)); }
__device__ inline uint64_t rangemask(int64_t a, int64_t b) { return lowmask(b) & ~lowmask(a); }  // bits [a, b)

// Bits [xw0, xw0 + 64 nx) of |X| in binary, as the words Xw[0 .. nx).  One
// pass over the 16-digit chunks of the stream: four digits (one 32-bit word
// of a chunk, already packed since a digit fills its byte) at a time are collected in a
// two-word register window, and each word is stored once, low to high.  For
// negative X the digit bits of the range are the two's complement of the
// digit integer: inverted, plus the +1 carried up from below its lowest set
// bit (low_x), which enters here when low_x lies in or above the range.  The
// top U lies above the digits.
__device__ __attribute__((always_inline)) inline void build_xwin(const Win8 st, int64_t xw0, int nx, int64_t low_x, uint64_t* Xw) {
  const int64_t nbits = (int64_t)I8_W * (st.Dmax + 1);
  const int64_t wlo = max(xw0, (int64_t)0), whi = min(xw0 + 64ll * nx, nbits);
  const bool digits = wlo < whi && !(st.neg && st.z < 0);
  const bool inv = digits && st.neg;
  const int64_t ra = wlo - xw0, rb = whi - xw0;  // the digit bits within the window
  const int wplus = inv && low_x >= wlo ? (int)(ra >> 6) : -1;
  int w = 0;                // next word to store
  uint64_t lo = 0, hi = 0;  // window bits [64 w, 64 w + 128)
  uint64_t cin = 0;         // carry of the +1 into word w
  auto flush = [&]() {
    uint64_t v = lo;
    if (inv) {
      v ^= rangemask(ra - 64ll * w, rb - 64ll * w);
      const uint64_t add = cin + (w == wplus ? 1ull << (ra & 63) : 0ull);
      const uint64_t s = v + add;
      cin = s < v ? 1ull : 0ull;
      v = s;
    }
    Xw[w] = v;
    lo = hi;
    hi = 0;
    ++w;
  };
  if (digits) {
    const int q0 = (int)(wlo / I8_W) & ~3, q1 = (int)((whi - 1) / I8_W);
    for (int c = q0 >> 4; c <= (q1 >> 4); ++c) {
      const uint4 cv = *reinterpret_cast<const uint4*>(st.glob + (size_t)c * 1024);
      const uint32_t words[4] = {cv.x, cv.y, cv.z, cv.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int qq = 16 * c + 4 * k;
        if (qq + 3 < q0 || qq > q1) continue;
        const uint32_t wd = words[k];
        uint64_t v = wd;  // four digits of I8_W = 8 bits: the word is their binary value
        const int nvalid = st.Dmax - qq + 1;  // digits beyond Dmax are not part of X
        if (nvalid < 4) v &= lowmask((int64_t)I8_W * (nvalid < 0 ? 0 : nvalid));
        int64_t bp = (int64_t)I8_W * qq - xw0;  // >= -(4 I8_W - 1)
        if (bp < 0) {
          v >>= -bp;
          bp = 0;
        }
        while (bp >= 64ll * (w + 1)) flush();  // bp < 64 nx
        const int rr = (int)(bp - 64ll * w);
        lo |= v << rr;
        if (rr > 64 - 4 * I8_W) hi |= v >> (64 - rr);
      }
    }
  }
  while (w < nx) flush();
  if (st.U && nbits < xw0 + 64ll * nx) {  // the top above the digits
    const int64_t bp = nbits - xw0;
    if (bp < 0) {
      if (-bp < 64) Xw[0] |= st.U >> (-bp);
    } else {
      const int64_t wu = bp >> 6;
      const int rr = (int)(bp & 63);
      Xw[wu] |= st.U << rr;
      if (rr && wu + 1 < nx) Xw[wu + 1] |= st.U >> (64 - rr);
    }
  }
}

// ----------------------------------------------------------------------------
// Accumulating form C := C + sgn X (X = A B on the digit grid), rounded once.
// Positions are grid bits (bit 0 = lowest bit of digit q = 0; the value of grid
// bit b is 2^(b + G_i + H_j - 7 (Dmax + 2))).  The addend's significand is at
// most p bits, so apart from the cases where one operand lies wholly below the
// other's lowest bit and a quarter ulp (it then only breaks a tie, or vanishes)
// the exact sum is formed over the addend's own bit range [cb, ct1) with one
// bit of headroom: below cb only X has bits (its tail passes through, or is
// complemented when |C| > |X|), and above ct1 X's digits change by the carry
// or borrow (+1 / -1) out of that range.
// ----------------------------------------------------------------------------

struct AccC {
  const uint64_t* mant;
  const uint64_t* cl;  // the limbs copied to this thread's LDS, or NULL: read them from mant
  int64_t ls, o, sh;   // sh: grid position of significand bit 0
  int L, drop;         // drop: bits below the precision in limb 0 (ignored)
  __device__ inline uint64_t limb(int64_t l) const {
    if (l < 0 || l >= L) return 0;
    uint64_t v = cl ? cl[l] : mant[l * ls + o];
    if (l == 0 && drop) v &= ~((1ull << drop) - 1ull);
    return v;
  }
  // bits [pos, pos + 64) of |C|
  __device__ inline uint64_t field(int64_t pos) const {
    const int64_t b = pos - sh;
    if (b >= 64ll * L || b <= -64) return 0;
    const int64_t l0 = b >= 0 ? b / 64 : -((-b + 63) / 64);
    const int r = (int)(b - 64 * l0);
    const uint64_t lo = limb(l0), hi = limb(l0 + 1);
    return r ? (lo >> r) | (hi << (64 - r)) : lo;
  }
  __device__ inline int64_t lowest() const {
    for (int l = 0; l < L; ++l) {
      const uint64_t v = limb(l);
      if (v) return sh + 64ll * l + __builtin_ctzll(v);
    }
    return sh;  // not reached for a nonzero addend
  }
};

struct AccSum {
  const Win8* st;
  const uint64_t* Y;  // the sum over [cb, cb + Wd), nl limbs
  const uint64_t* Xw; // |X| bits [xw0, xw0 + 64 nx) in binary (nx = 0: none)
  int64_t cb, ct1, Wd, low_x, r, xw0;
  int nl, delta, typ, xlo, nx;
  // bits [pos, pos + 64) of |X|: from the binary window when inside it
  __device__ inline uint64_t xf(int64_t pos) const {
    const int64_t b = pos - xw0;
    if (nx && b >= 0 && b + 64 <= 64ll * nx) {
      const int64_t w = b >> 6;
      const int rr = (int)(b & 63);
      return rr ? (Xw[w] >> rr) | (Xw[w + 1] << (64 - rr)) : Xw[w];
    }
    return st->fieldg(pos);
  }
  __device__ inline int64_t first_from(int64_t pos, int want, int64_t limit) const {
    while (pos <= limit) {
      const uint64_t f = xf(pos);
      const uint64_t g = want ? f : ~f;
      if (g) return pos + __builtin_ctzll(g);
      pos += 64;
    }
    return limit;
  }
  __device__ inline uint64_t yfield(int64_t pos) const {
    const int64_t b = pos - cb;
    if (b >= Wd || b <= -64) return 0;
    const int64_t l0 = b >= 0 ? b / 64 : -((-b + 63) / 64);
    const int rr = (int)(b - 64 * l0);
    const uint64_t lo = (l0 >= 0 && l0 < nl) ? Y[l0] : 0;
    const uint64_t hi = (l0 + 1 >= 0 && l0 + 1 < nl) ? Y[l0 + 1] : 0;
    return rr ? (lo >> rr) | (hi << (64 - rr)) : lo;
  }
  // bits [pos, pos + 64) of |S|
  __device__ inline uint64_t field(int64_t pos) const {
    if (typ == 1) {
      uint64_t f = yfield(pos);
      if (pos < cb) f |= xf(pos) & lowmask(cb - pos);
      if (pos + 64 > ct1) {
        uint64_t t = xf(pos);
        if (delta) {
          const uint64_t run = rangemask(ct1 - pos, r - pos);
          t = delta > 0 ? (t & ~run) : (t | run);
          if (r >= pos && r < pos + 64) t = delta > 0 ? (t | (1ull << (r - pos))) : (t & ~(1ull << (r - pos)));
        }
        f |= t & ~lowmask(ct1 - pos);
      }
      return f;
    }
    uint64_t f = yfield(pos);
    if (xlo && pos < cb) {
      f |= ~xf(pos) & rangemask(low_x + 1 - pos, cb - pos);
      if (low_x >= pos && low_x < pos + 64) f |= 1ull << (low_x - pos);
    }
    return f;
  }
};

// The general case: writes the rounded sum (sign, exponent, limbs) of entry o.
__device__ __attribute__((always_inline)) inline void round_acc_general(const Win8& st, int64_t lead_x, int64_t low_x, int sx, const AccC& C, int sc,
                                  int64_t gbase, int p, int L, DOutPart out, int64_t o, uint64_t* Y, uint64_t* Xw,
                                  int nx, int* status) {
  const int64_t nbits = (int64_t)I8_W * (st.Dmax + 1);
  const int64_t lead_c = 64ll * L - 1 + C.sh;
  const int64_t cb = C.lowest();
  const int64_t ct1 = lead_c + 2;
  const int64_t Wd = ct1 - cb;  // at most p + 1 bits
  const int nl = (int)((Wd + 63) / 64);
  const int wr = (int)(Wd & 63);
  const uint64_t wmask = wr ? ((1ull << wr) - 1ull) : ~0ull;
  const int xlo = low_x < cb;
  AccSum S;
  S.st = &st; S.Y = Y; S.cb = cb; S.ct1 = ct1; S.Wd = Wd; S.low_x = low_x; S.nl = nl; S.xlo = xlo; S.r = 0;
  S.delta = 0;
  // |X| around the addend's range in binary, built once from the digits
  S.Xw = Xw;
  S.nx = nx;
  S.xw0 = cb - 128;
  if (nx) build_xwin(st, S.xw0, nx, low_x, Xw);
  int s_out;
  if (sc == sx) {  // |X| + |C|
    uint64_t carry = 0;
    for (int l = 0; l < nl; ++l) {
      uint64_t a = S.xf(cb + 64ll * l);
      if (l == nl - 1) a &= wmask;
      const uint64_t b = C.field(cb + 64ll * l);
      const uint64_t s1 = a + b;
      const uint64_t c1 = s1 < a;
      const uint64_t s2 = s1 + carry;
      const uint64_t c2 = s2 < s1;
      Y[l] = s2;
      carry = c1 | c2;
    }
    if (wr) {
      S.delta = (int)((Y[nl - 1] >> wr) & 1ull);
      Y[nl - 1] &= wmask;
    } else {
      S.delta = (int)carry;
    }
    S.typ = 1;
    s_out = sx;
  } else {
    int xbig;
    if (lead_x != lead_c) {
      xbig = lead_x > lead_c;
    } else {
      xbig = 1;  // equal over the range: X's tail below cb makes |X| >= |C|
      for (int l = nl - 1; l >= 0; --l) {
        uint64_t a = S.xf(cb + 64ll * l);
        if (l == nl - 1) a &= wmask;
        const uint64_t b = C.field(cb + 64ll * l);
        if (a != b) {
          xbig = a > b;
          break;
        }
      }
    }
    uint64_t borrow = xbig ? 0ull : (uint64_t)xlo;
    for (int l = 0; l < nl; ++l) {
      uint64_t a = S.xf(cb + 64ll * l);
      if (l == nl - 1) a &= wmask;
      const uint64_t b = C.field(cb + 64ll * l);
      const uint64_t u = xbig ? a : b, v = xbig ? b : a;
      const uint64_t t = u - v;
      const uint64_t b1 = u < v;
      const uint64_t d = t - borrow;
      const uint64_t b2 = t < borrow;
      Y[l] = d;
      borrow = b1 | b2;
    }
    Y[nl - 1] &= wmask;
    if (xbig) {
      S.delta = borrow ? -1 : 0;
      S.typ = 1;
      s_out = sx;
    } else {
      S.typ = 2;
      s_out = sc;
    }
  }
  int ynz = 0;
  for (int l = 0; l < nl; ++l) ynz |= Y[l] != 0;
  const int64_t scan_limit = nbits + 128;
  // leading and lowest set bit of |S|
  int64_t lead = INT64_MIN, lows = 0;
  if (S.typ == 1) {
    if (S.delta > 0) S.r = S.first_from(ct1, 0, scan_limit);
    if (S.delta < 0) S.r = S.first_from(ct1, 1, scan_limit);
    if (S.delta == 0) {
      if (lead_x >= ct1) lead = lead_x;
    } else if (S.delta > 0) {
      lead = max(lead_x, S.r);
    } else {
      if (lead_x > S.r) lead = lead_x;
      else if (S.r > ct1) lead = S.r - 1;
    }
    if (lead == INT64_MIN) {
      if (ynz) {
        for (int l = nl - 1; l >= 0; --l)
          if (Y[l]) {
            lead = cb + 64ll * l + 63 - __builtin_clzll(Y[l]);
            break;
          }
      } else if (xlo) {
        int64_t hi = cb;  // highest set bit of X below cb (its lowest is low_x)
        while (hi > low_x) {
          const int64_t start = max(hi - 64, low_x);
          const uint64_t f = S.xf(start) & lowmask(hi - start);
          if (f) {
            lead = start + 63 - __builtin_clzll(f);
            break;
          }
          hi = start;
        }
      }
    }
    if (xlo) {
      lows = low_x;
    } else if (ynz) {
      for (int l = 0; l < nl; ++l)
        if (Y[l]) {
          lows = cb + 64ll * l + __builtin_ctzll(Y[l]);
          break;
        }
    } else if (S.delta == 0) {
      lows = S.first_from(ct1, 1, scan_limit);
    } else if (S.delta > 0) {
      lows = S.r;
    } else {
      lows = S.r > ct1 ? ct1 : S.first_from(S.r + 1, 1, scan_limit);
    }
  } else {
    if (ynz) {
      for (int l = nl - 1; l >= 0; --l)
        if (Y[l]) {
          lead = cb + 64ll * l + 63 - __builtin_clzll(Y[l]);
          break;
        }
    } else if (xlo) {
      lead = low_x;  // highest set bit of 2^cb - X_lo: its highest zero of X above low_x
      int64_t hi = cb;
      while (hi > low_x + 1) {
        const int64_t start = max(hi - 64, low_x + 1);
        const uint64_t f = ~S.xf(start) & lowmask(hi - start);
        if (f) {
          lead = start + 63 - __builtin_clzll(f);
          break;
        }
        hi = start;
      }
    }
    if (xlo) {
      lows = low_x;
    } else {
      for (int l = 0; l < nl; ++l)
        if (Y[l]) {
          lows = cb + 64ll * l + __builtin_ctzll(Y[l]);
          break;
        }
    }
  }
  if (lead == INT64_MIN) {  // exact cancellation -> +0
    out.sign[o] = 0;
    out.exp[o] = EXP_ZERO;
    for (int l = 0; l < L; ++l) out.mant[(int64_t)l * out.ls + o] = 0;
    return;
  }
  const int64_t low = lead - p + 1;
  const int rbit = (int)(S.field(low - 1) & 1ull);
  const int lsb = (int)(S.field(low) & 1ull);
  const int sticky = lows < low - 1;
  const int round_up = rbit && (sticky || lsb);
  const int keep_from = 64 * L - p;
  const int64_t off = lead + 1 - 64ll * L;
  uint64_t carry = round_up ? (1ull << keep_from) : 0;
  int64_t e_out = lead + 1 + gbase;
  uint64_t limbs_hi = 0;
  for (int l = 0; l < L; ++l) {
    uint64_t f = S.field(off + 64ll * l);
    if (l == 0 && keep_from) f &= ~((1ull << keep_from) - 1ull);
    const uint64_t sum = f + carry;
    carry = (sum < f) ? 1 : 0;
    limbs_hi = sum;
    if (l < L - 1) out.mant[(int64_t)l * out.ls + o] = sum;
  }
  if (carry) {
    limbs_hi = 1ull << 63;
    e_out += 1;
  }
  if (e_out > INT32_MAX || e_out <= (int64_t)INT32_MIN) {
    atomicOr(status, ST_OUT_RANGE);
    out.sign[o] = 0;
    out.exp[o] = EXP_ZERO;
    for (int l = 0; l < L; ++l) out.mant[(int64_t)l * out.ls + o] = 0;
    return;
  }
  out.mant[(int64_t)(L - 1) * out.ls + o] = limbs_hi;
  out.sign[o] = (uint8_t)s_out;
  out.exp[o] = (int32_t)e_out;
}

// The common general case in one pass.  |X| is built in binary over a window
// anchored at the addend's leading bit: L + 3 words, from 64 L + 126 bits
// below lead_C to 65 bits above it, so the addend's significand (its bit 0
// at window bit 127) lies wholly inside.  The addend is added or subtracted
// across the whole window; X's bits below the window only borrow one unit
// (when |C| > |X|) and set the sticky bit.  The sum is rounded from the
// window.  Returns false, having written nothing, when X reaches above the
// window or cancellation leaves the rounding bit or the lowest limb below
// it; the caller then takes the general path.  Sw: 2 (L + 3) words of this
// thread's LDS (the window, then the addend's aligned words).
__device__ __attribute__((always_inline)) inline bool round_acc_window(const Win8& st, int64_t lead_x, int64_t low_x, int sx, const AccC& C, int sc,
                                 int64_t gbase, int p, int L, DOutPart out, int64_t o, uint64_t* Sw, int* status) {
  const int64_t lead_c = 64ll * L - 1 + C.sh;
  if (lead_x > lead_c + 64) return false;
  const int nx = L + 3;
  const int64_t xw0 = lead_c + 66 - 64ll * nx;
  uint64_t* Cw = Sw + nx;
  build_xwin(st, xw0, nx, low_x, Sw);
  for (int w = 0; w < nx; ++w) Cw[w] = C.field(xw0 + 64ll * w);
  const int tail = low_x < xw0;  // X has set bits below the window
  int s_out;
  if (sc == sx) {  // |X| + |C| < 2^(lead_c + 66): no carry out of the window
    uint64_t carry = 0;
    for (int w = 0; w < nx; ++w) {
      const uint64_t a = Sw[w], b = Cw[w];
      const uint64_t s1 = a + b, c1 = s1 < a;
      const uint64_t s2 = s1 + carry, c2 = s2 < s1;
      Sw[w] = s2;
      carry = c1 | c2;
    }
    s_out = sx;
  } else {
    int cmp = 0;  // sign of (|X| in the window) - |C|
    for (int w = nx - 1; w >= 0 && !cmp; --w)
      if (Sw[w] != Cw[w]) cmp = Sw[w] > Cw[w] ? 1 : -1;
    if (cmp == 0) {
      if (tail) return false;  // only X's bits below the window remain
      out.sign[o] = 0;         // exact cancellation -> +0
      out.exp[o] = EXP_ZERO;
      for (int l = 0; l < L; ++l) out.mant[(int64_t)l * out.ls + o] = 0;
      return true;
    }
    const int xbig = cmp > 0;
    uint64_t borrow = xbig ? 0ull : (uint64_t)tail;
    for (int w = 0; w < nx; ++w) {
      const uint64_t u = xbig ? Sw[w] : Cw[w], v = xbig ? Cw[w] : Sw[w];
      const uint64_t t = u - v, b1 = u < v;
      const uint64_t d = t - borrow, b2 = t < borrow;
      Sw[w] = d;
      borrow = b1 | b2;
    }
    s_out = xbig ? sx : sc;
  }
  int64_t lead = -1;
  for (int w = nx - 1; w >= 0; --w)
    if (Sw[w]) {
      lead = xw0 + 64ll * w + 63 - __builtin_clzll(Sw[w]);
      break;
    }
  if (lead < 0) return false;
  const int64_t low = lead - p + 1;         // lowest kept bit
  const int64_t off = lead + 1 - 64ll * L;  // lowest bit of limb 0
  if (min(off, low - 1) < xw0) return false;
  auto sbit = [&](int64_t pos) -> int {
    const int64_t r = pos - xw0;
    return (int)((Sw[r >> 6] >> (r & 63)) & 1ull);
  };
  const int rbit = sbit(low - 1), lsb = sbit(low);
  int sticky = tail;
  {
    const int64_t r = low - 1 - xw0;  // bits of the window below the rounding bit
    const int wr = (int)(r >> 6);
    for (int w = 0; w < wr && !sticky; ++w) sticky = Sw[w] != 0;
    if (!sticky) sticky = (Sw[wr] & lowmask(r & 63)) != 0;
  }
  const int round_up = rbit && (sticky || lsb);
  const int keep_from = 64 * L - p;
  uint64_t carry = round_up ? (1ull << keep_from) : 0;
  int64_t e_out = lead + 1 + gbase;
  uint64_t limbs_hi = 0;
  for (int l = 0; l < L; ++l) {
    const int64_t r = off + 64ll * l - xw0;  // r + 64 <= 64 nx
    const int w = (int)(r >> 6), sh = (int)(r & 63);
    uint64_t f = sh ? (Sw[w] >> sh) | (Sw[w + 1] << (64 - sh)) : Sw[w];
    if (l == 0 && keep_from) f &= ~((1ull << keep_from) - 1ull);
    const uint64_t sum = f + carry;
    carry = (sum < f) ? 1 : 0;
    limbs_hi = sum;
    if (l < L - 1) out.mant[(int64_t)l * out.ls + o] = sum;
  }
  if (carry) {
    limbs_hi = 1ull << 63;
    e_out += 1;
  }
  if (e_out > INT32_MAX || e_out <= (int64_t)INT32_MIN) {
    atomicOr(status, ST_OUT_RANGE);
    out.sign[o] = 0;
    out.exp[o] = EXP_ZERO;
    for (int l = 0; l < L; ++l) out.mant[(int64_t)l * out.ls + o] = 0;
    return true;
  }
  out.mant[(int64_t)(L - 1) * out.ls + o] = limbs_hi;
  out.sign[o] = (uint8_t)s_out;
  out.exp[o] = (int32_t)e_out;
  return true;
}

// bytes of LDS per thread for L limbs: |X| in binary over the significand
// and one word below it (L + 1 words), or the accumulating form's sum over
// the addend's range (L + 2 words), in an odd number of 16-byte units so that
// the 64 lanes' areas start in 16 different bank groups instead of 4
__host__ __device__ inline int round_i8_window_bytes(int L) {
  const int units = (8 * (L + 2) + 15) / 16;
  return 16 * (units | 1);
}

// The accumulating form also keeps, per thread, the sum over the addend's
// range (L + 2 words) and |X| in binary from two words below the addend's
// lowest bit (L + 4 words), when 256 threads' worth fits the LDS (p <= 2304);
// beyond that |X| is read from global memory directly; and then the addend's
// L limbs, read once from global memory, when that fits too (p <= 1536).
// Bits of |X| outside the window are always read from global memory.
__host__ __device__ inline int round_i8_acc_words(int L) { return L + 4; }
__host__ __device__ inline int round_i8_lds_bytes(int L, int acc) {
  const int wb = round_i8_window_bytes(L);
  if (!acc) return wb;
  const int with_c = 16 * (((8 * ((L + 2) + round_i8_acc_words(L) + L) + 15) / 16) | 1);
  if (256 * with_c <= 160 * 1024) return with_c > wb ? with_c : wb;
  const int need = 16 * (((8 * ((L + 2) + round_i8_acc_words(L)) + 15) / 16) | 1);
  const int b = need > wb ? need : wb;
  return 256 * b <= 160 * 1024 ? b : wb;
}

__device__ inline void round_i8_block(const RoundArgs& a, int blk, uint8_t* lds_all) {
  const int tiles = a.mt * a.nt;
  const int tile = blk >> 1, comp = blk & 1;
  const int t = threadIdx.x;
  const int ii = t & 15, jj = t >> 4;
  const int lane = jj + 16 * (ii >> 2), slot = 4 * comp + (ii & 3);
  const int ti = tile % a.mt, tj = tile / a.mt;
  const int i = ti * 16 + ii, j = tj * 16 + jj;
  const int WB = round_i8_lds_bytes(a.L, a.acc);
  uint8_t* lds = lds_all + (size_t)t * WB;
  if (i >= a.m || j >= a.n) return;  // no barrier follows

  const size_t sstride = (size_t)tiles * 8 * a.nchunk * 1024;  // one contraction chunk's digits
  uint8_t* g0 = reinterpret_cast<uint8_t*>(const_cast<void*>(a.digits)) +
                ((size_t)tile * 8 + slot) * a.nchunk * 1024 + (size_t)lane * 16;
  const size_t tb0 = ((size_t)tile * 64 + lane) * 8 + slot;
  int Dmax = a.Dmax;  // digits of the integer rounded: more when shifted streams are merged
  int64_t gbase = (int64_t)a.G[i] + (int64_t)a.H[j] - (int64_t)I8_W * (a.Dmax + 2);

  int64_t T;
  int z;
  int zdig = 0;  // the lowest nonzero digit's value, when a merge found it
  uint4 topc = make_uint4(0u, 0u, 0u, 0u);  // the merged top chunk, when a merge formed it
  bool have_topc = false;
  if (a.parts) {
    // separately scaled parts: Re = P_rr - P_ii, Im = P_ri + P_ir, the stream
    // at the larger scale shifted up by the whole digits between the scales
    const PartsMerge& pm = *a.parts;
    const int64_t Gr = pm.Gre[i], Gi = pm.Gim[i], Hr = pm.Hre[j], Hi = pm.Him[j];
    const int64_t sU = comp ? Gr + Hi : Gr + Hr;
    const int64_t sV = comp ? Gi + Hr : Gi + Hi;
    const int sgV = comp ? 1 : -1;
    const int64_t dq = (sU - sV) / I8_W;  // exact: the scales agree modulo 8
    const int shU = dq > 0 ? (int)dq : 0, shV = dq < 0 ? (int)-dq : 0;
    const int D0 = a.Dmax;
    Dmax = D0 + shU + shV;
    gbase = (sU < sV ? sU : sV) - (int64_t)I8_W * (D0 + 2);
    const uint8_t* src = pm.dig[comp];
    const size_t cstride = (size_t)tiles * 8 * pm.nchunk * 1024;  // one contraction chunk's layout
    const size_t eoU = ((size_t)tile * 8 + (ii & 3)) * pm.nchunk * 1024 + (size_t)lane * 16;
    const size_t eoV = ((size_t)tile * 8 + 4 + (ii & 3)) * pm.nchunk * 1024 + (size_t)lane * 16;
    const size_t tU = ((size_t)tile * 64 + lane) * 8 + (ii & 3);
    int64_t TU = 0, TV = 0;
    for (int q = 0; q < pm.ksplit; ++q) {
      TU += pm.top[comp][(size_t)q * tiles * 512 + tU];
      TV += pm.top[comp][(size_t)q * tiles * 512 + tU + 4];
    }
    const int lastc = D0 >> 4;  // the sources' last chunk
    // digits 16 ch .. 16 ch + 15 of one source shifted up by sh digits, as two
    // 64-bit words (zero below the source's digit 0 and above digit D0)
    auto window16 = [&](const uint8_t* base, int ch, int sh, uint64_t& r0, uint64_t& r1)
                        __attribute__((always_inline)) {
      const int i0 = 16 * ch - sh;  // source digit under output digit 16 ch
      const int c0 = i0 >= 0 ? (i0 >> 4) : -((15 - i0) >> 4);
      const int o = i0 - 16 * c0;   // 0 .. 15
      // both chunks loaded from clamped (valid) positions, then zeroed where
      // they lie outside the source
      const int ca = min(max(c0, 0), lastc), cb = min(max(c0 + 1, 0), lastc);
      const uint4 v0 = *reinterpret_cast<const uint4*>(base + (size_t)ca * 1024);
      const uint4 v1 = *reinterpret_cast<const uint4*>(base + (size_t)cb * 1024);
      const bool in0 = c0 >= 0 && c0 <= lastc, in1 = c0 + 1 >= 0 && c0 + 1 <= lastc;
      // the 32-byte window as four 64-bit words; bytes o .. o + 15 of it
      const uint64_t q0 = in0 ? v0.x | ((uint64_t)v0.y << 32) : 0, q1 = in0 ? v0.z | ((uint64_t)v0.w << 32) : 0;
      const uint64_t q2 = in1 ? v1.x | ((uint64_t)v1.y << 32) : 0, q3 = in1 ? v1.z | ((uint64_t)v1.w << 32) : 0;
      const bool hi8 = o >= 8;
      const uint64_t a0 = hi8 ? q1 : q0, a1 = hi8 ? q2 : q1, a2 = hi8 ? q3 : q2;
      const int sb = 8 * (o & 7);
      r0 = sb ? (a0 >> sb) | (a1 << (64 - sb)) : a0;
      r1 = sb ? (a1 >> sb) | (a2 << (64 - sb)) : a1;
      // source digits above D0 (the unwritten end of the last chunk)
      const int nv = D0 - i0 + 1;  // digits of the window at or below D0
      if (nv < 16) {
        if (nv <= 0) {
          r0 = r1 = 0;
        } else if (nv <= 8) {
          r0 = nv == 8 ? r0 : (r0 & ((1ull << (8 * nv)) - 1));
          r1 = 0;
        } else {
          r1 &= (1ull << (8 * (nv - 8))) - 1;
        }
      }
    };
    // tops enter at digit D0 + 1 + sh of the merged integer, above it when that
    // is past the merged digits
    const int posU = D0 + 1 + shU, posV = D0 + 1 + shV;
    int64_t c = 0;
    int qz = -1;
    const int nq = Dmax + 1;
    for (int ch = 0; ch * 16 < nq; ++ch) {
      uint32_t out[4] = {0, 0, 0, 0};
      int32_t sum[16];
#pragma unroll
      for (int b = 0; b < 16; ++b) sum[b] = 0;
      for (int q = 0; q < pm.ksplit; ++q) {
        uint64_t u0, u1, v0, v1;
        window16(src + q * cstride + eoU, ch, shU, u0, u1);
        window16(src + q * cstride + eoV, ch, shV, v0, v1);
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          const int sh8 = 8 * (b & 7);
          const int32_t du = (int32_t)(((b < 8 ? u0 : u1) >> sh8) & 255u);
          const int32_t dv = (int32_t)(((b < 8 ? v0 : v1) >> sh8) & 255u);
          sum[b] += du + sgV * dv;
        }
      }
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const int qq = ch * 16 + b;
        if (qq < nq) {
          int64_t sv = c + sum[b];
          if (qq == posU) sv += TU;
          if (qq == posV) sv += sgV * TV;
          const uint32_t dg = (uint32_t)(sv & (DFULL - 1));
          c = sv >> I8_W;
          out[b >> 2] |= dg << (8 * (b & 3));
          if (dg && qz < 0) {
            qz = qq;
            zdig = (int)dg;
          }
        }
      }
      *reinterpret_cast<uint4*>(g0 + (size_t)ch * 1024) = make_uint4(out[0], out[1], out[2], out[3]);
      if (ch == (Dmax >> 4)) {
        topc = make_uint4(out[0], out[1], out[2], out[3]);
        have_topc = true;
      }
    }
    z = qz < 0 ? -1 : Dmax - qz;
    T = c + (posU > Dmax ? TU : 0) + (posV > Dmax ? sgV * TV : 0);
  } else if (a.nsrc > 0) {
    // the signed sum of the source streams, least significant digit first, 16
    // digits at a time, written to this element's digits
    const size_t eo = ((size_t)tile * 8 + slot) * a.nchunk * 1024 + (size_t)lane * 16;
    const int ns = comp ? a.nsrc_im : a.nsrc;  // this component's sources
    const MergeSrc* __restrict__ sl = a.src + (comp ? MAX_MERGE : 0);
    int64_t c = 0;
    int qz = -1;
    const int nq = Dmax + 1;
    for (int ch = 0; ch * 16 < nq; ++ch) {
      uint32_t out[4] = {0, 0, 0, 0};
      int32_t sum[16];
#pragma unroll
      for (int b = 0; b < 16; ++b) sum[b] = 0;
      // up to eight sources' loads in flight before any is used
      for (int q = 0; q < ns; q += 8) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          v[u] = q + u < ns ? *reinterpret_cast<const uint4*>(sl[q + u].dig + eo + (size_t)ch * 1024)
                            : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t wv[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
          const int sg = q + u < ns ? (int)sl[q + u].sign : 0;
#pragma unroll
          for (int b = 0; b < 16; ++b) sum[b] += sg * (int32_t)((wv[b >> 2] >> (8 * (b & 3))) & 255u);
        }
      }
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const int qq = ch * 16 + b;
        if (qq < nq) {
          const int64_t sv = c + sum[b];
          const uint32_t dg = (uint32_t)(sv & (DFULL - 1));
          c = sv >> I8_W;
          out[b >> 2] |= dg << (8 * (b & 3));
          if (dg && qz < 0) {
            qz = qq;
            zdig = (int)dg;
          }
        }
      }
      *reinterpret_cast<uint4*>(g0 + (size_t)ch * 1024) = make_uint4(out[0], out[1], out[2], out[3]);
      if (ch == (Dmax >> 4)) {
        topc = make_uint4(out[0], out[1], out[2], out[3]);
        have_topc = true;
      }
    }
    z = qz < 0 ? -1 : Dmax - qz;
    T = c;
    for (int q = 0; q < ns; ++q) T += sl[q].sign * sl[q].top[tb0];
  } else if (a.seg_bs > 1) {
    // band-group streams: group g's stream holds its own digits (zero to the
    // ends of its chunks) and its top the carry into group g + 1's first
    // digit.  A 16-digit chunk lies in at most two groups (bands of 8 or more
    // digits), so it takes two streams per contraction chunk and pass, and at
    // most two carries.
    const int bs = a.seg_bs, ps = a.seg_ps > 1 ? a.seg_ps : 1, W = a.seg_w, bpg = a.seg_bpg;
    const int nb_all = (a.Dmax + W) / W;
    const int nss = a.ksplit * ps;  // streams per group
    const size_t tstride = (size_t)tiles * 512;
    auto sidx = [&](int s2, int g) { return ((s2 / ps) * bs + g) * ps + s2 % ps; };
    int64_t Ttop = 0;  // the last group's carries, which lie above every digit (loaded first)
    for (int q = 0; q < nss; ++q) Ttop += a.top[(size_t)sidx(q, bs - 1) * tstride + tb0];
    int64_t c = 0;
    int qz = -1;
    const int nq = Dmax + 1;
    for (int ch = 0; ch * 16 < nq; ++ch) {
      const int gA = min(nb_all - 1, (16 * ch) / W) / bpg;
      const int gB = min(nb_all - 1, (16 * ch + 15) / W) / bpg;
      const int pA = W * gA * bpg, pB = W * gB * bpg;  // the groups' first digits
      const bool inA = gA > 0 && pA == 16 * ch;      // group gA starts at this chunk
      const bool inB = gB != gA;                     // group gB starts inside it
      uint32_t out[4] = {0, 0, 0, 0};
      int32_t sum[16];
#pragma unroll
      for (int b = 0; b < 16; ++b) sum[b] = 0;
      int64_t cA = 0, cB = 0;
      for (int q = 0; q < nss; q += 4) {  // four streams' loads per group and their carries in flight
        uint4 vA[4], vB[4];
        int64_t tA[4], tB[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool ok = q + u < nss;
          const size_t so = (size_t)ch * 1024;
          vA[u] = ok ? *reinterpret_cast<const uint4*>(g0 + (size_t)sidx(q + u, gA) * sstride + so)
                     : make_uint4(0u, 0u, 0u, 0u);
          vB[u] = ok && inB ? *reinterpret_cast<const uint4*>(g0 + (size_t)sidx(q + u, gB) * sstride + so)
                            : make_uint4(0u, 0u, 0u, 0u);
          tA[u] = ok && inA ? a.top[(size_t)sidx(q + u, gA - 1) * tstride + tb0] : 0;
          tB[u] = ok && inB ? a.top[(size_t)sidx(q + u, gA) * tstride + tb0] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t wa[4] = {vA[u].x, vA[u].y, vA[u].z, vA[u].w};
          const uint32_t wb[4] = {vB[u].x, vB[u].y, vB[u].z, vB[u].w};
#pragma unroll
          for (int b = 0; b < 16; ++b)
            sum[b] += (int32_t)((wa[b >> 2] >> (8 * (b & 3))) & 255u) + (int32_t)((wb[b >> 2] >> (8 * (b & 3))) & 255u);
          cA += tA[u];
          cB += tB[u];
        }
      }
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const int qq = ch * 16 + b;
        if (qq < nq) {
          int64_t sv = c + sum[b];
          if (inA && qq == pA) sv += cA;
          if (inB && qq == pB) sv += cB;
          const uint32_t dg = (uint32_t)(sv & (DFULL - 1));
          c = sv >> I8_W;
          out[b >> 2] |= dg << (8 * (b & 3));
          if (dg && qz < 0) {
            qz = qq;
            zdig = (int)dg;
          }
        }
      }
      *reinterpret_cast<uint4*>(g0 + (size_t)ch * 1024) = make_uint4(out[0], out[1], out[2], out[3]);
      if (ch == (Dmax >> 4)) {
        topc = make_uint4(out[0], out[1], out[2], out[3]);
        have_topc = true;
      }
    }
    z = qz < 0 ? -1 : Dmax - qz;
    T = c + Ttop;
  } else if (a.ksplit == 1) {
    T = a.top[tb0];
    z = a.lnz[tb0];
  } else {
    // add the chunk streams exactly, least significant digit first, 16 digits
    // at a time; the sum replaces chunk 0's digits
    int64_t Ttop = 0;  // the streams' tops (loaded first)
    for (int q = 0; q < a.ksplit; ++q) Ttop += a.top[(size_t)q * tiles * 64 * 8 + tb0];
    int64_t c = 0;
    int qz = -1;
    const int nq = Dmax + 1;
    for (int ch = 0; ch * 16 < nq; ++ch) {
      uint32_t out[4] = {0, 0, 0, 0};
      int32_t sum[16];
#pragma unroll
      for (int b = 0; b < 16; ++b) sum[b] = 0;
      // up to eight streams' loads in flight before any is used (a product
      // of few work items has one stream per band group and contraction
      // chunk, and its rounding waits on these loads one batch after another)
      for (int q = 0; q < a.ksplit; q += 8) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          v[u] = q + u < a.ksplit && !(a.onepass == 3 ? comp == 0 && (q + u) % 3 == 2
                                                       : a.onepass == 4 && ((q + u) % 4 < 2) != (comp == 0))
                     ? *reinterpret_cast<const uint4*>(g0 + (q + u) * sstride + (size_t)ch * 1024)
                     : make_uint4(0u, 0u, 0u, 0u);
        // two digits per 32-bit add: even and odd bytes in 16-bit lanes (8
        // sources of at most 255 fit a lane), then into the 32-bit sums
        uint32_t ev[4] = {0u, 0u, 0u, 0u}, od[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t wv[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            ev[w] += wv[w] & 0x00FF00FFu;
            od[w] += (wv[w] >> 8) & 0x00FF00FFu;
          }
        }
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          sum[4 * w] += (int32_t)(ev[w] & 0xFFFFu);
          sum[4 * w + 1] += (int32_t)(od[w] & 0xFFFFu);
          sum[4 * w + 2] += (int32_t)(ev[w] >> 16);
          sum[4 * w + 3] += (int32_t)(od[w] >> 16);
        }
      }
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const int qq = ch * 16 + b;
        if (qq < nq) {
          const int64_t sv = c + sum[b];
          const uint32_t dg = (uint32_t)(sv & (DFULL - 1));
          c = sv >> I8_W;
          out[b >> 2] |= dg << (8 * (b & 3));
          if (dg && qz < 0) {
            qz = qq;
            zdig = (int)dg;
          }
        }
      }
      *reinterpret_cast<uint4*>(g0 + (size_t)ch * 1024) = make_uint4(out[0], out[1], out[2], out[3]);
      if (ch == (Dmax >> 4)) {
        topc = make_uint4(out[0], out[1], out[2], out[3]);
        have_topc = true;
      }
    }
    z = qz < 0 ? -1 : Dmax - qz;
    T = c + Ttop;
  }

  DOutPart out = comp ? a.cim : a.cre;
  const int64_t o = (int64_t)j * a.ldc + i;
  const int L = a.L, p = a.prec;
  // accumulating form: the entry's current value is the addend
  const int negp = a.acc < 0;
  int32_t ce = EXP_ZERO;
  if (a.acc) ce = out.exp[o];
  const int cnz = ce != EXP_ZERO;
  if (T == 0 && z < 0) {  // exact zero -> +0 (or the addend, unchanged)
    if (cnz) return;
    out.sign[o] = 0;
    out.exp[o] = EXP_ZERO;
    for (int l = 0; l < L; ++l) out.mant[(int64_t)l * out.ls + o] = 0;
    return;
  }
  Win8 st;
  st.glob = g0;
  st.Dmax = Dmax;
  st.neg = T < 0;
  st.z = z;
  st.U = !st.neg ? (uint64_t)T : (z < 0 ? (uint64_t)(-T) : (uint64_t)(-T - 1));
  const int64_t nbits = (int64_t)I8_W * (Dmax + 1);
  // leading bit of |X|: in the top, else in the highest nonzero magnitude
  // digit, found a 16-digit chunk (one load) at a time
  int64_t lead = -1;
  if (st.U) {
    lead = nbits + 63 - __builtin_clzll(st.U);
  } else {
    for (int c = Dmax >> 4; c >= 0 && lead < 0; --c) {
      const uint4 cv =
          (have_topc && c == (Dmax >> 4)) ? topc : *reinterpret_cast<const uint4*>(g0 + (size_t)c * 1024);
      const uint32_t words[4] = {cv.x, cv.y, cv.z, cv.w};
#pragma unroll
      for (int b = 15; b >= 0; --b) {
        const int q = 16 * c + b;
        const uint64_t raw = (words[b >> 2] >> (8 * (b & 3))) & 255u;
        const int d = Dmax - q;
        const uint64_t v = q > Dmax ? 0ull : !st.neg ? raw : ((z < 0 || d > z) ? 0ull : (d == z ? DFULL - raw : DFULL - 1 - raw));
        if (lead < 0 && v) lead = (int64_t)I8_W * q + 63 - __builtin_clzll(v);
      }
    }
  }
  // lowest set bit of X (= of |X|)
  int64_t lowset;
  if (z >= 0)
    lowset = (int64_t)I8_W * (Dmax - z) + __builtin_ctzll(zdig ? (uint64_t)zdig : st.gn(Dmax - z));
  else
    lowset = nbits + __builtin_ctzll((uint64_t)T);

  const int sx = st.neg ^ negp;  // sign of the product term
  int tie = -1;                   // >= 0: a negligible addend breaks the tie
  if (cnz) {
    AccC C;
    C.mant = out.mant;
    C.cl = nullptr;
    if (WB >= 8 * ((L + 2) + round_i8_acc_words(L) + L)) {
      uint64_t* cl = reinterpret_cast<uint64_t*>(lds) + (L + 2) + round_i8_acc_words(L);
      for (int l = 0; l < L; ++l) cl[l] = out.mant[(int64_t)l * out.ls + o];
      C.cl = cl;
    }
    C.ls = out.ls;
    C.o = o;
    C.L = L;
    C.drop = 64 * L - p;
    C.sh = (int64_t)ce - 64ll * L - gbase;
    const int sc = out.sign[o] ? 1 : 0;
    const int64_t lead_c = 64ll * L - 1 + C.sh;
    if (lead_c < lowset && lead_c <= lead - (int64_t)p - 2) {
      tie = sc == sx;  // below X's lowest bit and a quarter ulp: only ties move
    } else {
      if (lead < C.lowest() && lead <= lead_c - (int64_t)p - 2) return;  // the sum rounds to the addend
      uint64_t* Yw = reinterpret_cast<uint64_t*>(lds);
      if (WB >= 16 * (L + 3) && round_acc_window(st, lead, lowset, sx, C, sc, gbase, p, L, out, o, Yw, a.status))
        return;
      const int have = WB >= 8 * ((L + 2) + round_i8_acc_words(L));
      const int nx = have ? round_i8_acc_words(L) : 0;
      round_acc_general(st, lead, lowset, sx, C, sc, gbase, p, L, out, o, Yw, Yw + (L + 2), nx, a.status);
      return;
    }
  }
  // |X| in binary from 64 bits below the significand's lowest limb bit (off)
  // up to its leading bit: limb l is word l + 1, and the rounding bit lies in
  // word 0 or above
  const int64_t off = lead + 1 - 64ll * L;
  const int64_t xw0 = off - 64;
  uint64_t* Xw = reinterpret_cast<uint64_t*>(lds);
  build_xwin(st, xw0, L + 1, lowset, Xw);
  auto xbit = [&](int64_t pos) -> int {
    const int64_t r = pos - xw0;
    return (int)((Xw[r >> 6] >> (r & 63)) & 1ull);
  };

  const int64_t low = lead - p + 1;  // lowest kept bit of |X|
  int round_up = 0;
  if (low > 0) {
    const int rbit = xbit(low - 1);
    const int sticky = lowset < low - 1;
    const int lsb = xbit(low);
    round_up = rbit && (sticky || (tie < 0 ? lsb : tie));
  }
  const int keep_from = 64 * L - p;  // 0..63
  uint64_t carry = round_up ? (1ull << keep_from) : 0;
  int64_t e_out = lead + 1 + gbase;
  uint64_t limbs_hi = 0;
  for (int l = 0; l < L; ++l) {
    uint64_t f = Xw[l + 1];
    if (l == 0 && keep_from) f &= ~((1ull << keep_from) - 1ull);
    const uint64_t sum = f + carry;
    carry = (sum < f) ? 1 : 0;
    limbs_hi = sum;
    if (l < L - 1) out.mant[(int64_t)l * out.ls + o] = sum;
  }
  if (carry) {  // significand overflowed to 2^p: 2^(p-1) with exponent + 1
    limbs_hi = 1ull << 63;
    e_out += 1;
  }
  if (e_out > INT32_MAX || e_out <= (int64_t)INT32_MIN) {
    atomicOr(a.status, ST_OUT_RANGE);
    out.sign[o] = 0;
    out.exp[o] = EXP_ZERO;
    for (int l = 0; l < L; ++l) out.mant[(int64_t)l * out.ls + o] = 0;
    return;
  }
  out.mant[(int64_t)(L - 1) * out.ls + o] = limbs_hi;
  out.sign[o] = (uint8_t)sx;
  out.exp[o] = (int32_t)e_out;
}

__global__ __launch_bounds__(256) void round_i8_kernel(RoundArgs a) {
  extern __shared__ __align__(16) uint8_t lds_win[];
  round_i8_block(a, blockIdx.x, lds_win);
}

// Batched form: job j is problem j with 2 mt nt blocks (tile, component).
__global__ __launch_bounds__(256) void round_i8_batched(const RoundArgs* __restrict__ jobs, int njobs,
                                                        const int* __restrict__ first) {
  extern __shared__ __align__(16) uint8_t lds_win[];
  const int j = job_of_block(first, njobs, blockIdx.x);
  round_i8_block(jobs[j], blockIdx.x - first[j], lds_win);
}

}  // namespace

hipError_t launch_store_words(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  const uint32_t* w = static_cast<const uint32_t*>(src);
  uint32_t* d = static_cast<uint32_t*>(dst);
  size_t n32 = (bytes + 3) / 4;  // callers pass 256-byte multiples
  while (n32 > 0) {
    StoreWords a;
    a.n = (uint32_t)std::min<size_t>(n32, StoreWords::N);
    memcpy(a.v, w, 4 * (size_t)a.n);
    store_words_kernel<<<1, 256, 0, stream>>>(d, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    w += a.n;
    d += a.n;
    n32 -= a.n;
  }
  return hipSuccess;
}

hipError_t launch_fill_zero(void* p, size_t n, hipStream_t stream) {
  const size_t n32 = (n + 3) / 4;  // caller allocations are 256-byte aligned and rounded
  fill_zero_kernel<<<dim3((unsigned)((n32 + 255) / 256)), dim3(256), 0, stream>>>(static_cast<uint32_t*>(p), n32);
  return hipGetLastError();
}

hipError_t launch_round(const RoundArgs& a, hipStream_t stream) {
  const int blocks = a.mt * a.nt * 2;
  if (a.digit_bytes == 1) {
    const size_t lds = (size_t)256 * round_i8_lds_bytes(a.L, a.acc);
    hipError_t e = hipFuncSetAttribute((const void*)round_i8_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    round_i8_kernel<<<dim3(blocks), dim3(256), lds, stream>>>(a);
  } else {
    round_kernel<uint32_t><<<dim3(blocks), dim3(256), 0, stream>>>(a);  // 512 digit words per tile
  }
  return hipGetLastError();
}

hipError_t launch_zero(DOutPart cre, DOutPart cim, int m, int n, int64_t ldc, int L, hipStream_t stream) {
  const int64_t total = (int64_t)m * n * 2;
  zero_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream>>>(cre, cim, m, n, ldc, L);
  return hipGetLastError();
}

hipError_t launch_round_batched(const RoundArgs* jobs, int njobs, const int* first, int blocks, int L, int acc,
                                hipStream_t stream) {
  if (njobs <= 0 || blocks <= 0) return hipSuccess;
  const size_t lds = (size_t)256 * round_i8_lds_bytes(L, acc);
  hipError_t e = hipFuncSetAttribute((const void*)round_i8_batched, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  round_i8_batched<<<dim3(blocks), dim3(256), lds, stream>>>(jobs, njobs, first);
  return hipGetLastError();
}

}  // namespace mpcg
