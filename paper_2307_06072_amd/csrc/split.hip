// Error-free split of a multi-precision operand into signed-digit slice planes.
//
// Algorithm 2 extracts each slice A_alpha = (A + S_A) - S_A in short floating
// point and carries the remainder A - A_alpha in long precision.  Here the same
// split is done exactly in fixed point: every row r has a power-of-two scale
// 2^G[r] (G = row exponent maximum + headroom), and each entry x is written as
//
//     x / 2^G[r] = sum_{s < S} d_s * 2^(-w (s + 1)),   |d_s| <= 2^(w-1),
//
// with balanced (signed) base-2^w digits d_s.  S is chosen by the host so that
// the last digit reaches the lowest significand bit of every entry of the
// operand, so the split has no remainder at all.  Digits are produced least
// significant first, a chunk of g = floor(56 / w) digits at a time, from a
// 56-bit window of the significand; the balanced normalisation carries upward
// and the topmost digit takes the final value (it stays within 2^(w-1) because
// |x| < 2^(G-1)).
//
// In the 3M form (eq. 6) a third plane holds the digits of Re x + Im x, formed
// exactly from the two signed windows with a carry of its own; in the 4M form
// the B side's third plane holds the digits of -Im x (its own carry too: the
// digit range [-2^(w-1), 2^(w-1)) is not symmetric) so that
// Re(A)Re(B) - Im(A)Im(B) accumulates as a sum (eq. 5).
//
// One block handles a 16 x 64 tile (16 rows of the operand, 64 contraction
// indices), two entries per thread; each thread reads the limbs of its
// entries once, in order, as the windows move up the significands.  Digits go to LDS in the matrix-core operand order and leave as
// contiguous fragments:
//   INT8: fragment = 16 rows x 64 k, lane l holds row l%16, k = 16*(l/16)..+16
//         (16 bytes), tile-major [R/16][op][pad_lo + s][K/64][1024 B] with
//         zero slices around the digits (Sstride slices per plane; with
//         Sstride = pad_lo + S a plane's lower pad is also the upper pad of
//         the plane before it, and one more pad follows the last tile).
//   FP64: fragment = 16 rows x 4 k, lane l holds row l%16, k = l/16 (one
//         double), planes [op][s][R/16][K/4][64 doubles].
#include "mpcg_internal.h"

namespace mpcg {

namespace {

// A block splits one 16 x 64 tile, EPT entries per thread.
constexpr int SPLIT_THREADS = 1024;
constexpr int EPT = 1024 / SPLIT_THREADS;

// Bits [pos, pos + 56) of one significand, pos rising by `step` <= 56 per
// window: limbs li and li + 1 (off: pos - 64 li), and limb li + 2 loaded one
// window ahead, so that its load is in flight while the current window is
// used; every limb is read once.  The limbs are kept as loaded and masked
// where a window uses them (limb 0 to the precision; a clear top bit of limb
// L-1 is noted in `denorm`), so that nothing waits for a load before the next
// window.
struct LimbStream {
  const uint64_t* p;  // limb li + 2 (NULL for a zero entry)
  int64_t li;
  int off;
  uint64_t a, b, c;
  __device__ inline uint64_t load(int64_t li2, int L) const { return (p && li2 >= 0 && li2 < L) ? *p : 0; }
  // pos: the first window's lowest bit
  __device__ inline void start(const uint64_t* mp, int64_t ls, int64_t pos, int L) {
    li = pos >> 6;  // floor
    off = (int)(pos & 63);
    p = mp ? mp + li * ls : nullptr;
    a = load(li, L);
    if (p) p += ls;
    b = load(li + 1, L);
    if (p) p += ls;
    c = load(li + 2, L);
  }
  // the current window, then a move up by step bits
  __device__ inline uint64_t window56(int64_t ls, int step, int L, uint64_t low_mask, int& denorm) {
    const uint64_t x = li == 0 ? a & low_mask : a;
    const uint64_t y = li == -1 ? b & low_mask : b;
    if (p && (li == L - 1 || li == L - 2)) denorm |= !((li == L - 1 ? x : y) >> 63);
    const uint64_t r = off ? ((x >> off) | (y << (64 - off))) : x;
    off += step;
    if (off >= 64) {
      off -= 64;
      ++li;
      a = b;
      b = c;
      if (p) p += ls;
      c = load(li + 2, L);
    }
    return r & ((1ull << 56) - 1ull);
  }
};

struct Entry {
  int64_t idx;
  int64_t sh_re, sh_im;  // F = M * 2^sh: F bit b <-> M bit b - sh
  int neg_re, neg_im;
  int z_re, z_im;        // zero flags (also set for padding)
};

template <typename DT>
struct Layout;

template <>
struct Layout<int8_t> {
  static constexpr int FRAG_BYTES = 1024;  // one 16 x 64 int8 fragment per tile
  __device__ static inline int offset(int rl, int kl) { return (rl + 16 * (kl >> 4)) * 16 + (kl & 15); }
  // tile-major: all planes (and slices) of one 16-row tile are contiguous, so
  // a tile's fragments span a compact range (32-bit offsets from the tile)
  __device__ static inline size_t tile_base(int64_t plane, int rt, int kt, int Rt, int Kpad, int64_t per_tile) {
    (void)Rt;
    return ((size_t)((int64_t)rt * per_tile + plane) * (size_t)(Kpad / 64) + kt) * 1024;  // bytes
  }
};

template <>
struct Layout<double> {
  static constexpr int FRAG_BYTES = 8192;  // sixteen 16 x 4 fp64 fragments per tile
  __device__ static inline int offset(int rl, int kl) { return (kl >> 2) * 64 + rl + 16 * (kl & 3); }
  __device__ static inline size_t tile_base(int64_t plane, int rt, int kt, int Rt, int Kpad, int64_t per_tile) {
    (void)per_tile;
    return ((size_t)(plane * Rt + rt) * (size_t)(Kpad / 4) + (size_t)kt * 16) * 64 * sizeof(double);
  }
};

// The scale of row r < R from the scan's statistics: the row's largest
// exponent plus the headroom x, 0 for a row of zeros (as the scales kernel).
__device__ inline int32_t row_scale(const RowStat* stats, int r, int x) {
  const int32_t e = stats[r].emax;
  return e == INT32_MIN ? 0 : e + x;
}

// WC: the digit width when known at compile time (I8_W for INT8), else 0 (w);
// TH: the third plane (Third) when known at compile time, else -1 (third).
// INT8 tiles alternate between two LDS buffers, so one barrier per chunk
// separates the digit writes of a chunk from their stores, and the stores of
// a chunk from the writes two chunks later.
// TWO: the operand split is op + sign2 * op2 (two operands of the same shape,
// each entry's exact sum formed in the windows; the scales G must cover it).
// Gim (optional): the Im parts' own row scales (the Re parts take G).
template <typename DT, bool ROWCONTIG, int WC, int TH, bool TWO = false>
__device__ inline void split_tile(const DOperand& op, int prec, int L, int S, int Sp, int Sstride, int pad_lo,
                                  int w_rt, int third_rt, const int32_t* __restrict__ G, int Rpad, int Kpad,
                                  DT* __restrict__ out, int* status, int kt, int rt, unsigned char* lds_raw,
                                  const DOperand* op2 = nullptr, int sign2 = 0,
                                  const int32_t* __restrict__ Gim = nullptr, int64_t cm_ld = 0,
                                  const RowStat* __restrict__ stats = nullptr, int sx = 0) {
  constexpr int FRAG = Layout<DT>::FRAG_BYTES / (int)sizeof(DT);  // elements per (op, digit) tile
  constexpr int NBUF = sizeof(DT) == 1 ? 2 : 1;

  const int w = WC ? WC : w_rt;
  const int third = TH >= 0 ? TH : third_rt;
  const int g = 56 / w;  // digits per window
  const int nops = third ? 3 : 2;
  const int t = threadIdx.x;
  const uint64_t low_mask = ~((1ull << (64 * L - prec)) - 1ull) | (64 * L - prec == 0 ? ~0ull : 0ull);
  const int64_t wS = (int64_t)w * S;

  Entry e[EPT], e2[TWO ? EPT : 1];
  int lofs[EPT];
  int bad = 0;
  LimbStream sre[EPT], sim[EPT], sre2[TWO ? EPT : 1], sim2[TWO ? EPT : 1];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    int rl, kl;
    if (ROWCONTIG) {
      rl = t & 15;
      kl = (t >> 4) + (SPLIT_THREADS / 16) * q;
    } else {
      kl = t & 63;
      rl = (t >> 6) + (SPLIT_THREADS / 64) * q;
    }
    lofs[q] = Layout<DT>::offset(rl, kl);
    const int r = rt * 16 + rl, kk = kt * 64 + kl;
    e[q].z_re = e[q].z_im = 1;
    e[q].neg_re = e[q].neg_im = 0;
    e[q].sh_re = e[q].sh_im = 0;
    e[q].idx = 0;
    auto fill = [&](const DOperand& o, Entry& en, int flip) {
      en.z_re = en.z_im = 1;
      en.neg_re = en.neg_im = 0;
      en.sh_re = en.sh_im = 0;
      en.idx = 0;
      if (r < o.R && kk < o.K) {
        const int64_t idx = (int64_t)r * o.rs + (int64_t)kk * o.ks;
        en.idx = idx;
        const int64_t base = (int64_t)(stats ? row_scale(stats, r, sx) : G[r]) - wS + 64 * (int64_t)L;  // sh = exp - base
        const int64_t base_im = Gim ? (int64_t)Gim[r] - wS + 64 * (int64_t)L : base;
        const int32_t er = o.re.exp[idx], ei = o.im.exp[idx];
        if (er != EXP_ZERO) {
          en.z_re = 0;
          en.neg_re = (o.re.sign[idx] ? 1 : 0) ^ flip;
          en.sh_re = (int64_t)er - base;
        }
        if (ei != EXP_ZERO) {
          en.z_im = 0;
          en.neg_im = (o.im.sign[idx] ? 1 : 0) ^ flip;
          en.sh_im = (int64_t)ei - base_im;
        }
      }
    };
    fill(op, e[q], 0);
    if (TWO) fill(*op2, e2[q], sign2 < 0 ? 1 : 0);
  }

  static_assert(sizeof(DT) != 1 || WC == 8, "INT8 slices take 8-bit digits");
  const int64_t half = 1ll << (w - 1);
  const int64_t dmask = (1ll << w) - 1;
  (void)dmask;
  int64_t carry[EPT][3];
#pragma unroll
  for (int q = 0; q < EPT; ++q) carry[q][0] = carry[q][1] = carry[q][2] = 0;

  const int nchunks = (Sp + g - 1) / g;
  const int nbits = g * w;  // <= 56
  const uint64_t wmask = (1ull << nbits) - 1ull;
  // half in every digit field of a window: the balanced digits of v are the
  // fields of v + kfield less half each, and the bits above the window are
  // the carry into the next one
  uint64_t kfield = 0;
  for (int i = 0; i < g; ++i) kfield |= (uint64_t)half << (w * i);
  {
    const int64_t f0 = (int64_t)w * (S - g * (nchunks - 1) - g);  // lowest window's first F bit
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      sre[q].start(e[q].z_re ? nullptr : op.re.mant + e[q].idx, op.re.ls, f0 - e[q].sh_re, L);
      sim[q].start(e[q].z_im ? nullptr : op.im.mant + e[q].idx, op.im.ls, f0 - e[q].sh_im, L);
      if (TWO) {
        sre2[q].start(e2[q].z_re ? nullptr : op2->re.mant + e2[q].idx, op2->re.ls, f0 - e2[q].sh_re, L);
        sim2[q].start(e2[q].z_im ? nullptr : op2->im.mant + e2[q].idx, op2->im.ls, f0 - e2[q].sh_im, L);
      }
    }
  }
  const int buf_bytes = nops * g * Layout<DT>::FRAG_BYTES;
  // INT8 stores: thread t moves 16-byte units t and t + SPLIT_THREADS of the
  // chunk's nops * g fragments; each unit's (plane, digit, offset) is the
  // same in every chunk, and its destination moves g slices per chunk
  constexpr int I8_UNITS = 1024 / 16;
  constexpr int I8_ITEMS = (3 * (56 / 8) * I8_UNITS + SPLIT_THREADS - 1) / SPLIT_THREADS;
  int8_t* st_dst[I8_ITEMS];
  int st_src[I8_ITEMS], st_j[I8_ITEMS];
  size_t st_step = 0;
  if constexpr (sizeof(DT) == 1) {
    const int64_t kb = Kpad / 64, per_tile = (int64_t)nops * Sstride;
    st_step = (size_t)g * kb * 1024;
#pragma unroll
    for (int it = 0; it < I8_ITEMS; ++it) {
      const int idx = t + it * SPLIT_THREADS;
      const int u = idx % I8_UNITS, oj = idx / I8_UNITS;
      const int o = oj / g, j = oj - o * g;
      st_src[it] = oj * 1024 + u * 16;
      st_j[it] = idx < nops * g * I8_UNITS ? j : Sp;  // Sp: never stored
      st_dst[it] = reinterpret_cast<int8_t*>(out) +
                   ((((int64_t)rt * per_tile + (int64_t)o * Sstride + pad_lo + j) * kb + kt) * 1024 + u * 16);
    }
  }
  for (int c = nchunks - 1; c >= 0; --c) {
    unsigned char* buf = lds_raw + (NBUF == 2 ? (c & 1) * buf_bytes : 0);
    DT* lds = reinterpret_cast<DT*>(buf);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      int64_t fre = (int64_t)(sre[q].window56(op.re.ls, nbits, L, low_mask, bad) & wmask);
      int64_t fim = (int64_t)(sim[q].window56(op.im.ls, nbits, L, low_mask, bad) & wmask);
      if (e[q].neg_re) fre = -fre;
      if (e[q].neg_im) fim = -fim;
      if (TWO) {  // the second operand's windows, signed (sign2 folded into neg)
        int64_t gre = (int64_t)(sre2[q].window56(op2->re.ls, nbits, L, low_mask, bad) & wmask);
        int64_t gim = (int64_t)(sim2[q].window56(op2->im.ls, nbits, L, low_mask, bad) & wmask);
        fre += e2[q].neg_re ? -gre : gre;
        fim += e2[q].neg_im ? -gim : gim;
      }
      int64_t v[3];
      v[0] = fre + carry[q][0];
      v[1] = fim + carry[q][1];
      // the third plane: Re + Im (3M), -Im (4M B side) with a carry chain
      // of its own, since negating a digit of -2^(w-1) would leave the range,
      // or Re again (the B side of separately scaled parts)
      v[2] = (third == (int)Third::SUM)      ? fre + fim + carry[q][2]
             : (third == (int)Third::NEG_IM) ? carry[q][2] - fim
             : (third == (int)Third::RE)     ? fre + carry[q][2]
                                             : 0;
      const bool top = c == 0;  // the chunk holding digit 0, which keeps the remaining value
      (void)top;
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        if (o == 2 && nops == 2) break;
        const int64_t u = v[o] + (int64_t)kfield;
        carry[q][o] = u >> nbits;
        if constexpr (sizeof(DT) == 1) {
          // w = 8: each byte of u ^ kfield is a digit as int8 (the top digit
          // of the top chunk, which fits, is the same byte as its full value)
          const uint64_t b = (uint64_t)u ^ kfield;
#pragma unroll
          for (int i = 0; i < 56 / 8; ++i) lds[(o * g + (g - 1 - i)) * FRAG + lofs[q]] = (DT)(int8_t)(b >> (8 * i));
        } else {
          for (int i = 0; i < g; ++i) {
            const int64_t d = (top && i == g - 1) ? (u >> (w * i)) - half : ((u >> (w * i)) & dmask) - half;
            lds[(o * g + (g - 1 - i)) * FRAG + lofs[q]] = (DT)d;
          }
        }
      }
    }
    __syncthreads();
    // write the chunk's digit tiles: contiguous (op, digit) fragments of FRAG_BYTES
    if constexpr (sizeof(DT) == 1) {
      const size_t adv = (size_t)c * st_step;
#pragma unroll
      for (int it = 0; it < I8_ITEMS; ++it) {
        if (g * c + st_j[it] >= Sp) continue;
        *reinterpret_cast<uint4*>(st_dst[it] + adv) = *reinterpret_cast<const uint4*>(buf + st_src[it]);
      }
    } else {
      constexpr int units = Layout<DT>::FRAG_BYTES / 16;
      for (int idx = t; idx < nops * g * units; idx += SPLIT_THREADS) {
        const int u = idx % units;
        const int oj = idx / units;  // = o * g + j
        const int o = oj / g, j = oj % g;
        const int s = g * c + j;
        if (s >= Sp) continue;
        const uint4* src = reinterpret_cast<const uint4*>(buf + (size_t)oj * Layout<DT>::FRAG_BYTES);
        // doubles: one column-major matrix of leading dimension cm_ld whose
        // row (plane, slice, r) is (o Sstride + pad_lo + s) Rpad + r; the
        // fragment holds 16 consecutive rows of each of its 64 columns
        const int kl = u >> 3, q2 = u & 7;
        const int64_t row0 = ((int64_t)o * Sstride + pad_lo + s) * Rpad + (int64_t)rt * 16;
        double* dst = reinterpret_cast<double*>(out) + ((int64_t)kt * 64 + kl) * cm_ld + row0 + 2 * q2;
        *reinterpret_cast<uint4*>(dst) = src[u];
      }
    }
    if (NBUF == 1) __syncthreads();
  }
  if (bad) atomicOr(status, ST_DENORM);
  // zero slices around the digits (this tile of every plane); planes whose
  // pads are shared (Sstride = pad_lo + Sp) have only lower ones, and the
  // last row tile also writes the pad after its last plane
  const int npad = Sstride - Sp;
  const int ntail = (sizeof(DT) == 1 && npad == pad_lo && rt == Rpad / 16 - 1) ? pad_lo : 0;
  if (npad > 0) {
    constexpr int units = Layout<DT>::FRAG_BYTES / 16;
    for (int idx = t; idx < (nops * npad + ntail) * units; idx += SPLIT_THREADS) {
      const int u = idx % units;
      const int oj = idx / units;
      const int o = oj / npad, j = oj % npad;  // o == nops: the pad after the last plane
      const int sl = j < pad_lo ? j : Sp + j;  // plane slice index
      uint4* dst = reinterpret_cast<uint4*>(reinterpret_cast<unsigned char*>(out) +
                                            Layout<DT>::tile_base((int64_t)o * Sstride + sl, rt, kt, Rpad / 16, Kpad,
                                                                  (int64_t)nops * Sstride));
      dst[u] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
}

template <typename DT, bool ROWCONTIG, int WC, int TH>
__global__ __launch_bounds__(SPLIT_THREADS) void split_kernel(DOperand op, int prec, int L, int S, int Sp, int Sstride,
                                                    int pad_lo, int w, int third,
                                                    const int32_t* __restrict__ G, int Rpad, int Kpad,
                                                    DT* __restrict__ out, int* status, int64_t cm_ld) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  split_tile<DT, ROWCONTIG, WC, TH>(op, prec, L, S, Sp, Sstride, pad_lo, w, third, G, Rpad, Kpad, out, status,
                                    blockIdx.x, blockIdx.y, lds_raw, nullptr, 0, nullptr, cm_ld);
}

// INT8 split of op + sign2 * op2.
template <bool ROWCONTIG, int TH>
__global__ __launch_bounds__(SPLIT_THREADS) void split2_kernel(DOperand op, DOperand op2, int sign2, int prec, int L,
                                                     int S, int Sp, int Sstride, int pad_lo,
                                                     const int32_t* __restrict__ G, int Rpad, int Kpad,
                                                     int8_t* __restrict__ out, int* status) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  split_tile<int8_t, ROWCONTIG, I8_W, TH, true>(op, prec, L, S, Sp, Sstride, pad_lo, I8_W, TH, G, Rpad, Kpad, out,
                                                 status, blockIdx.x, blockIdx.y, lds_raw, &op2, sign2);
}

// Both operands of a product: blocks [0, nA) split A (rows contiguous), the
// rest B (contraction contiguous); the first contraction tile's blocks store
// their rows' scales.
template <int THA, int THB>
__global__ __launch_bounds__(SPLIT_THREADS) void split_pair_kernel(SplitPair a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int kts = a.Kpad / 64;
  const int nA = kts * (a.mpad / 16);
  int blk = blockIdx.x;
  if (blk < nA) {
    const int kt = blk % kts, rt = blk / kts;
    if (kt == 0 && threadIdx.x < 16) {
      const int r = rt * 16 + threadIdx.x;
      a.G[r] = r < a.a.R ? row_scale(a.sa, r, a.x) : 0;
    }
    split_tile<int8_t, true, I8_W, THA>(a.a, a.prec, a.L, a.SA, a.SAp, a.xs, a.xlo, I8_W, THA, nullptr, a.mpad,
                                        a.Kpad, a.X, a.status, kt, rt, lds_raw, nullptr, 0, nullptr, 0, a.sa, a.x);
  } else {
    blk -= nA;
    const int kt = blk % kts, rt = blk / kts;
    if (kt == 0 && threadIdx.x < 16) {
      const int r = rt * 16 + threadIdx.x;
      a.H[r] = r < a.b.R ? row_scale(a.sb, r, a.x) : 0;
    }
    split_tile<int8_t, false, I8_W, THB>(a.b, a.prec, a.L, a.SB, a.SBp, a.ys, a.ylo, I8_W, THB, nullptr, a.npad,
                                         a.Kpad, a.Y, a.status, kt, rt, lds_raw, nullptr, 0, nullptr, 0, a.sb, a.x);
  }
}

// INT8 split with separate row scales for the Re (G) and Im (Gim) parts.
template <bool ROWCONTIG, int TH>
__global__ __launch_bounds__(SPLIT_THREADS) void split_parts_kernel(DOperand op, int prec, int L, int S, int Sp,
                                                          int Sstride, int pad_lo, const int32_t* __restrict__ G,
                                                          const int32_t* __restrict__ Gim, int Rpad, int Kpad,
                                                          int8_t* __restrict__ out, int* status) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  split_tile<int8_t, ROWCONTIG, I8_W, TH>(op, prec, L, S, Sp, Sstride, pad_lo, I8_W, TH, G, Rpad, Kpad, out, status,
                                          blockIdx.x, blockIdx.y, lds_raw, nullptr, 0, Gim);
}

// The A sides (rows contiguous) and the B sides of a batch in one launch:
// blocks [0, blocks_a) take A's jobs, the rest B's.
__global__ __launch_bounds__(SPLIT_THREADS) void split_i8_batched_pair(const SplitJob* __restrict__ ja, int na,
                                                             const int* __restrict__ fa, int blocks_a,
                                                             const SplitJob* __restrict__ jb, int nb,
                                                             const int* __restrict__ fb, int prec, int L,
                                                             int* status) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  if ((int)blockIdx.x < blocks_a) {
    const int j = job_of_block(fa, na, blockIdx.x);
    const SplitJob& J = ja[j];
    const int local = blockIdx.x - fa[j];
    const int kts = J.Kpad / 64;
    split_tile<int8_t, true, I8_W, -1>(J.op, prec, L, J.S, J.Sp, J.Sstride, J.pad_lo, I8_W, J.third, J.G, J.Rpad,
                                       J.Kpad, J.out, status, local % kts, local / kts, lds_raw);
  } else {
    const int b = blockIdx.x - blocks_a;
    const int j = job_of_block(fb, nb, b);
    const SplitJob& J = jb[j];
    const int local = b - fb[j];
    const int kts = J.Kpad / 64;
    split_tile<int8_t, false, I8_W, -1>(J.op, prec, L, J.S, J.Sp, J.Sstride, J.pad_lo, I8_W, J.third, J.G, J.Rpad,
                                        J.Kpad, J.out, status, local % kts, local / kts, lds_raw);
  }
}

template <typename DT, int WC, int TH>
hipError_t launch_split_t(const DOperand& op, int prec, int L, int S, int Sp, int Sstride, int pad_lo, int w,
                          Third third, const int32_t* G, int Rpad, int Kpad, DT* out, int* status,
                          hipStream_t stream, int64_t cm_ld = 0) {
  const int g = 56 / w;
  const int nops = third == Third::NONE ? 2 : 3;
  const size_t lds = (size_t)(sizeof(DT) == 1 ? 2 : 1) * nops * g * Layout<DT>::FRAG_BYTES;
  dim3 grid(Kpad / 64, Rpad / 16);
  if (op.rs == 1)
    split_kernel<DT, true, WC, TH><<<grid, dim3(SPLIT_THREADS), lds, stream>>>(op, prec, L, S, Sp, Sstride, pad_lo,
                                                                                w, (int)third, G, Rpad, Kpad, out,
                                                                                status, cm_ld);
  else
    split_kernel<DT, false, WC, TH><<<grid, dim3(SPLIT_THREADS), lds, stream>>>(op, prec, L, S, Sp, Sstride, pad_lo,
                                                                                 w, (int)third, G, Rpad, Kpad, out,
                                                                                 status, cm_ld);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_split_i8(const DOperand& op, int prec, int L, int S, int Sp, int Sstride, int pad_lo,
                           Third third, const int32_t* G, int Rpad, int Kpad, int8_t* out, int* status,
                           hipStream_t stream) {
  switch (third) {
    case Third::NONE:
      return launch_split_t<int8_t, I8_W, 0>(op, prec, L, S, Sp, Sstride, pad_lo, I8_W, third, G, Rpad, Kpad, out, status,
                                          stream);
    case Third::SUM:
      return launch_split_t<int8_t, I8_W, 1>(op, prec, L, S, Sp, Sstride, pad_lo, I8_W, third, G, Rpad, Kpad, out, status,
                                          stream);
    default:
      return launch_split_t<int8_t, I8_W, 2>(op, prec, L, S, Sp, Sstride, pad_lo, I8_W, third, G, Rpad, Kpad, out, status,
                                          stream);
  }
}

hipError_t launch_split2_i8(const DOperand& op, const DOperand& op2, int sign2, int prec, int L, int S, int Sp,
                            int Sstride, int pad_lo, Third third, const int32_t* G, int Rpad, int Kpad, int8_t* out,
                            int* status, hipStream_t stream) {
  const int nops = third == Third::NONE ? 2 : 3;
  const size_t lds = (size_t)2 * nops * (56 / I8_W) * Layout<int8_t>::FRAG_BYTES;
  dim3 grid(Kpad / 64, Rpad / 16);
  const bool rc = op.rs == 1;
#define MPCG_SPLIT2(RC, T)                                                                                      \
  split2_kernel<RC, T><<<grid, dim3(SPLIT_THREADS), lds, stream>>>(op, op2, sign2, prec, L, S, Sp, Sstride, pad_lo, \
                                                                   G, Rpad, Kpad, out, status)
  switch (third) {
    case Third::NONE:
      if (rc) MPCG_SPLIT2(true, 0); else MPCG_SPLIT2(false, 0);
      break;
    case Third::SUM:
      if (rc) MPCG_SPLIT2(true, 1); else MPCG_SPLIT2(false, 1);
      break;
    default:
      if (rc) MPCG_SPLIT2(true, 2); else MPCG_SPLIT2(false, 2);
      break;
  }
#undef MPCG_SPLIT2
  return hipGetLastError();
}

hipError_t launch_split_parts_i8(const DOperand& op, int prec, int L, int S, int Sp, int Sstride, int pad_lo,
                                 Third third, const int32_t* G, const int32_t* Gim, int Rpad, int Kpad, int8_t* out,
                                 int* status, hipStream_t stream) {
  if (third != Third::NONE && third != Third::RE) return hipErrorInvalidValue;
  const int nops = third == Third::NONE ? 2 : 3;
  const size_t lds = (size_t)2 * nops * (56 / I8_W) * Layout<int8_t>::FRAG_BYTES;
  dim3 grid(Kpad / 64, Rpad / 16);
  const bool rc = op.rs == 1;
#define MPCG_SPLITP(RC, T)                                                                                        \
  split_parts_kernel<RC, T><<<grid, dim3(SPLIT_THREADS), lds, stream>>>(op, prec, L, S, Sp, Sstride, pad_lo, G, Gim, \
                                                                        Rpad, Kpad, out, status)
  if (third == Third::NONE) {
    if (rc) MPCG_SPLITP(true, 0); else MPCG_SPLITP(false, 0);
  } else {
    if (rc) MPCG_SPLITP(true, 3); else MPCG_SPLITP(false, 3);
  }
#undef MPCG_SPLITP
  return hipGetLastError();
}

hipError_t launch_split_pair_i8(const SplitPair& a, bool mode3m, hipStream_t stream) {
  const int kts = a.Kpad / 64;
  const int blocks = kts * (a.mpad / 16) + kts * (a.npad / 16);
  const size_t lds = (size_t)2 * 3 * (56 / I8_W) * Layout<int8_t>::FRAG_BYTES;  // two buffers of up to three planes
  if (mode3m)
    split_pair_kernel<1, 1><<<dim3(blocks), dim3(SPLIT_THREADS), lds, stream>>>(a);
  else
    split_pair_kernel<0, 2><<<dim3(blocks), dim3(SPLIT_THREADS), lds, stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_split_f64(const DOperand& op, int prec, int L, int S, int Sp, int w, Third third,
                            const int32_t* G, int Rpad, int Kpad, double* out, int* status, hipStream_t stream) {
  const int nops = third == Third::NONE ? 2 : 3;
  return launch_split_t<double, 0, -1>(op, prec, L, S, Sp, Sp, 0, w, third, G, Rpad, Kpad, out, status, stream,
                                       (int64_t)nops * Sp * Rpad);
}

hipError_t launch_split_i8_batched_pair(const SplitJob* ja, const int* fa, int blocks_a, const SplitJob* jb,
                                        const int* fb, int blocks_b, int njobs, int prec, int L, int* status,
                                        hipStream_t stream) {
  if (njobs <= 0 || blocks_a + blocks_b <= 0) return hipSuccess;
  const size_t lds = (size_t)2 * 3 * (56 / I8_W) * Layout<int8_t>::FRAG_BYTES;  // two buffers of up to three planes
  split_i8_batched_pair<<<dim3(blocks_a + blocks_b), dim3(SPLIT_THREADS), lds, stream>>>(ja, njobs, fa, blocks_a, jb,
                                                                                         njobs, fb, prec, L, status);
  return hipGetLastError();
}

}  // namespace mpcg
