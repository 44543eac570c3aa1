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
//         zero slices around the digits (Sstride slices per plane).
//   FP64: fragment = 16 rows x 4 k, lane l holds row l%16, k = l/16 (one
//         double), planes [op][s][R/16][K/4][64 doubles].
#include "mpcg_internal.h"

namespace mpcg {

namespace {

// A block splits one 16 x 64 tile, EPT entries per thread.
constexpr int SPLIT_THREADS = 1024;
constexpr int EPT = 1024 / SPLIT_THREADS;

// Limb li of one significand (0 outside [0, L); limb 0 masked to the
// precision); `denorm` collects a clear top bit of limb L-1.
__device__ inline uint64_t limb_at(const uint64_t* m, int64_t ls, int64_t li, int L, uint64_t low_mask,
                                   int& denorm) {
  if (!m || li < 0 || li >= L) return 0;
  uint64_t v = m[li * ls];
  if (li == L - 1) denorm |= !(v >> 63);
  return li == 0 ? (v & low_mask) : v;
}

// Bits [pos, pos + 56) of one significand for pos rising by at most 64 per
// call: limbs li, li + 1 and (loaded a window ahead) li + 2, so every limb is
// read once.
struct LimbStream {
  const uint64_t* m;  // mant + entry index, NULL for a zero entry
  int64_t li;
  uint64_t a, b, c;
  __device__ inline void start(const uint64_t* mp, int64_t ls, int64_t pos, int L, uint64_t low_mask,
                               int& denorm) {
    m = mp;
    li = pos >> 6;  // floor
    a = limb_at(m, ls, li, L, low_mask, denorm);
    b = limb_at(m, ls, li + 1, L, low_mask, denorm);
    c = limb_at(m, ls, li + 2, L, low_mask, denorm);
  }
  __device__ inline uint64_t window56(int64_t ls, int64_t pos, int L, uint64_t low_mask, int& denorm) {
    if ((pos >> 6) > li) {
      ++li;
      a = b;
      b = c;
      c = limb_at(m, ls, li + 2, L, low_mask, denorm);
    }
    const int off = (int)(pos - 64 * li);
    const uint64_t r = off ? ((a >> off) | (b << (64 - off))) : a;
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
                                  const int32_t* __restrict__ Gim = nullptr, int64_t cm_ld = 0) {
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
        const int64_t base = (int64_t)G[r] - wS + 64 * (int64_t)L;  // sh = exp - base
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

  const int64_t half = 1ll << (w - 1);
  const int64_t dmask = (1ll << w) - 1;
  int64_t carry[EPT][3];
#pragma unroll
  for (int q = 0; q < EPT; ++q) carry[q][0] = carry[q][1] = carry[q][2] = 0;

  const int nchunks = (Sp + g - 1) / g;
  const int nbits = g * w;  // <= 56
  const uint64_t wmask = (1ull << nbits) - 1ull;
  {
    const int64_t f0 = (int64_t)w * (S - g * (nchunks - 1) - g);  // lowest window's first F bit
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      sre[q].start(e[q].z_re ? nullptr : op.re.mant + e[q].idx, op.re.ls, f0 - e[q].sh_re, L, low_mask, bad);
      sim[q].start(e[q].z_im ? nullptr : op.im.mant + e[q].idx, op.im.ls, f0 - e[q].sh_im, L, low_mask, bad);
      if (TWO) {
        sre2[q].start(e2[q].z_re ? nullptr : op2->re.mant + e2[q].idx, op2->re.ls, f0 - e2[q].sh_re, L, low_mask,
                      bad);
        sim2[q].start(e2[q].z_im ? nullptr : op2->im.mant + e2[q].idx, op2->im.ls, f0 - e2[q].sh_im, L, low_mask,
                      bad);
      }
    }
  }
  const int buf_bytes = nops * g * Layout<DT>::FRAG_BYTES;
  for (int c = nchunks - 1; c >= 0; --c) {
    unsigned char* buf = lds_raw + (NBUF == 2 ? (c & 1) * buf_bytes : 0);
    DT* lds = reinterpret_cast<DT*>(buf);
    const int64_t fstart = (int64_t)w * (S - g * c - g);  // F bit of the window's lowest digit
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      int64_t fre = (int64_t)(sre[q].window56(op.re.ls, fstart - e[q].sh_re, L, low_mask, bad) & wmask);
      int64_t fim = (int64_t)(sim[q].window56(op.im.ls, fstart - e[q].sh_im, L, low_mask, bad) & wmask);
      if (e[q].neg_re) fre = -fre;
      if (e[q].neg_im) fim = -fim;
      if (TWO) {  // the second operand's windows, signed (sign2 folded into neg)
        int64_t gre = (int64_t)(sre2[q].window56(op2->re.ls, fstart - e2[q].sh_re, L, low_mask, bad) & wmask);
        int64_t gim = (int64_t)(sim2[q].window56(op2->im.ls, fstart - e2[q].sh_im, L, low_mask, bad) & wmask);
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
#pragma unroll
      for (int j = g - 1; j >= 0; --j) {
        DT dig[3];
#pragma unroll
        for (int o = 0; o < 3; ++o) {
          int64_t d;
          if (top && j == 0) {
            d = v[o];
          } else {
            d = ((v[o] + half) & dmask) - half;
            v[o] = (v[o] - d) >> w;
          }
          dig[o] = (DT)d;
        }
        lds[(0 * g + j) * FRAG + lofs[q]] = dig[0];
        lds[(1 * g + j) * FRAG + lofs[q]] = dig[1];
        if (nops == 3) lds[(2 * g + j) * FRAG + lofs[q]] = dig[2];
      }
      carry[q][0] = v[0];
      carry[q][1] = v[1];
      carry[q][2] = v[2];
    }
    __syncthreads();
    // write the chunk's digit tiles: contiguous (op, digit) fragments of FRAG_BYTES
    constexpr int units = Layout<DT>::FRAG_BYTES / 16;
    for (int idx = t; idx < nops * g * units; idx += SPLIT_THREADS) {
      const int u = idx % units;
      const int oj = idx / units;  // = o * g + j
      const int o = oj / g, j = oj % g;
      const int s = g * c + j;
      if (s >= Sp) continue;
      const uint4* src = reinterpret_cast<const uint4*>(buf + (size_t)oj * Layout<DT>::FRAG_BYTES);
      if constexpr (sizeof(DT) == 8) {
        // doubles: one column-major matrix of leading dimension cm_ld whose
        // row (plane, slice, r) is (o Sstride + pad_lo + s) Rpad + r; the
        // fragment holds 16 consecutive rows of each of its 64 columns
        const int kl = u >> 3, q2 = u & 7;
        const int64_t row0 = ((int64_t)o * Sstride + pad_lo + s) * Rpad + (int64_t)rt * 16;
        double* dst = reinterpret_cast<double*>(out) + ((int64_t)kt * 64 + kl) * cm_ld + row0 + 2 * q2;
        *reinterpret_cast<uint4*>(dst) = src[u];
      } else {
        uint4* dst = reinterpret_cast<uint4*>(reinterpret_cast<unsigned char*>(out) +
                                              Layout<DT>::tile_base((int64_t)o * Sstride + pad_lo + s, rt, kt,
                                                                    Rpad / 16, Kpad, (int64_t)nops * Sstride));
        dst[u] = src[u];
      }
    }
    if (NBUF == 1) __syncthreads();
  }
  if (bad) atomicOr(status, ST_DENORM);
  // zero slices around the digits (this tile of every plane)
  const int npad = Sstride - Sp;
  if (npad > 0) {
    constexpr int units = Layout<DT>::FRAG_BYTES / 16;
    for (int idx = t; idx < nops * npad * units; idx += SPLIT_THREADS) {
      const int u = idx % units;
      const int oj = idx / units;
      const int o = oj / npad, j = oj % npad;
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

// Batched INT8 form: job j owns (Kpad/64) * (Rpad/16) blocks.
template <bool ROWCONTIG>
__global__ __launch_bounds__(SPLIT_THREADS) void split_i8_batched(const SplitJob* __restrict__ jobs, int njobs,
                                                        const int* __restrict__ first, int prec, int L,
                                                        int* status) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int j = job_of_block(first, njobs, blockIdx.x);
  const SplitJob& J = jobs[j];
  const int local = blockIdx.x - first[j];
  const int kts = J.Kpad / 64;
  split_tile<int8_t, ROWCONTIG, I8_W, -1>(J.op, prec, L, J.S, J.Sp, J.Sstride, J.pad_lo, I8_W, J.third, J.G, J.Rpad,
                                       J.Kpad, J.out, status, local % kts, local / kts, lds_raw);
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

hipError_t launch_split_f64(const DOperand& op, int prec, int L, int S, int Sp, int w, Third third,
                            const int32_t* G, int Rpad, int Kpad, double* out, int* status, hipStream_t stream) {
  const int nops = third == Third::NONE ? 2 : 3;
  return launch_split_t<double, 0, -1>(op, prec, L, S, Sp, Sp, 0, w, third, G, Rpad, Kpad, out, status, stream,
                                       (int64_t)nops * Sp * Rpad);
}

hipError_t launch_split_i8_batched(const SplitJob* jobs, int njobs, const int* first, int blocks, int prec, int L,
                                   bool rows_contiguous, int* status, hipStream_t stream) {
  if (njobs <= 0 || blocks <= 0) return hipSuccess;
  const size_t lds = (size_t)2 * 3 * (56 / I8_W) * Layout<int8_t>::FRAG_BYTES;  // two buffers of up to three planes
  if (rows_contiguous)
    split_i8_batched<true><<<dim3(blocks), dim3(SPLIT_THREADS), lds, stream>>>(jobs, njobs, first, prec, L, status);
  else
    split_i8_batched<false><<<dim3(blocks), dim3(SPLIT_THREADS), lds, stream>>>(jobs, njobs, first, prec, L, status);
  return hipGetLastError();
}

}  // namespace mpcg
