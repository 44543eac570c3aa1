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
// exactly from the two signed windows with one shared carry; in the 4M form
// the B side's third plane holds the digits of -Im x so that
// Re(A)Re(B) - Im(A)Im(B) accumulates as a sum (eq. 5).
//
// One block handles a 16 x 64 tile (16 rows of the operand, 64 contraction
// indices).  Digits go to LDS in the matrix-core operand order and leave as
// contiguous fragments:
//   INT8: fragment = 16 rows x 64 k, lane l holds row l%16, k = 16*(l/16)..+16
//         (16 bytes), tile-major [R/16][op][pad_lo + s][K/64][1024 B] with
//         zero slices around the digits (Sstride slices per plane).
//   FP64: fragment = 16 rows x 4 k, lane l holds row l%16, k = l/16 (one
//         double), planes [op][s][R/16][K/4][64 doubles].
#include "mpcg_internal.h"

namespace mpcg {

namespace {

// Bits [pos, pos + nbits) of the significand M (nbits <= 56); bits below the
// precision (mask on limb 0) and outside [0, 64L) read as zero.
__device__ inline uint64_t window_bits(const uint64_t* mant, int64_t ls, int64_t idx, int L,
                                       uint64_t low_mask, int64_t pos, int nbits) {
  const int64_t li = pos >> 6;  // floor
  const int off = (int)(pos & 63);
  uint64_t a = 0, b = 0;
  if (li >= 0 && li < L) {
    a = mant[li * ls + idx];
    if (li == 0) a &= low_mask;
  }
  if (li + 1 >= 0 && li + 1 < L) {
    b = mant[(li + 1) * ls + idx];
    if (li + 1 == 0) b &= low_mask;
  }
  const uint64_t r = off ? ((a >> off) | (b << (64 - off))) : a;
  return r & ((1ull << nbits) - 1ull);
}

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

template <typename DT, bool ROWCONTIG>
__device__ inline void split_tile(const DOperand& op, int prec, int L, int S, int Sp, int Sstride, int pad_lo,
                                  int w, int third, const int32_t* __restrict__ G, int Rpad, int Kpad,
                                  DT* __restrict__ out, int* status, int kt, int rt, unsigned char* lds_raw) {
  DT* lds = reinterpret_cast<DT*>(lds_raw);
  constexpr int FRAG = Layout<DT>::FRAG_BYTES / (int)sizeof(DT);  // elements per (op, digit) tile

  const int g = 56 / w;  // digits per window
  const int nops = third ? 3 : 2;
  const int t = threadIdx.x;
  const uint64_t low_mask = ~((1ull << (64 * L - prec)) - 1ull) | (64 * L - prec == 0 ? ~0ull : 0ull);
  const int64_t wS = (int64_t)w * S;

  Entry e[4];
  int lofs[4];
  int bad = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int rl, kl;
    if (ROWCONTIG) {
      rl = t & 15;
      kl = (t >> 4) + 16 * q;
    } else {
      kl = t & 63;
      rl = (t >> 6) + 4 * q;
    }
    lofs[q] = Layout<DT>::offset(rl, kl);
    const int r = rt * 16 + rl, kk = kt * 64 + kl;
    e[q].z_re = e[q].z_im = 1;
    e[q].neg_re = e[q].neg_im = 0;
    e[q].sh_re = e[q].sh_im = 0;
    e[q].idx = 0;
    if (r < op.R && kk < op.K) {
      const int64_t idx = (int64_t)r * op.rs + (int64_t)kk * op.ks;
      e[q].idx = idx;
      const int64_t base = (int64_t)G[r] - wS + 64 * (int64_t)L;  // sh = exp - base
      const int32_t er = op.re.exp[idx], ei = op.im.exp[idx];
      if (er != EXP_ZERO) {
        e[q].z_re = 0;
        e[q].neg_re = op.re.sign[idx] ? 1 : 0;
        e[q].sh_re = (int64_t)er - base;
        bad |= !(op.re.mant[(int64_t)(L - 1) * op.re.ls + idx] >> 63);
      }
      if (ei != EXP_ZERO) {
        e[q].z_im = 0;
        e[q].neg_im = op.im.sign[idx] ? 1 : 0;
        e[q].sh_im = (int64_t)ei - base;
        bad |= !(op.im.mant[(int64_t)(L - 1) * op.im.ls + idx] >> 63);
      }
    }
  }
  if (bad) atomicOr(status, ST_DENORM);

  const int64_t half = 1ll << (w - 1);
  const int64_t dmask = (1ll << w) - 1;
  int64_t carry[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) carry[q][0] = carry[q][1] = carry[q][2] = 0;

  const int nchunks = (Sp + g - 1) / g;
  for (int c = nchunks - 1; c >= 0; --c) {
    const int64_t fstart = (int64_t)w * (S - g * c - g);  // F bit of the window's lowest digit
    const int nbits = g * w;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int64_t fre = 0, fim = 0;
      if (!e[q].z_re)
        fre = (int64_t)window_bits(op.re.mant, op.re.ls, e[q].idx, L, low_mask, fstart - e[q].sh_re, nbits);
      if (!e[q].z_im)
        fim = (int64_t)window_bits(op.im.mant, op.im.ls, e[q].idx, L, low_mask, fstart - e[q].sh_im, nbits);
      if (e[q].neg_re) fre = -fre;
      if (e[q].neg_im) fim = -fim;
      int64_t v[3];
      v[0] = fre + carry[q][0];
      v[1] = fim + carry[q][1];
      v[2] = (third == (int)Third::SUM) ? fre + fim + carry[q][2] : 0;
      for (int j = g - 1; j >= 0; --j) {
        const int s = g * c + j;
        DT dig[3];
#pragma unroll
        for (int o = 0; o < 3; ++o) {
          int64_t d;
          if (s == 0) {
            d = v[o];  // topmost digit keeps the remaining value
          } else {
            d = ((v[o] + half) & dmask) - half;
            v[o] = (v[o] - d) >> w;
          }
          dig[o] = (DT)d;
        }
        if (third == (int)Third::NEG_IM) dig[2] = (DT)(-dig[1]);
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
    for (int idx = t; idx < nops * g * units; idx += 256) {
      const int u = idx % units;
      const int oj = idx / units;  // = o * g + j
      const int o = oj / g, j = oj % g;
      const int s = g * c + j;
      if (s >= Sp) continue;
      const uint4* src = reinterpret_cast<const uint4*>(lds_raw + (size_t)oj * Layout<DT>::FRAG_BYTES);
      uint4* dst = reinterpret_cast<uint4*>(reinterpret_cast<unsigned char*>(out) +
                                            Layout<DT>::tile_base((int64_t)o * Sstride + pad_lo + s, rt, kt,
                                                                  Rpad / 16, Kpad, (int64_t)nops * Sstride));
      dst[u] = src[u];
    }
    __syncthreads();
  }
  // zero slices around the digits (this tile of every plane)
  const int npad = Sstride - Sp;
  if (npad > 0) {
    constexpr int units = Layout<DT>::FRAG_BYTES / 16;
    for (int idx = t; idx < nops * npad * units; idx += 256) {
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

template <typename DT, bool ROWCONTIG>
__global__ __launch_bounds__(256) void split_kernel(DOperand op, int prec, int L, int S, int Sp, int Sstride,
                                                    int pad_lo, int w, int third,
                                                    const int32_t* __restrict__ G, int Rpad, int Kpad,
                                                    DT* __restrict__ out, int* status) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  split_tile<DT, ROWCONTIG>(op, prec, L, S, Sp, Sstride, pad_lo, w, third, G, Rpad, Kpad, out, status, blockIdx.x,
                            blockIdx.y, lds_raw);
}

// Batched INT8 form: job j owns (Kpad/64) * (Rpad/16) blocks.
template <bool ROWCONTIG>
__global__ __launch_bounds__(256) void split_i8_batched(const SplitJob* __restrict__ jobs, int njobs,
                                                        const int* __restrict__ first, int prec, int L,
                                                        int* status) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int j = job_of_block(first, njobs, blockIdx.x);
  const SplitJob& J = jobs[j];
  const int local = blockIdx.x - first[j];
  const int kts = J.Kpad / 64;
  split_tile<int8_t, ROWCONTIG>(J.op, prec, L, J.S, J.Sp, J.Sstride, J.pad_lo, 7, J.third, J.G, J.Rpad, J.Kpad,
                                J.out, status, local % kts, local / kts, lds_raw);
}

template <typename DT>
hipError_t launch_split_t(const DOperand& op, int prec, int L, int S, int Sp, int Sstride, int pad_lo, int w,
                          Third third, const int32_t* G, int Rpad, int Kpad, DT* out, int* status,
                          hipStream_t stream) {
  const int g = 56 / w;
  const int nops = third == Third::NONE ? 2 : 3;
  const size_t lds = (size_t)nops * g * Layout<DT>::FRAG_BYTES;
  dim3 grid(Kpad / 64, Rpad / 16);
  if (op.rs == 1)
    split_kernel<DT, true><<<grid, dim3(256), lds, stream>>>(op, prec, L, S, Sp, Sstride, pad_lo, w, (int)third, G, Rpad, Kpad,
                                                             out, status);
  else
    split_kernel<DT, false><<<grid, dim3(256), lds, stream>>>(op, prec, L, S, Sp, Sstride, pad_lo, w, (int)third, G, Rpad, Kpad,
                                                              out, status);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_split_i8(const DOperand& op, int prec, int L, int S, int Sp, int Sstride, int pad_lo,
                           Third third, const int32_t* G, int Rpad, int Kpad, int8_t* out, int* status,
                           hipStream_t stream) {
  return launch_split_t<int8_t>(op, prec, L, S, Sp, Sstride, pad_lo, 7, third, G, Rpad, Kpad, out, status, stream);
}

hipError_t launch_split_f64(const DOperand& op, int prec, int L, int S, int Sp, int w, Third third,
                            const int32_t* G, int Rpad, int Kpad, double* out, int* status, hipStream_t stream) {
  return launch_split_t<double>(op, prec, L, S, Sp, Sp, 0, w, third, G, Rpad, Kpad, out, status, stream);
}

hipError_t launch_split_i8_batched(const SplitJob* jobs, int njobs, const int* first, int blocks, int prec, int L,
                                   bool rows_contiguous, int* status, hipStream_t stream) {
  if (njobs <= 0 || blocks <= 0) return hipSuccess;
  const size_t lds = (size_t)3 * (56 / 7) * Layout<int8_t>::FRAG_BYTES;  // up to three planes
  if (rows_contiguous)
    split_i8_batched<true><<<dim3(blocks), dim3(256), lds, stream>>>(jobs, njobs, first, prec, L, status);
  else
    split_i8_batched<false><<<dim3(blocks), dim3(256), lds, stream>>>(jobs, njobs, first, prec, L, status);
  return hipGetLastError();
}

}  // namespace mpcg
