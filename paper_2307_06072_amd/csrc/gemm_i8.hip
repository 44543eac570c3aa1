// Slice-pair products on the INT8 matrix cores, fused with the exact
// combination of the real products and the carry chain.
//
// With A = diag(2^G) sum_s X_s 2^(-w(s+1)) and B = sum_t Y_t 2^(-w(t+1)) diag(2^H)
// (balanced 7-bit digits, |digit| <= 64), every real product is
//     X Y = diag(2^G) [ sum_d D_d 2^(-w(d+2)) ] diag(2^H),   D_d = sum_{s+t=d} X_s Y_t,
// i.e. the slice-pair products C_{alpha beta} of Algorithm 2 grouped by
// anti-diagonal d = s + t.  Each D_d is an exact integer matrix: products of
// digits are at most 2^12 in magnitude and the planner limits the terms per
// diagonal so that int32 accumulation cannot overflow.
//
// Work of one wavefront: a 16 x 16 output tile (v_mfma_i32_16x16x64_i8) and a
// contraction chunk.  The diagonals are processed in bands of W consecutive
// diagonals [d0, d0 + W), least significant band first, with one int32
// accumulator per diagonal (and per real product).  Inside a band and a 64-wide
// k-block the wave walks s upward; the B fragments Y_t with s + t in the band
// form a sliding window of W registers (a ring: slot t mod W), so each step
// loads one A fragment X_s and one new B fragment Y_{d0-s} and issues W MFMAs
// (every pair (s, t) of the band exactly once).  Loads run PF steps ahead of
// their use through a small register queue.
//
// When a band is complete its W diagonals are combined into Re and Im
// (4M, eq. 5: the accumulators already hold Re and Im, the B side supplying
// -Im B; 3M, eq. 6: T1, T2, T3 with Re = T1 - T2, Im = T3 - T1 - T2) and pushed,
// least significant first, through a per-element int64 carry chain that emits
// one normalised base-2^7 digit per diagonal; the final carry is the signed top
// of the exact result.
//
// Operand fragments (16 rows x 64 k, 16 bytes per lane) are read straight
// from the digit planes of the split kernel.  Workgroups are 2 x 2 tiles; their
// order is XCD-aware so that the workgroups resident on one XCD cover a compact
// block of the output and share operand panels in that XCD's L2.
#include "mpcg_internal.h"

namespace mpcg {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ inline v4i mfma(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

__device__ inline v4i ld(const int8_t* p) { return *reinterpret_cast<const v4i*>(p); }

// Workgroup -> (contraction chunk, 2x2 tile group).  Blocks are dispatched to
// the 8 XCDs round-robin; consecutive blocks of one XCD get consecutive
// positions of a grouped (4 tile-group rows at a time) order.
__device__ inline void map_block(int b, int nblk, int gm, int gn, int& split, int& gi, int& gj) {
  constexpr int NXCD = 8, GROUP = 4;
  const int per = nblk / NXCD, rem = nblk % NXCD;
  const int xcd = b % NXCD, slot = b / NXCD;
  const int lin = (xcd < rem) ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
  const int groups = gm * gn;
  split = lin / groups;
  const int gid = lin - split * groups;
  const int gsz = GROUP * gn;
  const int grp = gid / gsz, in = gid - grp * gsz;
  const int rows_here = min(GROUP, gm - grp * GROUP);
  gi = grp * GROUP + in % rows_here;
  gj = in / rows_here;
}

// One pass over a band: A plane xa, B plane y0 into accumulator Q0 and, when
// TWO, B plane y1 into accumulator Q1 (both sharing the A fragment).
//
// Step u = s - s_lo loads the new fragment B_{d0-s} into ring slot u mod W;
// slot r then holds the B fragment of diagonal d0 + ((u - r) mod W), so every
// register index is static inside the W-step unrolled body.  Pairs whose t
// falls outside [0, SB) meet a zero fragment: they are issued but add nothing,
// which keeps the MFMA stream free of branches (branches there would force the
// compiler to wait for every outstanding load before each MFMA).
template <int W, int PF, bool TWO, int Q0, int Q1, int NACC>
__device__ __forceinline__ void band_pass(v4i (&acc)[NACC][W], const int8_t* xa_base, const int8_t* y0_base,
                                          const int8_t* y1_base, const int8_t* zp, size_t xplane, size_t yplane,
                                          int d0, int s_lo, int s_hi, int SB, int kb0, int kb1) {
  static_assert(W % PF == 0, "look-ahead depth must divide the band width");
  // fragments outside the operand (t < 0, t >= SB, s > s_hi) are read from a
  // zero block: every load is unconditional, only its address is selected
#define MPCG_YA(base, t) (((t) >= 0 && (t) < SB) ? (base) + (size_t)(t) * yplane + ko : zp)
#define MPCG_XA(s) (((s) <= s_hi) ? xa_base + (size_t)(s) * xplane + ko : zp)
#pragma unroll 1
  for (int kb = kb0; kb < kb1; ++kb) {
    const size_t ko = (size_t)kb * 1024;
    // window before the first step: t = d0 - s_lo + q, q = 1..W-1, in slot W - q
    v4i ring0[W], ring1[TWO ? W : 1];
#pragma unroll
    for (int q = 1; q < W; ++q) {
      const int t = d0 - s_lo + q;
      ring0[W - q] = ld(MPCG_YA(y0_base, t));
      if (TWO) ring1[W - q] = ld(MPCG_YA(y1_base, t));
    }
    // look-ahead queue: the operands of step u sit in slot u mod PF
    v4i qa[PF], qb0[PF], qb1[TWO ? PF : 1];
#pragma unroll
    for (int v = 0; v < PF; ++v) {
      const int s = s_lo + v, t = s <= s_hi ? d0 - s : -1;
      qa[v] = ld(MPCG_XA(s));
      qb0[v] = ld(MPCG_YA(y0_base, t));
      if (TWO) qb1[v] = ld(MPCG_YA(y1_base, t));
    }
    for (int s0 = s_lo; s0 <= s_hi; s0 += W) {
#pragma unroll
      for (int u = 0; u < W; ++u) {
        const int s = s0 + u;
        if (s > s_hi) break;
        const v4i xa = qa[u % PF];
        ring0[u] = qb0[u % PF];
        if (TWO) ring1[u] = qb1[u % PF];
        {  // refill the queue slot with step s + PF
          const int sn = s + PF, tn = sn <= s_hi ? d0 - sn : -1;
          qa[u % PF] = ld(MPCG_XA(sn));
          qb0[u % PF] = ld(MPCG_YA(y0_base, tn));
          if (TWO) qb1[u % PF] = ld(MPCG_YA(y1_base, tn));
        }
#pragma unroll
        for (int r = 0; r < W; ++r) {
          const int j = (u - r + W) % W;  // diagonal d0 + j
          acc[Q0][j] = mfma(xa, ring0[r], acc[Q0][j]);
          if (TWO) acc[Q1][j] = mfma(xa, ring1[r], acc[Q1][j]);
        }
      }
    }
  }
#undef MPCG_YA
#undef MPCG_XA
}

template <int W, bool M3>
__global__ __launch_bounds__(256) void gemm_i8_kernel(GemmArgs a) {
  constexpr int NACC = M3 ? 3 : 2;
  constexpr int PF = W >= 16 ? 8 : 4;  // steps of load look-ahead
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;

  int split, gi, gj;
  map_block(blockIdx.x, gridDim.x, a.mt >> 1, a.nt >> 1, split, gi, gj);
  const int ti = 2 * gi + (wv & 1);
  const int tj = 2 * gj + (wv >> 1);
  const int tile = tj * a.mt + ti;
  const int kbps = (a.kblocks + a.ksplit - 1) / a.ksplit;
  const int kb0 = split * kbps;
  const int kb1 = min(a.kblocks, kb0 + kbps);

  const size_t xplane = (size_t)a.mt * a.kblocks * 1024;  // bytes per (op, s) plane
  const size_t yplane = (size_t)a.nt * a.kblocks * 1024;
  const int8_t* Xb = a.X + (size_t)ti * a.kblocks * 1024 + lane * 16;
  const int8_t* Yb = a.Y + (size_t)tj * a.kblocks * 1024 + lane * 16;
  const int SA = a.SAp, SB = a.SBp;
  const int8_t* zp = a.zero + lane * 16;

  int64_t cre[4], cim[4];
  int32_t lre[4], lim[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    cre[r] = cim[r] = 0;
    lre[r] = lim[r] = -1;
  }
  const int nd = a.Dmax + 1;
  uint64_t* dig = reinterpret_cast<uint64_t*>(a.digits) + ((size_t)(split * a.mt * a.nt + tile) * nd) * 64 + lane;

  const int nbands = (a.Dmax + W) / W;
#pragma unroll 1
  for (int band = 0; band < nbands; ++band) {
    const int d0 = a.Dmax + 1 - W * (band + 1);  // band covers diagonals [d0, d0 + W)
    v4i acc[NACC][W];
#pragma unroll
    for (int p = 0; p < NACC; ++p)
#pragma unroll
      for (int j = 0; j < W; ++j) acc[p][j] = v4i{0, 0, 0, 0};

    const int s_lo = max(0, d0 - (SB - 1)), s_hi = min(SA - 1, d0 + W - 1);
    if (s_lo <= s_hi) {
      const int8_t* X0 = Xb;
      const int8_t* X1 = Xb + (size_t)SA * xplane;
      const int8_t* Y0 = Yb;
      const int8_t* Y1 = Yb + (size_t)SB * yplane;
      const int8_t* Y2 = Yb + (size_t)2 * SB * yplane;
      if constexpr (M3) {  // T1 = Re Re, T2 = Im Im, T3 = (Re+Im)(Re+Im)
        const int8_t* X2 = Xb + (size_t)2 * SA * xplane;
        band_pass<W, PF, false, 0, 0>(acc, X0, Y0, Y0, zp, xplane, yplane, d0, s_lo, s_hi, SB, kb0, kb1);
        band_pass<W, PF, false, 1, 1>(acc, X1, Y1, Y1, zp, xplane, yplane, d0, s_lo, s_hi, SB, kb0, kb1);
        band_pass<W, PF, false, 2, 2>(acc, X2, Y2, Y2, zp, xplane, yplane, d0, s_lo, s_hi, SB, kb0, kb1);
      } else {  // Re += ReA ReB + ImA (-ImB),  Im += ReA ImB + ImA ReB
        band_pass<W, PF, true, 0, 1>(acc, X0, Y0, Y1, zp, xplane, yplane, d0, s_lo, s_hi, SB, kb0, kb1);
        band_pass<W, PF, true, 0, 1>(acc, X1, Y2, Y0, zp, xplane, yplane, d0, s_lo, s_hi, SB, kb0, kb1);
      }
    }
    // the band is complete: emit its diagonals least significant first
#pragma unroll
    for (int j = W - 1; j >= 0; --j) {
      const int d = d0 + j;
      if (d >= 0) {
        uint64_t packed = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int64_t vre, vim;
          if constexpr (M3) {
            const int64_t t1 = acc[0][j][r], t2 = acc[1][j][r], t3 = acc[2][j][r];
            vre = t1 - t2;
            vim = t3 - t1 - t2;
          } else {
            vre = acc[0][j][r];
            vim = acc[1][j][r];
          }
          cre[r] += vre;
          cim[r] += vim;
          const uint64_t dre = (uint64_t)(cre[r] & 127), dim = (uint64_t)(cim[r] & 127);
          cre[r] >>= 7;
          cim[r] >>= 7;
          if (dre && lre[r] < 0) lre[r] = d;
          if (dim && lim[r] < 0) lim[r] = d;
          packed |= dre << (8 * r);
          packed |= dim << (8 * (4 + r));
        }
        dig[(size_t)d * 64] = packed;
      }
    }
  }

  const size_t ob = ((size_t)(split * a.mt * a.nt + tile) * 64 + lane) * 8;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    a.top[ob + r] = cre[r];
    a.top[ob + 4 + r] = cim[r];
    a.lnz[ob + r] = lre[r];
    a.lnz[ob + 4 + r] = lim[r];
  }
}

template <int W>
hipError_t launch_w(const GemmArgs& a, hipStream_t stream) {
  const int blocks = (a.mt / 2) * (a.nt / 2) * a.ksplit;
  if (a.mode3m)
    gemm_i8_kernel<W, true><<<dim3(blocks), dim3(256), 0, stream>>>(a);
  else
    gemm_i8_kernel<W, false><<<dim3(blocks), dim3(256), 0, stream>>>(a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_i8(const GemmArgs& a, int band, hipStream_t stream) {
  switch (band) {
    case 8: return launch_w<8>(a, stream);
    case 12: return launch_w<12>(a, stream);
    case 16: return launch_w<16>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mpcg
