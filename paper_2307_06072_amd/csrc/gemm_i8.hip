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
// A wavefront owns a 16 x 16 output tile and walks the (s, t) pair square in
// NB x NB blocks, block anti-diagonal by block anti-diagonal from the least
// significant end.  A block contributes to 2NB-1 consecutive diagonals, held
// in a window of int32 MFMA accumulators; after a block anti-diagonal the top
// NB diagonals of the window are complete.  They are combined into Re and Im
// (4M, eq. 5: two accumulators per diagonal; 3M, eq. 6: T1, T2, T3 with
// Re = T1 - T2, Im = T3 - T1 - T2) and pushed, least significant first, into
// a per-element int64 carry chain that emits one normalised base-2^7 digit per
// diagonal.  The final carry is the signed top part of the exact result.
// The NB x NB register block is what makes the kernel compute-bound: each
// pair of operand fragments loaded is reused NB times.
//
// Operand fragments (16 rows x 64 k, 16 bytes per lane) are read straight
// from the digit planes written by the split kernel.  The contraction can be
// cut into ksplit chunks; each chunk writes its own digit stream and the
// rounding kernel adds the streams exactly.
#include "mpcg_internal.h"

namespace mpcg {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ inline v4i mfma(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

template <int NB, bool M3>
__global__ __launch_bounds__(256) void gemm_i8_kernel(GemmArgs a) {
  constexpr int NACC = M3 ? 3 : 2;
  constexpr int W = 2 * NB - 1;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;

  // block -> (2x2 tile group, contraction chunk)
  const int gm = a.mt >> 1, gn = a.nt >> 1;
  const int groups = gm * gn;
  const int split = blockIdx.x / groups;
  const int gid = blockIdx.x - split * groups;
  const int ti = 2 * (gid % gm) + (wv & 1);
  const int tj = 2 * (gid / gm) + (wv >> 1);
  const int tile = tj * a.mt + ti;
  const int kbps = (a.kblocks + a.ksplit - 1) / a.ksplit;
  const int kb0 = split * kbps;
  const int kb1 = min(a.kblocks, kb0 + kbps);

  const size_t xplane = (size_t)a.mt * a.kblocks * 1024;  // bytes per (op, s) plane
  const size_t yplane = (size_t)a.nt * a.kblocks * 1024;
  const int8_t* Xb = a.X + (size_t)ti * a.kblocks * 1024 + lane * 16;
  const int8_t* Yb = a.Y + (size_t)tj * a.kblocks * 1024 + lane * 16;

  v4i acc[NACC][W];
#pragma unroll
  for (int p = 0; p < NACC; ++p)
#pragma unroll
    for (int q = 0; q < W; ++q) acc[p][q] = v4i{0, 0, 0, 0};

  int64_t cre[4], cim[4];
  int32_t lre[4], lim[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    cre[r] = cim[r] = 0;
    lre[r] = lim[r] = -1;
  }

  const int nSB = a.SAp / NB, nTB = a.SBp / NB;
  const int Btop = min(nSB - 1 + nTB - 1, a.Dmax / NB);
  const int nd = a.Dmax + 1;
  uint64_t* dig = reinterpret_cast<uint64_t*>(a.digits) + ((size_t)(split * a.mt * a.nt + tile) * nd) * 64 + lane;

  for (int Bd = Btop; Bd >= -1; --Bd) {
    if (Bd >= 0) {
      const int sb_lo = max(0, Bd - (nTB - 1)), sb_hi = min(Bd, nSB - 1);
      for (int sb = sb_lo; sb <= sb_hi; ++sb) {
        const int tb = Bd - sb;
        const int8_t* xs = Xb + (size_t)(NB * sb) * xplane;
        const int8_t* yt = Yb + (size_t)(NB * tb) * yplane;
        for (int kb = kb0; kb < kb1; ++kb) {
          const size_t ko = (size_t)kb * 1024;
          if constexpr (M3) {
#pragma unroll
            for (int p = 0; p < 3; ++p) {
              v4i xa[NB], yb[NB];
#pragma unroll
              for (int i = 0; i < NB; ++i)
                xa[i] = *reinterpret_cast<const v4i*>(xs + ((size_t)p * a.SAp + i) * xplane + ko);
#pragma unroll
              for (int j = 0; j < NB; ++j)
                yb[j] = *reinterpret_cast<const v4i*>(yt + ((size_t)p * a.SBp + j) * yplane + ko);
#pragma unroll
              for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[p][i + j] = mfma(xa[i], yb[j], acc[p][i + j]);
            }
          } else {
            v4i xr[NB], xi[NB], yr[NB], yi[NB], yn[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
              xr[i] = *reinterpret_cast<const v4i*>(xs + ((size_t)0 * a.SAp + i) * xplane + ko);
              xi[i] = *reinterpret_cast<const v4i*>(xs + ((size_t)1 * a.SAp + i) * xplane + ko);
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              yr[j] = *reinterpret_cast<const v4i*>(yt + ((size_t)0 * a.SBp + j) * yplane + ko);
              yi[j] = *reinterpret_cast<const v4i*>(yt + ((size_t)1 * a.SBp + j) * yplane + ko);
              yn[j] = *reinterpret_cast<const v4i*>(yt + ((size_t)2 * a.SBp + j) * yplane + ko);
            }
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
              for (int j = 0; j < NB; ++j) {
                acc[0][i + j] = mfma(xr[i], yr[j], acc[0][i + j]);
                acc[1][i + j] = mfma(xr[i], yi[j], acc[1][i + j]);
                acc[0][i + j] = mfma(xi[i], yn[j], acc[0][i + j]);
                acc[1][i + j] = mfma(xi[i], yr[j], acc[1][i + j]);
              }
          }
        }
      }
    }
    // the top NB slots of the window are complete: emit them least significant first
#pragma unroll
    for (int slot = W - 1; slot >= NB - 1; --slot) {
      const int d = NB * Bd + slot;
      if (d >= 0 && d <= a.Dmax) {
        uint64_t packed = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int64_t vre, vim;
          if constexpr (M3) {
            const int64_t t1 = acc[0][slot][r], t2 = acc[1][slot][r], t3 = acc[2][slot][r];
            vre = t1 - t2;
            vim = t3 - t1 - t2;
          } else {
            vre = acc[0][slot][r];
            vim = acc[1][slot][r];
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
    // slide the window down by NB diagonals
#pragma unroll
    for (int p = 0; p < NACC; ++p) {
#pragma unroll
      for (int q = W - 1; q >= NB; --q) acc[p][q] = acc[p][q - NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) acc[p][q] = v4i{0, 0, 0, 0};
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

template <int NB>
hipError_t launch_nb(const GemmArgs& a, hipStream_t stream) {
  const int blocks = (a.mt / 2) * (a.nt / 2) * a.ksplit;
  if (a.mode3m)
    gemm_i8_kernel<NB, true><<<dim3(blocks), dim3(256), 0, stream>>>(a);
  else
    gemm_i8_kernel<NB, false><<<dim3(blocks), dim3(256), 0, stream>>>(a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_i8(const GemmArgs& a, int block, hipStream_t stream) {
  switch (block) {
    case 4: return launch_nb<4>(a, stream);
    case 6: return launch_nb<6>(a, stream);
    case 8: return launch_nb<8>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mpcg
