// Slice-pair products on the FP64 matrix cores: the plain form of the Ozaki
// scheme with floating-point slices, as in Algorithm 2 (binary64 GEMMs of
// slices short enough that each product is error-free).
//
// Digits are balanced base-2^w integers held in doubles with
// w = floor((53 - ceil(log2 k)) / 2) (the slice width rule of Algorithm 2),
// so every slice-pair GEMM, accumulated in fp64 over the whole contraction
// chunk, is exact.  Each pair's fp64 tile is converted to int64 (exact) and
// added into the int64 diagonal window; completed diagonals are combined into
// Re/Im (eq. 5 or eq. 6) and pushed through a base-2^w carry chain exactly
// like the INT8 kernel.  A wavefront owns a 16 x 16 output tile and walks the
// pair square in 2 x 2 blocks.  The fp64 16x16x4 instruction returns element
// (i, j) of the tile in lane j + 16*(i%4), register i/4; the digit streams
// keep that order and the rounding kernel reads them accordingly.
#include "mpcg_internal.h"

namespace mpcg {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int NBF = 2;

template <bool M3>
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmF64Args a) {
  constexpr int NACC = M3 ? 3 : 2;
  constexpr int W = 2 * NBF - 1;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;

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

  const size_t xplane = (size_t)a.mt * a.kblocks * 64;  // doubles per (op, s) plane
  const size_t yplane = (size_t)a.nt * a.kblocks * 64;
  const double* Xb = a.X + (size_t)ti * a.kblocks * 64 + lane;
  const double* Yb = a.Y + (size_t)tj * a.kblocks * 64 + lane;

  // int64 diagonal window: [acc][slot][element]
  int64_t win[NACC][W][4];
#pragma unroll
  for (int p = 0; p < NACC; ++p)
#pragma unroll
    for (int q = 0; q < W; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) win[p][q][r] = 0;

  int64_t cre[4], cim[4];
  int32_t lre[4], lim[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    cre[r] = cim[r] = 0;
    lre[r] = lim[r] = -1;
  }
  const int w = a.w;
  const int64_t dmask = (1ll << w) - 1;

  const int SAp = (a.SA + NBF - 1) / NBF * NBF, SBp = (a.SB + NBF - 1) / NBF * NBF;
  const int nSB = SAp / NBF, nTB = SBp / NBF;
  const int Btop = min(nSB - 1 + nTB - 1, a.Dmax / NBF);
  const int nd = a.Dmax + 1;
  uint32_t* dig = a.digits + ((size_t)(split * a.mt * a.nt + tile) * nd) * 64 * 8 + lane * 8;

  for (int Bd = Btop; Bd >= -1; --Bd) {
    if (Bd >= 0) {
      const int sb_lo = max(0, Bd - (nTB - 1)), sb_hi = min(Bd, nSB - 1);
      for (int sb = sb_lo; sb <= sb_hi; ++sb) {
        const int tb = Bd - sb;
        v4d acc[NBF][NBF][NACC];
#pragma unroll
        for (int i = 0; i < NBF; ++i)
#pragma unroll
          for (int j = 0; j < NBF; ++j)
#pragma unroll
            for (int p = 0; p < NACC; ++p) acc[i][j][p] = v4d{0.0, 0.0, 0.0, 0.0};
        const double* xs = Xb + (size_t)(NBF * sb) * xplane;
        const double* yt = Yb + (size_t)(NBF * tb) * yplane;
        for (int kb = kb0; kb < kb1; ++kb) {
          const size_t ko = (size_t)kb * 64;
          if constexpr (M3) {
#pragma unroll
            for (int p = 0; p < 3; ++p) {
              double xa[NBF], yb[NBF];
#pragma unroll
              for (int i = 0; i < NBF; ++i) xa[i] = xs[((size_t)p * SAp + i) * xplane + ko];
#pragma unroll
              for (int j = 0; j < NBF; ++j) yb[j] = yt[((size_t)p * SBp + j) * yplane + ko];
#pragma unroll
              for (int i = 0; i < NBF; ++i)
#pragma unroll
                for (int j = 0; j < NBF; ++j) acc[i][j][p] = mfma(xa[i], yb[j], acc[i][j][p]);
            }
          } else {
            double xr[NBF], xi[NBF], yr[NBF], yi[NBF], yn[NBF];
#pragma unroll
            for (int i = 0; i < NBF; ++i) {
              xr[i] = xs[((size_t)0 * SAp + i) * xplane + ko];
              xi[i] = xs[((size_t)1 * SAp + i) * xplane + ko];
            }
#pragma unroll
            for (int j = 0; j < NBF; ++j) {
              yr[j] = yt[((size_t)0 * SBp + j) * yplane + ko];
              yi[j] = yt[((size_t)1 * SBp + j) * yplane + ko];
              yn[j] = yt[((size_t)2 * SBp + j) * yplane + ko];
            }
#pragma unroll
            for (int i = 0; i < NBF; ++i)
#pragma unroll
              for (int j = 0; j < NBF; ++j) {
                acc[i][j][0] = mfma(xr[i], yr[j], acc[i][j][0]);
                acc[i][j][1] = mfma(xr[i], yi[j], acc[i][j][1]);
                acc[i][j][0] = mfma(xi[i], yn[j], acc[i][j][0]);
                acc[i][j][1] = mfma(xi[i], yr[j], acc[i][j][1]);
              }
          }
        }
        // each pair's tile is an exact integer below 2^53: move it to int64
#pragma unroll
        for (int i = 0; i < NBF; ++i)
#pragma unroll
          for (int j = 0; j < NBF; ++j)
#pragma unroll
            for (int p = 0; p < NACC; ++p)
#pragma unroll
              for (int r = 0; r < 4; ++r) win[p][i + j][r] += (int64_t)acc[i][j][p][r];
      }
    }
#pragma unroll
    for (int slot = W - 1; slot >= NBF - 1; --slot) {
      const int d = NBF * Bd + slot;
      if (d >= 0 && d <= a.Dmax) {
        uint32_t out[8];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int64_t vre, vim;
          if constexpr (M3) {
            const int64_t t1 = win[0][slot][r], t2 = win[1][slot][r], t3 = win[2][slot][r];
            vre = t1 - t2;
            vim = t3 - t1 - t2;
          } else {
            vre = win[0][slot][r];
            vim = win[1][slot][r];
          }
          cre[r] += vre;
          cim[r] += vim;
          const uint32_t dre = (uint32_t)(cre[r] & dmask), dim = (uint32_t)(cim[r] & dmask);
          cre[r] >>= w;
          cim[r] >>= w;
          if (dre && lre[r] < 0) lre[r] = d;
          if (dim && lim[r] < 0) lim[r] = d;
          out[r] = dre;
          out[4 + r] = dim;
        }
        uint4* dst = reinterpret_cast<uint4*>(dig + (size_t)d * 64 * 8);
        dst[0] = uint4{out[0], out[1], out[2], out[3]};
        dst[1] = uint4{out[4], out[5], out[6], out[7]};
      }
    }
#pragma unroll
    for (int p = 0; p < NACC; ++p) {
#pragma unroll
      for (int q = W - 1; q >= NBF; --q)
#pragma unroll
        for (int r = 0; r < 4; ++r) win[p][q][r] = win[p][q - NBF][r];
#pragma unroll
      for (int q = 0; q < NBF; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) win[p][q][r] = 0;
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

}  // namespace

hipError_t launch_gemm_f64(const GemmF64Args& a, hipStream_t stream) {
  const int blocks = (a.mt / 2) * (a.nt / 2) * a.ksplit;
  if (a.mode3m)
    gemm_f64_kernel<true><<<dim3(blocks), dim3(256), 0, stream>>>(a);
  else
    gemm_f64_kernel<false><<<dim3(blocks), dim3(256), 0, stream>>>(a);
  return hipGetLastError();
}

}  // namespace mpcg
