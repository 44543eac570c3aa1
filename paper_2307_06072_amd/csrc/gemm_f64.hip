// The plain form of the Ozaki scheme with floating-point slices, as in
// Algorithm 2: binary64 GEMMs of slices short enough that each product is
// error-free, then their exact accumulation.
//
// Digits are balanced base-2^w integers held in doubles with
// w = floor((53 - ceil(log2 k)) / 2) (the slice width rule of Algorithm 2),
// so every entry of a slice-plane product X_s Y_t^T is an integer below 2^53
// whatever order the GEMM sums in: the products are plain DGEMMs (rocBLAS, on
// the FP64 matrix cores), of the stacked slice planes of one block of s
// against all t at once.  The kernels here turn them into digits:
//   f64_accumulate_kernel  adds each product entry, as an exact int64, into
//                          its anti-diagonal d = s + t, combined into Re and
//                          Im (eq. 5 or eq. 6);
//   f64_carry_kernel       pushes the diagonals through a base-2^w carry chain
//                          into the digit streams the rounding kernel reads
//                          (element (i, j) of a 16 x 16 tile in lane
//                          j + 16 (i % 4), slot 4 comp + i / 4).
#include "mpcg_internal.h"

namespace mpcg {

namespace {

__device__ inline int64_t at(const double* C, int64_t row, int64_t col, int64_t ldc) {
  return (int64_t)C[col * ldc + row];  // an exact integer below 2^53
}

// One thread per entry (i, j): the diagonals d that the block s0 .. s1 - 1
// (against t = 0 .. tcnt - 1) reaches.
__global__ __launch_bounds__(256) void f64_accumulate_kernel(F64AccArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)a.m * a.n) return;
  const int i = (int)(gid % a.m), j = (int)(gid / a.m);
  const int dlast = min(a.s1 - 1 + a.tcnt - 1, a.Dmax);
  const int64_t mn = (int64_t)a.m * a.n;
  for (int d = a.s0; d <= dlast; ++d) {
    const int slo = max(a.s0, d - (a.tcnt - 1)), shi = min(a.s1 - 1, d);
    int64_t re = 0, im = 0;
    for (int s = slo; s <= shi; ++s) {
      const int t = d - s;
      const int64_t row = (int64_t)(s - a.s0) * a.mpad + i, col = (int64_t)t * a.npad + j;
      if (a.mode3m) {
        const int64_t t1 = at(a.C[0], row, col, a.ldc), t2 = at(a.C[1], row, col, a.ldc),
                      t3 = at(a.C[2], row, col, a.ldc);
        re += t1 - t2;
        im += t3 - t1 - t2;
      } else {
        re += at(a.C[0], row, col, a.ldc) - at(a.C[1], row, col, a.ldc);
        im += at(a.C[2], row, col, a.ldc) + at(a.C[3], row, col, a.ldc);
      }
    }
    a.acc[(int64_t)d * mn + gid] += re;
    a.acc[(int64_t)(a.Dmax + 1 + d) * mn + gid] += im;
  }
}

// One thread per (tile, lane, slot) of the rounding kernel's order, so the
// digit stores of a wavefront are contiguous.
__global__ __launch_bounds__(256) void f64_carry_kernel(F64CarryArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int tiles = a.mt * a.nt;
  if (gid >= (int64_t)tiles * 512) return;
  const int tile = (int)(gid >> 9), lane = (int)(gid >> 3) & 63, slot = (int)gid & 7;
  const int comp = slot >> 2;
  const int ii = (lane >> 4) + 4 * (slot & 3), jj = lane & 15;
  const int i = (tile % a.mt) * 16 + ii, j = (tile / a.mt) * 16 + jj;
  if (i >= a.m || j >= a.n) return;
  const int64_t mn = (int64_t)a.m * a.n, e = (int64_t)j * a.m + i;
  const int64_t* acc = a.acc + (int64_t)comp * (a.Dmax + 1) * mn;
  const int64_t dmask = (1ll << a.w) - 1;
  const int nd = a.Dmax + 1;
  int64_t c = 0;
  int lnz = -1;
  for (int d = a.Dmax; d >= 0; --d) {  // least significant first
    c += acc[(int64_t)d * mn + e];
    const uint32_t dg = (uint32_t)(c & dmask);
    c >>= a.w;
    a.digits[(((size_t)tile * nd + d) * 64 + lane) * 8 + slot] = dg;
    if (dg && lnz < 0) lnz = d;
  }
  a.top[gid] = c;
  a.lnz[gid] = lnz;
}

}  // namespace

hipError_t launch_f64_accumulate(const F64AccArgs& a, hipStream_t stream) {
  const int64_t total = (int64_t)a.m * a.n;
  f64_accumulate_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_f64_carry(const F64CarryArgs& a, hipStream_t stream) {
  const int64_t total = (int64_t)a.mt * a.nt * 512;
  f64_carry_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream>>>(a);
  return hipGetLastError();
}

}  // namespace mpcg
