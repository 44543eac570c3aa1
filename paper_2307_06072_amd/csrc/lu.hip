// Scalar and row kernels of the blocked complex LU factorization (Sec. IV-B):
// block copies (plain, conjugate, absolute value), the pivot search over a
// column of keys, row interchanges and small constants.  The products and
// updates of the factorization run through the product kernels and the pivot
// reciprocals through recip.hip; the kernels here only move and compare
// numbers.
#include "mpcg_internal.h"

namespace mpcg {
namespace {

constexpr int LU_THREADS = 256;

// dst(i) := src(i) for one entry of one real component; flip the sign
// (nonzero entries only) when `neg`, clear it when `absval`.
__device__ inline void copy_entry(DPart s, int64_t si, DOutPart d, int64_t di, int L, bool neg, bool absval) {
  const int32_t e = s.exp[si];
  uint8_t sg = s.sign[si];
  if (e == EXP_ZERO || absval) sg = 0;
  else if (neg) sg ^= 1;
  d.sign[di] = sg;
  d.exp[di] = e;
  for (int l = 0; l < L; ++l) d.mant[l * d.ls + di] = (e == EXP_ZERO) ? 0 : s.mant[l * s.ls + si];
}

__device__ inline void swap_entry(DOutPart p, int64_t a, int64_t b, int L) {
  const uint8_t sa = p.sign[a];
  p.sign[a] = p.sign[b];
  p.sign[b] = sa;
  const int32_t ea = p.exp[a];
  p.exp[a] = p.exp[b];
  p.exp[b] = ea;
  for (int l = 0; l < L; ++l) {
    const uint64_t ma = p.mant[l * p.ls + a];
    p.mant[l * p.ls + a] = p.mant[l * p.ls + b];
    p.mant[l * p.ls + b] = ma;
  }
}

// Value +-1 or 0 into entry 0 of one component.
__device__ inline void write_small(DOutPart p, int v, int L) {
  p.sign[0] = v < 0 ? 1 : 0;
  p.exp[0] = v == 0 ? EXP_ZERO : 1;  // 1 = 2^(64L-1) * 2^(1-64L)
  for (int l = 0; l < L; ++l) p.mant[l * p.ls] = (v != 0 && l == L - 1) ? (1ull << 63) : 0;
}

// mode 0: copy, 1: conjugate (negate Im), 2: componentwise absolute value.
__global__ void __launch_bounds__(LU_THREADS) copy_block_kernel(DPart sre, DPart sim, int64_t lds, DOutPart dre,
                                                                DOutPart dim, int64_t ldd, int rows, int cols,
                                                                int L, int mode) {
  const int64_t t = (int64_t)blockIdx.x * LU_THREADS + threadIdx.x;
  if (t >= (int64_t)rows * cols) return;
  const int64_t c = t / rows, r = t - c * rows;
  copy_entry(sre, c * lds + r, dre, c * ldd + r, L, false, mode == 2);
  copy_entry(sim, c * lds + r, dim, c * ldd + r, L, mode == 1, mode == 2);
}

// key(i) compared with key(j), keys nonnegative: -1, 0, +1.
__device__ inline int cmp_key(DPart k, int i, int j, int L) {
  const int32_t ei = k.exp[i], ej = k.exp[j];
  if (ei != ej) return ei > ej ? 1 : -1;  // EXP_ZERO (zero) is below every exponent
  if (ei == EXP_ZERO) return 0;
  for (int l = L - 1; l >= 0; --l) {
    const uint64_t a = k.mant[l * k.ls + i], b = k.mant[l * k.ls + j];
    if (a != b) return a > b ? 1 : -1;
  }
  return 0;
}

// The first index of the largest key among keys[0, m) (one block).  Writes
// base + index to *piv; if the largest key is zero and *info is still 0,
// *info := col + 1.
__global__ void __launch_bounds__(LU_THREADS) pivot_kernel(DPart key, int m, int L, int base, int* piv,
                                                           int* info, int col) {
  __shared__ int best[LU_THREADS];
  int b = -1;
  for (int i = threadIdx.x; i < m; i += LU_THREADS)
    if (b < 0 || cmp_key(key, i, b, L) > 0) b = i;  // ascending scan: ties keep the earlier index
  best[threadIdx.x] = b;
  __syncthreads();
  for (int s = LU_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const int a = best[threadIdx.x], c = best[threadIdx.x + s];
      if (c >= 0 && (a < 0 || cmp_key(key, c, a, L) > 0 || (cmp_key(key, c, a, L) == 0 && c < a)))
        best[threadIdx.x] = c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int i = best[0] < 0 ? 0 : best[0];
    piv[0] = base + i;
    if (key.exp[i] == EXP_ZERO && info[0] == 0) info[0] = col + 1;
  }
}

// Rows `row` and *piv exchanged over columns [0, ncols) of both components.
__global__ void __launch_bounds__(LU_THREADS) swap_rows_kernel(DOutPart re, DOutPart im, int64_t ld, int ncols,
                                                               int L, int row, const int* piv) {
  const int j = blockIdx.x * LU_THREADS + threadIdx.x;
  const int p = piv[0];
  if (j >= ncols || p == row) return;
  swap_entry(re, (int64_t)j * ld + row, (int64_t)j * ld + p, L);
  swap_entry(im, (int64_t)j * ld + row, (int64_t)j * ld + p, L);
}

// The interchanges ipiv[0], ..., ipiv[n-1], in that order, applied to the
// rows of an n x ncols block (one column per thread); an entry outside
// [0, n) is skipped rather than followed out of the block.
__global__ void __launch_bounds__(LU_THREADS) laswp_kernel(DOutPart re, DOutPart im, int64_t ld, int ncols, int n,
                                                           int L, const int* ipiv) {
  const int j = blockIdx.x * LU_THREADS + threadIdx.x;
  if (j >= ncols) return;
  for (int c = 0; c < n; ++c) {
    const int p = ipiv[c];
    if (p == c || p < 0 || p >= n) continue;
    swap_entry(re, (int64_t)j * ld + c, (int64_t)j * ld + p, L);
    swap_entry(im, (int64_t)j * ld + c, (int64_t)j * ld + p, L);
  }
}

__global__ void const_kernel(DOutPart re, DOutPart im, int L, int vre, int vim) {
  if (threadIdx.x == 0) {
    write_small(re, vre, L);
    write_small(im, vim, L);
  }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + LU_THREADS - 1) / LU_THREADS); }

}  // namespace

hipError_t launch_lu_copy(DPart sre, DPart sim, int64_t lds, DOutPart dre, DOutPart dim, int64_t ldd, int rows,
                          int cols, int L, int mode, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  copy_block_kernel<<<blocks_for((int64_t)rows * cols), LU_THREADS, 0, stream>>>(sre, sim, lds, dre, dim, ldd, rows,
                                                                                cols, L, mode);
  return hipGetLastError();
}

hipError_t launch_lu_pivot(DPart key, int m, int L, int base, int* piv, int* info, int col, hipStream_t stream) {
  pivot_kernel<<<1, LU_THREADS, 0, stream>>>(key, m, L, base, piv, info, col);
  return hipGetLastError();
}

hipError_t launch_lu_swap(DOutPart re, DOutPart im, int64_t ld, int ncols, int L, int row, const int* piv,
                          hipStream_t stream) {
  if (ncols <= 0) return hipSuccess;
  swap_rows_kernel<<<blocks_for(ncols), LU_THREADS, 0, stream>>>(re, im, ld, ncols, L, row, piv);
  return hipGetLastError();
}

hipError_t launch_lu_laswp(DOutPart re, DOutPart im, int64_t ld, int ncols, int n, int L, const int* ipiv,
                           hipStream_t stream) {
  if (ncols <= 0 || n <= 0) return hipSuccess;
  laswp_kernel<<<blocks_for(ncols), LU_THREADS, 0, stream>>>(re, im, ld, ncols, n, L, ipiv);
  return hipGetLastError();
}

hipError_t launch_lu_const(DOutPart re, DOutPart im, int L, int vre, int vim, hipStream_t stream) {
  const_kernel<<<1, 64, 0, stream>>>(re, im, L, vre, vim);
  return hipGetLastError();
}

}  // namespace mpcg
