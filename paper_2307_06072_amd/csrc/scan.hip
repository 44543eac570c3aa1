// Exponent scan: per row of A (per column of B) the largest and smallest
// exponent of its nonzero real/imaginary components, and the smallest
// "entry exponent" max(e_re, e_im).  This is the exact, integer counterpart of
// the row/column maxima mu_A, mu_B of Algorithm 2: the largest exponent fixes
// the power-of-two row scale (tau_A), the spread fixes how many slices an
// error-free split needs.  Real and imaginary parts share one scale per row
// (the common number of divisions of Section III-C).
#include "mpcg_internal.h"

namespace mpcg {

namespace {

__global__ void stats_init_kernel(RowStat* stats, int R, ScanSummary* summary) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < R) {
    RowStat s;
    s.emax = INT32_MIN;
    s.emin = INT32_MAX;
    s.ehat = INT32_MAX;
    s.pad = 0;
    stats[r] = s;
  }
  if (r == 0) {
    ScanSummary z;
    z.spread = 0;
    z.hat = 0;
    z.nonzero = 0;
    z.status = 0;
    *summary = z;
  }
}

struct Acc {
  int32_t emax, emin, ehat;
  int bad;
};

__device__ inline void consume(Acc& a, int32_t er, int32_t ei) {
  const bool zr = er == EXP_ZERO, zi = ei == EXP_ZERO;
  if (!zr) {
    a.emax = max(a.emax, er);
    a.emin = min(a.emin, er);
    a.bad |= (er > EXP_LIMIT || er < -EXP_LIMIT);
  }
  if (!zi) {
    a.emax = max(a.emax, ei);
    a.emin = min(a.emin, ei);
    a.bad |= (ei > EXP_LIMIT || ei < -EXP_LIMIT);
  }
  if (!(zr && zi)) {
    const int32_t top = zr ? ei : (zi ? er : max(er, ei));
    a.ehat = min(a.ehat, top);
  }
}

// Rows contiguous (A): 64 rows x 4 contraction lanes per block, grid.y splits K.
__global__ __launch_bounds__(256) void scan_rows_kernel(DOperand op, RowStat* stats, int kchunk,
                                                        ScanSummary* summary) {
  __shared__ Acc part[4][64];
  const int rl = threadIdx.x & 63, kl = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + rl;
  const int k0 = blockIdx.y * kchunk;
  const int k1 = min(op.K, k0 + kchunk);
  Acc a{INT32_MIN, INT32_MAX, INT32_MAX, 0};
  if (r < op.R) {
    for (int kk = k0 + kl; kk < k1; kk += 4) {
      const int64_t idx = (int64_t)r * op.rs + (int64_t)kk * op.ks;
      consume(a, op.re.exp[idx], op.im.exp[idx]);
    }
  }
  part[kl][rl] = a;
  __syncthreads();
  if (kl == 0 && r < op.R) {
    for (int q = 1; q < 4; ++q) {
      a.emax = max(a.emax, part[q][rl].emax);
      a.emin = min(a.emin, part[q][rl].emin);
      a.ehat = min(a.ehat, part[q][rl].ehat);
      a.bad |= part[q][rl].bad;
    }
    if (a.emax != INT32_MIN) {
      atomicMax(&stats[r].emax, a.emax);
      atomicMin(&stats[r].emin, a.emin);
      atomicMin(&stats[r].ehat, a.ehat);
    }
    if (a.bad) atomicOr(&summary->status, ST_IN_RANGE);
  }
}

// Contraction contiguous (B): one wavefront per row, lanes along K, grid.y splits K.
__global__ __launch_bounds__(256) void scan_cols_kernel(DOperand op, RowStat* stats, int kchunk,
                                                        ScanSummary* summary) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= op.R) return;
  const int k0 = blockIdx.y * kchunk;
  const int k1 = min(op.K, k0 + kchunk);
  Acc a{INT32_MIN, INT32_MAX, INT32_MAX, 0};
  for (int kk = k0 + lane; kk < k1; kk += 64) {
    const int64_t idx = (int64_t)r * op.rs + (int64_t)kk * op.ks;
    consume(a, op.re.exp[idx], op.im.exp[idx]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    a.emax = max(a.emax, __shfl_xor(a.emax, off));
    a.emin = min(a.emin, __shfl_xor(a.emin, off));
    a.ehat = min(a.ehat, __shfl_xor(a.ehat, off));
    a.bad |= __shfl_xor(a.bad, off);
  }
  if (lane == 0) {
    if (a.emax != INT32_MIN) {
      atomicMax(&stats[r].emax, a.emax);
      atomicMin(&stats[r].emin, a.emin);
      atomicMin(&stats[r].ehat, a.ehat);
    }
    if (a.bad) atomicOr(&summary->status, ST_IN_RANGE);
  }
}

// Operand-wide maxima of the spreads and the number of nonzero rows.
__global__ __launch_bounds__(256) void summary_kernel(const RowStat* stats, int R, ScanSummary* summary) {
  __shared__ int32_t s_sp[256], s_hat[256], s_nz[256];
  int32_t sp = 0, hat = 0, nz = 0;
  for (int r = threadIdx.x; r < R; r += 256) {
    const RowStat s = stats[r];
    if (s.emax != INT32_MIN) {
      sp = max(sp, s.emax - s.emin);
      hat = max(hat, s.emax - s.ehat);
      nz += 1;
    }
  }
  s_sp[threadIdx.x] = sp;
  s_hat[threadIdx.x] = hat;
  s_nz[threadIdx.x] = nz;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s_sp[threadIdx.x] = max(s_sp[threadIdx.x], s_sp[threadIdx.x + off]);
      s_hat[threadIdx.x] = max(s_hat[threadIdx.x], s_hat[threadIdx.x + off]);
      s_nz[threadIdx.x] += s_nz[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    summary->spread = s_sp[0];
    summary->hat = s_hat[0];
    summary->nonzero = s_nz[0];
  }
}

__global__ void scales_kernel(const RowStat* stats, int R, int Rpad, int x, int32_t* G) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= Rpad) return;
  int32_t g = 0;
  if (r < R) {
    const int32_t e = stats[r].emax;
    g = (e == INT32_MIN) ? 0 : e + x;
  }
  G[r] = g;
}

}  // namespace

hipError_t launch_scan(const DOperand& op, RowStat* stats, ScanSummary* summary, hipStream_t stream) {
  const int R = op.R, K = op.K;
  stats_init_kernel<<<dim3((R + 255) / 256 + 1), dim3(256), 0, stream>>>(stats, R, summary);
  if (R > 0 && K > 0) {
    if (op.rs == 1) {
      const int rblocks = (R + 63) / 64;
      int ksplit = max(1, min((K + 255) / 256, 2048 / rblocks + 1));
      const int kchunk = (K + ksplit - 1) / ksplit;
      ksplit = (K + kchunk - 1) / kchunk;
      scan_rows_kernel<<<dim3(rblocks, ksplit), dim3(256), 0, stream>>>(op, stats, kchunk, summary);
    } else {
      const int rblocks = (R + 3) / 4;
      int ksplit = max(1, min((K + 1023) / 1024, 2048 / rblocks + 1));
      const int kchunk = (K + ksplit - 1) / ksplit;
      ksplit = (K + kchunk - 1) / kchunk;
      scan_cols_kernel<<<dim3(rblocks, ksplit), dim3(256), 0, stream>>>(op, stats, kchunk, summary);
    }
  }
  summary_kernel<<<dim3(1), dim3(256), 0, stream>>>(stats, R, summary);
  return hipGetLastError();
}

hipError_t launch_scales(const RowStat* stats, int R, int Rpad, int x, int32_t* G, hipStream_t stream) {
  scales_kernel<<<dim3((Rpad + 255) / 256), dim3(256), 0, stream>>>(stats, R, Rpad, x, G);
  return hipGetLastError();
}

}  // namespace mpcg
