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

__device__ inline void stats_init_body(RowStat* stats, int R, ScanSummary* summary, int blk) {
  const int r = blk * 256 + (int)threadIdx.x;
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

__global__ __launch_bounds__(256) void stats_init_kernel(RowStat* stats, int R, ScanSummary* summary) {
  stats_init_body(stats, R, summary, blockIdx.x);
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

// Rows contiguous (A): 64 rows x 4 contraction lanes per block, by splits K.
__device__ inline void scan_rows_body(const DOperand& op, RowStat* stats, int kchunk, ScanSummary* summary,
                                      int bx, int by) {
  __shared__ Acc part[4][64];
  const int rl = threadIdx.x & 63, kl = threadIdx.x >> 6;
  const int r = bx * 64 + rl;
  const int k0 = by * kchunk;
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

__global__ __launch_bounds__(256) void scan_rows_kernel(DOperand op, RowStat* stats, int kchunk,
                                                        ScanSummary* summary) {
  scan_rows_body(op, stats, kchunk, summary, blockIdx.x, blockIdx.y);
}

// Contraction contiguous (B): one wavefront per row, lanes along K, by splits K.
__device__ inline void scan_cols_body(const DOperand& op, RowStat* stats, int kchunk, ScanSummary* summary,
                                      int bx, int by) {
  const int lane = threadIdx.x & 63;
  const int r = bx * 4 + (threadIdx.x >> 6);
  if (r >= op.R) return;
  const int k0 = by * kchunk;
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

__global__ __launch_bounds__(256) void scan_cols_kernel(DOperand op, RowStat* stats, int kchunk,
                                                        ScanSummary* summary) {
  scan_cols_body(op, stats, kchunk, summary, blockIdx.x, blockIdx.y);
}

// Operand-wide maxima of the spreads and the number of nonzero rows.
__device__ inline void summary_body(const RowStat* stats, int R, ScanSummary* summary, int limit = 0,
                                    int* status_word = nullptr) {
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
    if (status_word) {
      int bits = summary->status;
      if (s_sp[0] > limit || s_hat[0] > limit) bits |= ST_SPREAD;
      if (bits) atomicOr(status_word, bits);
    }
  }
}

__global__ __launch_bounds__(256) void summary_kernel(const RowStat* stats, int R, ScanSummary* summary,
                                                      int limit, int* status_word) {
  summary_body(stats, R, summary, limit, status_word);
}

// A small operand (at most 512 rows of at most 256, 2^16 entries) in one launch:
// one workgroup scans 64 rows at a time with 16 lanes per row, then reduces
// the summary (what stats_init, the scan and the summary kernels do in three
// launches).
constexpr int64_t SCAN_SMALL_ENTRIES = 1 << 16;

__device__ __attribute__((always_inline)) inline void scan_small_body(const DOperand& op, RowStat* stats,
                                                                      ScanSummary* summary, int limit,
                                                                      int* status_word) {
  // 64 rows at a time, 16 contraction lanes per row
  __shared__ Acc part[16][64];
  __shared__ int32_t s_sp[1024], s_hat[1024], s_nz[1024], s_bad[1024];
  const int rl = threadIdx.x & 63, kl = threadIdx.x >> 6;
  int32_t sp = 0, hat = 0, nz = 0, bad = 0;
  for (int r0 = 0; r0 < op.R; r0 += 64) {
    const int r = r0 + rl;
    Acc a{INT32_MIN, INT32_MAX, INT32_MAX, 0};
    if (r < op.R)
      for (int kk = kl; kk < op.K; kk += 16) {
        const int64_t idx = (int64_t)r * op.rs + (int64_t)kk * op.ks;
        consume(a, op.re.exp[idx], op.im.exp[idx]);
      }
    part[kl][rl] = a;
    __syncthreads();
    if (kl == 0 && r < op.R) {
      for (int q = 1; q < 16; ++q) {
        a.emax = max(a.emax, part[q][rl].emax);
        a.emin = min(a.emin, part[q][rl].emin);
        a.ehat = min(a.ehat, part[q][rl].ehat);
        a.bad |= part[q][rl].bad;
      }
      RowStat st;
      st.emax = a.emax;
      st.emin = a.emax == INT32_MIN ? INT32_MAX : a.emin;
      st.ehat = a.emax == INT32_MIN ? INT32_MAX : a.ehat;
      st.pad = 0;
      stats[r] = st;
      if (a.emax != INT32_MIN) {
        sp = max(sp, a.emax - a.emin);
        hat = max(hat, a.emax - a.ehat);
        nz += 1;
      }
      bad |= a.bad;
    }
    __syncthreads();
  }
  s_sp[threadIdx.x] = sp;
  s_hat[threadIdx.x] = hat;
  s_nz[threadIdx.x] = nz;
  s_bad[threadIdx.x] = bad;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_sp[threadIdx.x] = max(s_sp[threadIdx.x], s_sp[threadIdx.x + off]);
      s_hat[threadIdx.x] = max(s_hat[threadIdx.x], s_hat[threadIdx.x + off]);
      s_nz[threadIdx.x] += s_nz[threadIdx.x + off];
      s_bad[threadIdx.x] |= s_bad[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ScanSummary z;
    z.spread = s_sp[0];
    z.hat = s_hat[0];
    z.nonzero = s_nz[0];
    z.status = s_bad[0] ? ST_IN_RANGE : 0;
    *summary = z;
    if (status_word) {
      int bits = z.status;
      if (z.spread > limit || z.hat > limit) bits |= ST_SPREAD;
      if (bits) atomicOr(status_word, bits);
    }
  }
}

__global__ __launch_bounds__(1024) void scan_small_kernel(DOperand op, RowStat* stats, ScanSummary* summary,
                                                          int limit, int* status_word) {
  scan_small_body(op, stats, summary, limit, status_word);
}

// Both operands of a product in one launch: block 0 scans A, block 1 B.
__global__ __launch_bounds__(1024) void scan_small_pair_kernel(DOperand a, RowStat* sa, DOperand b, RowStat* sb,
                                                               ScanSummary* summary, int limit, int* status_word) {
  if (blockIdx.x == 0)
    scan_small_body(a, sa, summary, limit, status_word);
  else
    scan_small_body(b, sb, summary + 1, limit, status_word);
}

__device__ inline void scales_body(const RowStat* stats, int R, int Rpad, int x, int32_t* G, int blk) {
  const int r = blk * 256 + (int)threadIdx.x;
  if (r >= Rpad) return;
  int32_t g = 0;
  if (r < R) {
    const int32_t e = stats[r].emax;
    g = (e == INT32_MIN) ? 0 : e + x;
  }
  G[r] = g;
}

__global__ __launch_bounds__(256) void scales_kernel(const RowStat* stats, int R, int Rpad, int x, int32_t* G) {
  scales_body(stats, R, Rpad, x, G, blockIdx.x);
}

// Scales of the folded rows of one level of Strassen's recursion: row r < half
// of every operand combination mixes rows r and r + half, whose exponents all
// lie below max(emax) (one bit more for a sum); 0 where both are zero.
__global__ __launch_bounds__(256) void fold_scales_kernel(const RowStat* stats, int half, int Rpad, int x,
                                                          int32_t* G) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= Rpad) return;
  int32_t g = 0;
  if (r < half) {
    const int32_t a = stats[r].emax, b = stats[r + half].emax;
    const int32_t e = a == INT32_MIN ? b : (b == INT32_MIN ? a : (a > b ? a : b));
    g = e == INT32_MIN ? 0 : e + x;
  }
  G[r] = g;
}

// ---- batched forms ----------------------------------------------------------
__global__ __launch_bounds__(256) void stats_init_batched(const ScanJob* __restrict__ jobs, int njobs,
                                                          const int* __restrict__ first) {
  const int j = job_of_block(first, njobs, blockIdx.x);
  const ScanJob& J = jobs[j];
  stats_init_body(J.stats, J.op.R, J.summary, blockIdx.x - first[j]);
}

template <bool ROWS>
__global__ __launch_bounds__(256) void scan_batched(const ScanJob* __restrict__ jobs, int njobs,
                                                    const int* __restrict__ first) {
  const int j = job_of_block(first, njobs, blockIdx.x);
  const ScanJob& J = jobs[j];
  const int local = blockIdx.x - first[j];
  const int bx = local % J.rblocks, by = local / J.rblocks;
  if (ROWS) scan_rows_body(J.op, J.stats, J.kchunk, J.summary, bx, by);
  else scan_cols_body(J.op, J.stats, J.kchunk, J.summary, bx, by);
}

__global__ __launch_bounds__(256) void summary_batched(const ScanJob* __restrict__ jobs, int limit,
                                                       int* status_word) {
  const ScanJob& J = jobs[blockIdx.x];
  summary_body(J.stats, J.op.R, J.summary, limit, status_word);
}

__global__ __launch_bounds__(256) void scales_batched(const ScaleJob* __restrict__ jobs, int njobs,
                                                      const int* __restrict__ first) {
  const int j = job_of_block(first, njobs, blockIdx.x);
  const ScaleJob& J = jobs[j];
  scales_body(J.stats, J.R, J.Rpad, J.x, J.G, blockIdx.x - first[j]);
}

}  // namespace

void scan_blocks(const DOperand& op, int* init_blocks, int* nblocks, int* kchunk, int* rblocks) {
  const int R = op.R, K = op.K;
  *init_blocks = (R + 255) / 256 + 1;
  *nblocks = 0;
  *kchunk = 1;
  *rblocks = 1;
  if (R <= 0 || K <= 0) return;
  int rb, ksplit;
  if (op.rs == 1) {
    rb = (R + 63) / 64;
    ksplit = max(1, min((K + 255) / 256, 2048 / rb + 1));
  } else {
    rb = (R + 3) / 4;
    ksplit = max(1, min((K + 1023) / 1024, 2048 / rb + 1));
  }
  const int kc = (K + ksplit - 1) / ksplit;
  ksplit = (K + kc - 1) / kc;
  *kchunk = kc;
  *rblocks = rb;
  *nblocks = rb * ksplit;
}

hipError_t launch_scan(const DOperand& op, RowStat* stats, ScanSummary* summary, int limit, int* status_word,
                       hipStream_t stream) {
  if ((int64_t)op.R * op.K <= SCAN_SMALL_ENTRIES && op.K <= 256 && op.R <= 512) {
    scan_small_kernel<<<dim3(1), dim3(1024), 0, stream>>>(op, stats, summary, limit, status_word);
    return hipGetLastError();
  }
  int ib, nb, kchunk, rblocks;
  scan_blocks(op, &ib, &nb, &kchunk, &rblocks);
  stats_init_kernel<<<dim3(ib), dim3(256), 0, stream>>>(stats, op.R, summary);
  if (nb > 0) {
    const int ksplit = nb / rblocks;
    if (op.rs == 1)
      scan_rows_kernel<<<dim3(rblocks, ksplit), dim3(256), 0, stream>>>(op, stats, kchunk, summary);
    else
      scan_cols_kernel<<<dim3(rblocks, ksplit), dim3(256), 0, stream>>>(op, stats, kchunk, summary);
  }
  summary_kernel<<<dim3(1), dim3(256), 0, stream>>>(stats, op.R, summary, limit, status_word);
  return hipGetLastError();
}

hipError_t launch_scan_pair(const DOperand& a, RowStat* sa, const DOperand& b, RowStat* sb, ScanSummary* summary,
                            int limit, int* status_word, hipStream_t stream) {
  auto small = [](const DOperand& op) {
    return (int64_t)op.R * op.K <= SCAN_SMALL_ENTRIES && op.K <= 256 && op.R <= 512;
  };
  if (small(a) && small(b)) {
    scan_small_pair_kernel<<<dim3(2), dim3(1024), 0, stream>>>(a, sa, b, sb, summary, limit, status_word);
    return hipGetLastError();
  }
  hipError_t e = launch_scan(a, sa, summary, limit, status_word, stream);
  if (e != hipSuccess) return e;
  return launch_scan(b, sb, summary + 1, limit, status_word, stream);
}

hipError_t launch_scales(const RowStat* stats, int R, int Rpad, int x, int32_t* G, hipStream_t stream) {
  scales_kernel<<<dim3((Rpad + 255) / 256), dim3(256), 0, stream>>>(stats, R, Rpad, x, G);
  return hipGetLastError();
}

hipError_t launch_scan_batched(const ScanJob* jobs, int njobs, const int* first_init, int init_blocks,
                               const int* first_scan, int scan_blocks_total, bool rows_contiguous, int limit,
                               int* status_word, hipStream_t stream) {
  if (njobs <= 0) return hipSuccess;
  stats_init_batched<<<dim3(init_blocks), dim3(256), 0, stream>>>(jobs, njobs, first_init);
  if (scan_blocks_total > 0) {
    if (rows_contiguous)
      scan_batched<true><<<dim3(scan_blocks_total), dim3(256), 0, stream>>>(jobs, njobs, first_scan);
    else
      scan_batched<false><<<dim3(scan_blocks_total), dim3(256), 0, stream>>>(jobs, njobs, first_scan);
  }
  summary_batched<<<dim3(njobs), dim3(256), 0, stream>>>(jobs, limit, status_word);
  return hipGetLastError();
}

hipError_t launch_fold_scales(const RowStat* stats, int half, int Rpad, int x, int32_t* G, hipStream_t stream) {
  fold_scales_kernel<<<dim3((Rpad + 255) / 256), dim3(256), 0, stream>>>(stats, half, Rpad, x, G);
  return hipGetLastError();
}

hipError_t launch_scales_batched(const ScaleJob* jobs, int njobs, const int* first, int blocks, hipStream_t stream) {
  if (njobs <= 0 || blocks <= 0) return hipSuccess;
  scales_batched<<<dim3(blocks), dim3(256), 0, stream>>>(jobs, njobs, first);
  return hipGetLastError();
}

}  // namespace mpcg
