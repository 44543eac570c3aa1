// Host side of libmpcgemm: argument validation, planning (slice counts,
// cutoff, padding, contraction chunks), workspace management and the launch
// sequence scan -> split -> slice GEMM -> round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <array>
#include <vector>

#include "../../include/mpcgemm.h"
#include "mpcg_internal.h"

using namespace mpcg;

namespace {

thread_local std::string g_err;
hipStream_t g_stream = nullptr;
std::mutex g_mu;

// caller-provided workspace
void* g_user_ws = nullptr;
size_t g_user_ws_bytes = 0;
// library-owned buffers
void* g_ws = nullptr;
size_t g_ws_bytes = 0;
void* g_scan = nullptr;  // row statistics + summaries
size_t g_scan_bytes = 0;
int* g_status = nullptr;  // persistent device status word
ScanSummary* g_host_summary = nullptr;  // pinned
int g_fault_inject = -1;  // test hook: MPCG_FAULT_INJECT=hip makes HIP calls fail

// per-call stage events: [call][boundary], boundaries = start, after scan,
// after split, after slice GEMM, after round
bool g_timing = false;
std::vector<std::array<hipEvent_t, 5>> g_ev;
int g_ncalls = 0;          // calls recorded since the last report
bool g_timing_valid = false;

int set_err(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

bool fault_injected() {
  if (g_fault_inject < 0) {
    const char* v = getenv("MPCG_FAULT_INJECT");
    g_fault_inject = (v && strcmp(v, "hip") == 0) ? 1 : 0;
  }
  return g_fault_inject == 1;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = fault_injected() ? hipErrorNotReady : (expr);                          \
    if (e_ != hipSuccess)                                                                  \
      return set_err(MPCG_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                     __FILE__, __LINE__);                                                  \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

int ceil_log2(long long v) {
  int r = 0;
  while ((1ll << r) < v) ++r;
  return r;
}

struct Region {
  uintptr_t lo, hi;
};

bool overlap(Region a, Region b) { return a.lo < b.hi && b.lo < a.hi; }

int check_part(const mpcg_part& p, int rows, int cols, int ld, int L, const char* name, Region out[3]) {
  if (!p.sign || !p.exp || !p.mant) return set_err(MPCG_EINVAL, "%s: NULL pointer", name);
  const int64_t n = (int64_t)ld * cols;
  const int64_t ls = p.limb_stride ? p.limb_stride : n;
  if (ls < n) return set_err(MPCG_EINVAL, "%s: limb_stride %lld < ld*cols %lld", name, (long long)ls, (long long)n);
  (void)rows;
  out[0] = {(uintptr_t)p.sign, (uintptr_t)p.sign + (uintptr_t)n};
  out[1] = {(uintptr_t)p.exp, (uintptr_t)p.exp + (uintptr_t)(4 * n)};
  out[2] = {(uintptr_t)p.mant, (uintptr_t)p.mant + (uintptr_t)(8 * (ls * (L - 1) + n))};
  return MPCG_OK;
}

DPart dpart(const mpcg_part& p, int64_t n) {
  return DPart{p.sign, p.exp, p.mant, p.limb_stride ? p.limb_stride : n};
}
DOutPart doutpart(const mpcg_part& p, int64_t n) {
  return DOutPart{p.sign, p.exp, p.mant, p.limb_stride ? p.limb_stride : n};
}

// Everything the launch sequence needs, derived from the shapes and the scan.
struct Plan {
  int m, n, k, p, L, mode3m, trunc, f64;
  int w, x;
  int SA, SB, SAp, SBp, Dmax, cutoff;
  int xs, ys, xlo, ylo;  // slices per plane with zero pads, lower pads
  int block;
  int mpad, npad, kpad, mt, nt, kblocks, ksplit;
  int nopsA, nopsB;
  long long pairs;
  double algo_ops, bound_bits;
  size_t off_G, off_H, off_X, off_Y, off_dig, off_top, off_lnz, total;
};

int plan_slices(Plan& P, int spreadA, int spreadB, int hatA, int hatB, const mpcg_options* opt) {
  P.L = (P.p + 63) / 64;
  P.x = P.mode3m ? 2 : 1;
  P.w = P.f64 ? std::max(1, (53 - ceil_log2(std::max(1, P.k))) / 2) : 7;
  if (P.w > 31) P.w = 31;
  P.SA = ceil_div(P.p + P.x + spreadA, P.w);
  P.SB = ceil_div(P.p + P.x + spreadB, P.w);
  const int Dexact = P.SA + P.SB - 2;
  P.bound_bits = 0.0;
  if (!P.trunc) {
    P.Dmax = Dexact;
  } else {
    int c;
    if (opt && opt->cutoff_override > 0) {
      c = opt->cutoff_override;
    } else {
      const int S = std::max(P.SA, P.SB);
      const int lg = ceil_log2(6ll * (S + 2));
      c = ceil_div(P.p - 3 + lg + hatA + hatB + 2 * P.x, P.w) - 1;
      P.bound_bits = P.p - 4;
    }
    P.Dmax = std::min(Dexact, std::max(0, c));
  }
  P.cutoff = P.Dmax;
  // kept pairs
  long long pairs = 0;
  for (int s = 0; s < P.SA; ++s) {
    const int tmax = std::min(P.SB - 1, P.Dmax - s);
    if (tmax >= 0) pairs += tmax + 1;
  }
  P.pairs = pairs;
  const int nprod = P.mode3m ? 3 : 4;
  P.algo_ops = 2.0 * P.m * (double)P.n * P.k * (double)pairs * nprod;
  return MPCG_OK;
}

int plan_layout(Plan& P, const mpcg_options* opt) {
  P.mpad = (int)round_up(P.m, 32);
  P.npad = (int)round_up(P.n, 32);
  P.kpad = (int)round_up(P.k, 64);
  P.mt = P.mpad / 16;
  P.nt = P.npad / 16;
  P.nopsA = P.mode3m ? 3 : 2;
  P.nopsB = 3;
  const int groups = (P.mpad / 32) * (P.npad / 32);
  if (!P.f64) {
    // band width: diagonals accumulated together by one wavefront
    P.block = (opt && opt->block_override) ? opt->block_override : 16;
    if (P.block != 8 && P.block != 12 && P.block != 16)
      return set_err(MPCG_EINVAL, "block_override (band width) must be 8, 12 or 16");
    P.SAp = P.SA;
    P.SBp = P.SB;
    int ahi, bhi;
    gemm_i8_pads(P.block, &P.xlo, &ahi, &P.ylo, &bhi);
    P.xs = P.xlo + P.SA + ahi;
    P.ys = P.ylo + P.SB + bhi;
    P.kblocks = P.kpad / 64;
    // int32 accumulators: terms per diagonal * 64*64 must stay below 2^31
    const long long terms_per_k = (long long)(P.mode3m ? 1 : 2) * std::min(P.SA, P.SB);
    const long long kc_max = ((1ll << 31) - 1) / (4096ll * terms_per_k);
    const long long kb_max = kc_max / 64;
    if (kb_max < 1) return set_err(MPCG_EUNSUPPORTED, "precision/spread too large for int32 slice accumulation");
    int ks = (int)((P.kblocks + kb_max - 1) / kb_max);
    int want = std::max(1, ceil_div(512, groups));
    ks = std::max(ks, std::min(want, P.kblocks));
    P.ksplit = ks;
  } else {
    P.block = 2;
    P.SAp = (int)round_up(P.SA, 2);
    P.SBp = (int)round_up(P.SB, 2);
    P.xs = P.SAp;
    P.ys = P.SBp;
    P.xlo = P.ylo = 0;
    P.kblocks = P.kpad / 4;
    int want = std::max(1, ceil_div(512, groups));
    P.ksplit = std::min(want, std::max(1, P.kpad / 64));
  }
  if (opt && opt->ksplit_override > 0) {
    if (!P.f64) {
      const long long terms_per_k = (long long)(P.mode3m ? 1 : 2) * std::min(P.SA, P.SB);
      const long long kc_max = ((1ll << 31) - 1) / (4096ll * terms_per_k);
      const long long kc = (long long)ceil_div(P.kblocks, opt->ksplit_override) * 64;
      if (kc > kc_max) return set_err(MPCG_EINVAL, "ksplit_override too small for exact int32 accumulation");
    }
    P.ksplit = std::min(opt->ksplit_override, P.kblocks);
  }
  // make every chunk non-empty
  {
    const int kbps = ceil_div(P.kblocks, P.ksplit);
    P.ksplit = ceil_div(P.kblocks, kbps);
  }
  const size_t esz = P.f64 ? 8 : 1;
  const size_t tiles = (size_t)P.mt * P.nt;
  const size_t nd = (size_t)P.Dmax + 1;
  const size_t dig_bytes = P.f64 ? 4 : 1;
  size_t o = 0;
  P.off_G = o; o = align256(o + 4 * (size_t)P.mpad);
  P.off_H = o; o = align256(o + 4 * (size_t)P.npad);
  P.off_X = o; o = align256(o + (size_t)P.nopsA * P.xs * P.mpad * (size_t)P.kpad * esz);
  P.off_Y = o; o = align256(o + (size_t)P.nopsB * P.ys * P.npad * (size_t)P.kpad * esz);
  P.off_dig = o; o = align256(o + (size_t)P.ksplit * tiles * nd * 512 * dig_bytes);
  P.off_top = o; o = align256(o + (size_t)P.ksplit * tiles * 512 * 8);
  P.off_lnz = o; o = align256(o + (size_t)P.ksplit * tiles * 512 * 4);
  P.total = o;
  return MPCG_OK;
}

int ensure_status_and_pinned() {
  if (!g_status) {
    HIP_TRY(hipMalloc(&g_status, 256));
    HIP_TRY(hipMemset(g_status, 0, 256));
  }
  if (!g_host_summary) HIP_TRY(hipHostMalloc((void**)&g_host_summary, 2 * sizeof(ScanSummary), 0));
  return MPCG_OK;
}

int ensure_scan(size_t bytes) {
  if (bytes <= g_scan_bytes) return MPCG_OK;
  if (g_scan) {
    HIP_TRY(hipStreamSynchronize(g_stream));
    HIP_TRY(hipFree(g_scan));
    g_scan = nullptr;
    g_scan_bytes = 0;
  }
  HIP_TRY(hipMalloc(&g_scan, bytes));
  g_scan_bytes = bytes;
  return MPCG_OK;
}

int ensure_workspace(size_t bytes, void** ptr) {
  if (g_user_ws) {
    if (bytes > g_user_ws_bytes)
      return set_err(MPCG_ENOMEM, "workspace of %zu bytes is too small: %zu needed", g_user_ws_bytes, bytes);
    *ptr = g_user_ws;
    return MPCG_OK;
  }
  if (bytes > g_ws_bytes) {
    if (g_ws) {
      HIP_TRY(hipStreamSynchronize(g_stream));
      HIP_TRY(hipFree(g_ws));
      g_ws = nullptr;
      g_ws_bytes = 0;
    }
    hipError_t e = fault_injected() ? hipErrorNotReady : hipMalloc(&g_ws, bytes);
    if (e == hipErrorOutOfMemory) return set_err(MPCG_ENOMEM, "hipMalloc(%zu) failed: out of memory", bytes);
    if (e != hipSuccess) return set_err(MPCG_EHIP, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    g_ws_bytes = bytes;
  }
  *ptr = g_ws;
  return MPCG_OK;
}

int record(int idx) {
  if (!g_timing) return MPCG_OK;
  if (idx == 0) {
    if (g_ncalls == (int)g_ev.size()) {
      std::array<hipEvent_t, 5> ev{};
      for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
      g_ev.push_back(ev);
    }
    ++g_ncalls;
  }
  HIP_TRY(hipEventRecord(g_ev[g_ncalls - 1][idx], g_stream));
  return MPCG_OK;
}

int validate(int m, int n, int k, const mpcg_cmat* A, int lda, const mpcg_cmat* B, int ldb, mpcg_cmat* C,
             int ldc, int prec_bits, int mode, int scheme, const mpcg_options* opt) {
  if (m < 0 || n < 0 || k < 0) return set_err(MPCG_EINVAL, "negative dimension (m=%d n=%d k=%d)", m, n, k);
  if (prec_bits < MPCG_MIN_PREC || prec_bits > MPCG_MAX_PREC)
    return set_err(MPCG_EINVAL, "prec_bits %d outside [%d, %d]", prec_bits, MPCG_MIN_PREC, MPCG_MAX_PREC);
  if (mode != MPCG_4M && mode != MPCG_3M) return set_err(MPCG_EINVAL, "bad mode %d", mode);
  if (scheme != MPCG_EXACT && scheme != MPCG_TRUNCATED) return set_err(MPCG_EINVAL, "bad scheme %d", scheme);
  if (opt) {
    if (opt->slice_type != MPCG_SLICE_INT8 && opt->slice_type != MPCG_SLICE_FP64)
      return set_err(MPCG_EINVAL, "bad slice_type %d", opt->slice_type);
    if (opt->cutoff_override < 0 || opt->ksplit_override < 0 || opt->block_override < 0)
      return set_err(MPCG_EINVAL, "negative option override");
  }
  if (lda < std::max(1, m)) return set_err(MPCG_EINVAL, "lda %d < max(1, m=%d)", lda, m);
  if (ldb < std::max(1, k)) return set_err(MPCG_EINVAL, "ldb %d < max(1, k=%d)", ldb, k);
  if (ldc < std::max(1, m)) return set_err(MPCG_EINVAL, "ldc %d < max(1, m=%d)", ldc, m);
  if (m == 0 || n == 0) return MPCG_OK;
  if (!C) return set_err(MPCG_EINVAL, "C is NULL");
  const int L = (prec_bits + 63) / 64;
  Region rc[6];
  int st;
  if ((st = check_part(C->re, m, n, ldc, L, "C.re", rc))) return st;
  if ((st = check_part(C->im, m, n, ldc, L, "C.im", rc + 3))) return st;
  for (int a = 0; a < 6; ++a)
    for (int b = a + 1; b < 6; ++b)
      if (overlap(rc[a], rc[b])) return set_err(MPCG_EINVAL, "C arrays overlap each other");
  if (k == 0) return MPCG_OK;
  if (!A || !B) return set_err(MPCG_EINVAL, "A or B is NULL");
  Region ra[12];
  if ((st = check_part(A->re, m, k, lda, L, "A.re", ra))) return st;
  if ((st = check_part(A->im, m, k, lda, L, "A.im", ra + 3))) return st;
  if ((st = check_part(B->re, k, n, ldb, L, "B.re", ra + 6))) return st;
  if ((st = check_part(B->im, k, n, ldb, L, "B.im", ra + 9))) return st;
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 12; ++b)
      if (overlap(rc[a], ra[b])) return set_err(MPCG_EINVAL, "C overlaps A or B");
  return MPCG_OK;
}

int run(int m, int n, int k, const mpcg_cmat* A, int lda, const mpcg_cmat* B, int ldb, mpcg_cmat* C, int ldc,
        int prec_bits, int mode, int scheme, const mpcg_options* opt, mpcg_info* info) {
  g_err.clear();
  int st = validate(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, opt);
  if (st) return st;
  if (info) memset(info, 0, sizeof(*info));
  if (m == 0 || n == 0) return MPCG_OK;
  std::lock_guard<std::mutex> lock(g_mu);
  g_timing_valid = false;
  const int L = (prec_bits + 63) / 64;
  const DOutPart cre = doutpart(C->re, (int64_t)ldc * n), cim = doutpart(C->im, (int64_t)ldc * n);
  if ((st = ensure_status_and_pinned())) return st;
  if (k == 0) {
    HIP_TRY(launch_zero(cre, cim, m, n, ldc, L, g_stream));
    return MPCG_OK;
  }

  // ---- exponent scan -------------------------------------------------------
  DOperand opA{dpart(A->re, (int64_t)lda * k), dpart(A->im, (int64_t)lda * k), m, k, 1, lda};
  DOperand opB{dpart(B->re, (int64_t)ldb * n), dpart(B->im, (int64_t)ldb * n), n, k, ldb, 1};
  const size_t sA = align256(sizeof(RowStat) * (size_t)m), sB = align256(sizeof(RowStat) * (size_t)n);
  if ((st = ensure_scan(sA + sB + 256))) return st;
  RowStat* statA = reinterpret_cast<RowStat*>(g_scan);
  RowStat* statB = reinterpret_cast<RowStat*>((char*)g_scan + sA);
  ScanSummary* summ = reinterpret_cast<ScanSummary*>((char*)g_scan + sA + sB);
  if ((st = record(0))) return st;
  HIP_TRY(launch_scan(opA, statA, summ, g_stream));
  HIP_TRY(launch_scan(opB, statB, summ + 1, g_stream));
  HIP_TRY(hipMemcpyAsync(g_host_summary, summ, 2 * sizeof(ScanSummary), hipMemcpyDeviceToHost, g_stream));
  if ((st = record(1))) return st;
  HIP_TRY(hipStreamSynchronize(g_stream));
  const ScanSummary sa = g_host_summary[0], sb = g_host_summary[1];
  if ((sa.status | sb.status) & ST_IN_RANGE)
    return set_err(MPCG_ERANGE, "input exponent outside [-2^30, 2^30]");
  if (sa.nonzero == 0 || sb.nonzero == 0) {
    HIP_TRY(launch_zero(cre, cim, m, n, ldc, L, g_stream));
    return MPCG_OK;
  }

  // ---- plan ----------------------------------------------------------------
  Plan P{};
  P.m = m; P.n = n; P.k = k; P.p = prec_bits;
  P.mode3m = mode == MPCG_3M;
  P.trunc = scheme == MPCG_TRUNCATED;
  P.f64 = opt && opt->slice_type == MPCG_SLICE_FP64;
  if ((st = plan_slices(P, sa.spread, sb.spread, sa.hat, sb.hat, opt))) return st;
  if ((st = plan_layout(P, opt))) return st;
  if (info) {
    info->S_A = P.SA; info->S_B = P.SB; info->w = P.w; info->cutoff = P.cutoff;
    info->nprod = P.mode3m ? 3 : 4; info->ksplit = P.ksplit; info->block = P.block;
    info->pairs = P.pairs; info->algo_ops = P.algo_ops; info->bound_bits = P.bound_bits;
  }
  void* ws = nullptr;
  if ((st = ensure_workspace(P.total, &ws))) return st;
  char* base = static_cast<char*>(ws);
  int32_t* G = reinterpret_cast<int32_t*>(base + P.off_G);
  int32_t* H = reinterpret_cast<int32_t*>(base + P.off_H);

  // ---- split ---------------------------------------------------------------
  HIP_TRY(launch_scales(statA, m, P.mpad, P.x, G, g_stream));
  HIP_TRY(launch_scales(statB, n, P.npad, P.x, H, g_stream));
  const Third thirdA = P.mode3m ? Third::SUM : Third::NONE;
  const Third thirdB = P.mode3m ? Third::SUM : Third::NEG_IM;
  if (!P.f64) {
    HIP_TRY(launch_split_i8(opA, prec_bits, L, P.SA, P.SAp, P.xs, P.xlo, thirdA, G, P.mpad, P.kpad,
                            reinterpret_cast<int8_t*>(base + P.off_X), g_status, g_stream));
    HIP_TRY(launch_split_i8(opB, prec_bits, L, P.SB, P.SBp, P.ys, P.ylo, thirdB, H, P.npad, P.kpad,
                            reinterpret_cast<int8_t*>(base + P.off_Y), g_status, g_stream));
  } else {
    HIP_TRY(launch_split_f64(opA, prec_bits, L, P.SA, P.SAp, P.w, thirdA, G, P.mpad, P.kpad,
                             reinterpret_cast<double*>(base + P.off_X), g_status, g_stream));
    HIP_TRY(launch_split_f64(opB, prec_bits, L, P.SB, P.SBp, P.w, thirdB, H, P.npad, P.kpad,
                             reinterpret_cast<double*>(base + P.off_Y), g_status, g_stream));
  }
  if ((st = record(2))) return st;

  // ---- slice GEMM + carry chain -------------------------------------------
  int64_t* top = reinterpret_cast<int64_t*>(base + P.off_top);
  int32_t* lnz = reinterpret_cast<int32_t*>(base + P.off_lnz);
  if (!P.f64) {
    GemmArgs ga{};
    ga.X = reinterpret_cast<const int8_t*>(base + P.off_X);
    ga.Y = reinterpret_cast<const int8_t*>(base + P.off_Y);
    ga.mt = P.mt; ga.nt = P.nt; ga.kblocks = P.kblocks; ga.ksplit = P.ksplit;
    ga.SAp = P.SAp; ga.SBp = P.SBp; ga.Dmax = P.Dmax; ga.mode3m = P.mode3m;
    ga.digits = base + P.off_dig; ga.top = top; ga.lnz = lnz;
    ga.xs = P.xs; ga.ys = P.ys; ga.xlo = P.xlo; ga.ylo = P.ylo;
    HIP_TRY(launch_gemm_i8(ga, P.block, g_stream));
  } else {
    GemmF64Args ga{};
    ga.X = reinterpret_cast<const double*>(base + P.off_X);
    ga.Y = reinterpret_cast<const double*>(base + P.off_Y);
    ga.mt = P.mt; ga.nt = P.nt; ga.kblocks = P.kblocks; ga.ksplit = P.ksplit;
    ga.SA = P.SAp; ga.SB = P.SBp; ga.Dmax = P.Dmax; ga.mode3m = P.mode3m; ga.w = P.w;
    ga.digits = reinterpret_cast<uint32_t*>(base + P.off_dig); ga.top = top; ga.lnz = lnz;
    HIP_TRY(launch_gemm_f64(ga, g_stream));
  }
  if ((st = record(3))) return st;

  // ---- merge chunks, round, store -------------------------------------------
  RoundArgs ra{};
  ra.digits = base + P.off_dig;
  ra.digit_bytes = P.f64 ? 4 : 1;
  ra.f64_layout = P.f64;
  ra.top = top; ra.lnz = lnz;
  ra.ksplit = P.ksplit; ra.mt = P.mt; ra.nt = P.nt; ra.Dmax = P.Dmax; ra.w = P.w;
  ra.G = G; ra.H = H; ra.m = m; ra.n = n; ra.prec = prec_bits; ra.L = L;
  ra.cre = cre; ra.cim = cim; ra.ldc = ldc; ra.status = g_status;
  HIP_TRY(launch_round(ra, g_stream));
  if ((st = record(4))) return st;
  g_timing_valid = g_timing;
  return MPCG_OK;
}

}  // namespace

extern "C" {

int mp_cgemm(int m, int n, int k, const mpcg_cmat* A, int lda, const mpcg_cmat* B, int ldb, mpcg_cmat* C, int ldc,
             int prec_bits, int mode, int scheme) {
  return run(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, nullptr, nullptr);
}

int mp_cgemm_ex(int m, int n, int k, const mpcg_cmat* A, int lda, const mpcg_cmat* B, int ldb, mpcg_cmat* C,
                int ldc, int prec_bits, int mode, int scheme, const mpcg_options* opt, mpcg_info* info) {
  return run(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, opt, info);
}

int mpcg_set_stream(void* hip_stream) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_stream = static_cast<hipStream_t>(hip_stream);
  return MPCG_OK;
}

int mpcg_set_workspace(void* dev_ptr, size_t bytes) {
  std::lock_guard<std::mutex> lock(g_mu);
  if ((dev_ptr == nullptr) != (bytes == 0)) return set_err(MPCG_EINVAL, "workspace pointer and size disagree");
  g_user_ws = dev_ptr;
  g_user_ws_bytes = bytes;
  return MPCG_OK;
}

size_t mpcg_workspace_size(int m, int n, int k, int prec_bits, int mode, int scheme, const mpcg_options* opt,
                           int max_spread) {
  if (m <= 0 || n <= 0 || k <= 0 || prec_bits < MPCG_MIN_PREC || prec_bits > MPCG_MAX_PREC || max_spread < 0)
    return 0;
  Plan P{};
  P.m = m; P.n = n; P.k = k; P.p = prec_bits;
  P.mode3m = mode == MPCG_3M;
  P.trunc = scheme == MPCG_TRUNCATED;
  P.f64 = opt && opt->slice_type == MPCG_SLICE_FP64;
  if (plan_slices(P, max_spread, max_spread, max_spread, max_spread, opt)) return 0;
  if (plan_layout(P, opt)) return 0;
  return P.total;
}

int mpcg_stream_status(void* hip_stream) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_status) return MPCG_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  HIP_TRY(hipStreamSynchronize(s));
  int v = 0;
  HIP_TRY(hipMemcpy(&v, g_status, sizeof(int), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(g_status, 0, sizeof(int)));
  if (v & ST_OUT_RANGE) return set_err(MPCG_ERANGE, "output exponent outside int32");
  if (v & ST_DENORM) return set_err(MPCG_EDOMAIN, "nonzero input with clear significand top bit");
  return MPCG_OK;
}

const char* mpcg_last_error(void) { return g_err.c_str(); }

int mpcg_enable_timing(int on) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_timing = on != 0;
  return MPCG_OK;
}

int mpcg_last_timing(float us[4]) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!us) return set_err(MPCG_EINVAL, "NULL output");
  if (!g_timing_valid || g_ncalls == 0) return set_err(MPCG_EINVAL, "no timed multiplication");
  const auto& ev = g_ev[g_ncalls - 1];
  HIP_TRY(hipEventSynchronize(ev[4]));
  for (int s = 0; s < 4; ++s) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev[s], ev[s + 1]));
    us[s] = ms * 1000.f;
  }
  return MPCG_OK;
}

int mpcg_timing_report(float us_sum[4], int* ncalls) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!us_sum || !ncalls) return set_err(MPCG_EINVAL, "NULL output");
  for (int s = 0; s < 4; ++s) us_sum[s] = 0.f;
  *ncalls = 0;
  if (g_ncalls == 0) return MPCG_OK;
  HIP_TRY(hipEventSynchronize(g_ev[g_ncalls - 1][4]));
  int done = 0;
  for (int c = 0; c < g_ncalls; ++c) {
    float st[4];
    bool ok = true;
    for (int s = 0; s < 4 && ok; ++s) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, g_ev[c][s], g_ev[c][s + 1]) != hipSuccess) ok = false;
      st[s] = ms * 1000.f;
    }
    if (!ok) continue;  // a call that returned early (zero result) recorded fewer events
    for (int s = 0; s < 4; ++s) us_sum[s] += st[s];
    ++done;
  }
  *ncalls = done;
  g_ncalls = 0;
  g_timing_valid = false;
  return MPCG_OK;
}

}  // extern "C"
