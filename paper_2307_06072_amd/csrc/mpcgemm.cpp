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

#include <map>

#include <rocblas/rocblas.h>

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
// size-class tuning: the cache of MPCG_TUNE_CACHE is read on first use; while
// mpcg_autotune measures a candidate, g_tune_forced_groups sets the work-item
// target and the cache is not consulted
bool g_tune_env_done = false;
int g_tune_forced_groups = 0;
bool g_tune_bypass = false;                 // plans ignore the cache (tuning measures its candidates)
// when set, a batch records its problems' size classes and band widths
std::vector<std::pair<TuneKey, int>>* g_tune_keys = nullptr;

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
  // the entries addressed: columns 0 .. cols-2 whole (ld each), `rows` of the last
  const int64_t n = cols > 0 ? (int64_t)ld * (cols - 1) + rows : 0;
  const int64_t ls = p.limb_stride ? p.limb_stride : (int64_t)ld * cols;
  if (ls < n)
    return set_err(MPCG_EINVAL, "%s: limb_stride %lld < (cols-1)*ld + rows = %lld", name, (long long)ls,
                   (long long)n);
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
  int want_groups;   // contraction chunks are added until this many work items exist
  int mode_req;      // the caller's form (MPCG_AUTO resolved into mode3m), the tuning cache's key
  int tune_S;        // MPCG_AUTO: the 3M slice count the cache is keyed by (else the plan's own)
  int extra_x;       // more headroom bits (1 for the operand sums of Strassen's recursion)
  int sep;           // the four real products of separately scaled parts (FSEP GEMM form)
  int allow_bsplit;  // the plain path: a product of few work items may run its bands apart
  int bsplit;        // bands on separate workgroups (1: all bands in one work item)
  int psplit;        // with bsplit > 1: the real products of a band group on workgroups of their own
  int allow_onepass; // the plain path and Strassen's products may run one real product per work item
  int onepass_pays;  // ... and that form is expected to be faster for this product (onepass_pays())
  long long fused_items;  // work items of the products together (tile groups x contraction chunks)
  int onepass;       // one real product per work item (GEMM form F3P, psplit = 3, or F4P, psplit = 4;
                     // not with bsplit)
  int nchunk;        // INT8: 16-digit chunks per output component
  size_t off_G, off_H, off_X, off_Y, off_dig, off_top, off_lnz, off_scan, total;
  // FP64 form: slices of A per DGEMM block, the block's products and the diagonal sums
  int schunk, tcnt, ncombo;
  size_t off_C, off_acc;
};

int plan_slices(Plan& P, int spreadA, int spreadB, int hatA, int hatB, const mpcg_options* opt) {
  P.L = (P.p + 63) / 64;
  // headroom bits above the row maximum: the top digit keeps the remaining
  // value, at most 2^(w - x) (twice that for Re + Im in 3M), which must fit
  // an int8 for the INT8 slices (|d| <= 64 with w = 8 and x = 2 or 3)
  P.x = (P.f64 ? (P.mode3m ? 2 : 1) : (P.mode3m ? 3 : 2)) + P.extra_x;
  P.w = P.f64 ? std::max(1, (53 - ceil_log2(std::max(1, P.k))) / 2) : I8_W;
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

// Row statistics of A and B and the two summaries.
size_t scan_bytes(int m, int n) {
  return align256(sizeof(RowStat) * (size_t)m) + align256(sizeof(RowStat) * (size_t)n) + 256;
}

// Work items (2x2 tile groups x contraction chunks) below which the bands of
// a product run on separate workgroups.
constexpr long long BSPLIT_ITEMS = 128;
constexpr int BSPLIT_STREAMS = 16;

// Band width for a product of this form and slice count (measured on MI355X,
// exact 3M and 4M from S = 40 (256 bits) to S = 156 (1024 bits)): in the 3M
// form 20 diagonals per band cut the fragment traffic per MFMA and win from
// S = 76 up; below that the wider band's extra pairs outside the slice square
// cost more.  The 4M form keeps two accumulators and two rings per diagonal,
// for which 16 is the widest band that fits the registers.  A product of at
// most four work items (2 x 2 tile groups x contraction chunks) runs its
// bands in groups on workgroups of their own, and its time follows the
// longest group: narrower bands make more and shorter groups (at 256 bits,
// 1^3 to 64^3 run fastest with 8 diagonals per band; from 5 work items on,
// 16 served the n = 1024 LU's products best, 12 and 8 giving 0.51 s against
// 0.48 s).  A product that is not split in band groups runs each real
// product (3M: 3, 4M: 4) on a workgroup of its own (one accumulator set: two workgroups per
// compute unit) with 16 diagonals, the widest band that then fits; at 2048^3
// and 1024 bits its slice GEMM takes 321 ms against 342 ms for the three
// products together with 20 diagonals, at 512^3 and 512 bits 1.30 against
// 1.50-1.62 ms.
bool onepass_form(const Plan& P, long long items) {
  return P.allow_onepass && P.onepass_pays && !P.f64 && !P.sep && !(P.allow_bsplit && items < BSPLIT_ITEMS);
}
// The form saves slice-GEMM time in proportion to k S per output entry and
// costs the rounding kernel about two more digit streams per contraction
// chunk (and a merge where one chunk needed none), in proportion to S (ks + 1):
// it pays when k S >= 2^14 (ks + 1).  (The 31 trailing updates of the order-
// 4096 LU, k = 128 at 256 bits, lose with it: 97 against 102 ms of GEMM, 36
// against 15 ms of rounding per pass; 512^3 at 512 bits gains, 1.47 against
// 1.65 ms.)  It also pays when the products together would make fewer than
// ONEPASS_FILL_ITEMS work items, two rounds of one workgroup per compute
// unit: apart they fill the chip three times over (256 products of shapes on
// [16, 768]^3 at 256 bits, one call each: 109 against 137 ms).  For 4M only
// the latter holds: its fused kernel already issues two MFMAs per pair of
// fragments, and apart its slice GEMM at 2048^3 / 1024 bits gains 1.4%
// (431 against 437 ms), about what the doubled streams cost the rounding;
// 512^3 at 512 bits, which fills the chip poorly, 1.69 against 1.79 ms.
constexpr long long ONEPASS_FILL_ITEMS = 1024;
bool onepass_pays(const Plan& P, int ks, long long fused_items) {
  return fused_items < ONEPASS_FILL_ITEMS ||
         (P.mode3m && (long long)P.k * std::max(P.SA, P.SB) >= (1ll << 14) * (ks + 1));
}
int pick_band(const Plan& P, long long items) {
  if (P.allow_bsplit && items <= 4 && std::min(P.SA, P.SB) < 64) return 8;
  if (onepass_form(P, items)) return 16;
  return ((P.mode3m || P.sep) && std::min(P.SA, P.SB) >= 64) ? 20 : 16;
}


// Bytes of one block of FP64 slice-plane products (at least one slice of A).
constexpr size_t F64_BLOCK_BYTES = size_t(4) << 30;

int plan_layout(Plan& P, const mpcg_options* opt) {
  P.mpad = (int)round_up(P.m, 32);
  P.npad = (int)round_up(P.n, 32);
  P.kpad = (int)round_up(P.k, 64);
  P.mt = P.mpad / 16;
  P.nt = P.npad / 16;
  P.nopsA = P.mode3m ? 3 : 2;
  P.nopsB = (P.f64 && !P.mode3m) ? 2 : 3;  // the FP64 4M products take Im B itself
  const int groups = (P.mpad / 32) * (P.npad / 32);
  if (!P.f64) {
    // band width: diagonals accumulated together by one wavefront; from the
    // tuning cache for this size class if it has an entry
    TuneChoice tc;
    if (opt && opt->block_override) {
      P.block = opt->block_override;
    } else if (!g_tune_bypass && !P.sep && !(opt && opt->ksplit_override) &&
               tune_find(tune_key(P.trunc, P.mode_req, P.m, P.n, P.k, P.tune_S ? P.tune_S : std::max(P.SA, P.SB)),
                         &tc) &&
               tc.mode3m == P.mode3m) {
      P.block = tc.band;
      P.want_groups = tc.groups;
    } else {
      P.block = 0;  // chosen once the work items are known
    }
    if (g_tune_forced_groups) P.want_groups = g_tune_forced_groups;
    P.kblocks = P.kpad / 64;
    // int32 accumulators: terms per diagonal * 128^2 (the largest digit product)
    // must stay below 2^31
    const long long terms_per_k = (long long)(P.mode3m || P.sep ? 1 : 2) * std::min(P.SA, P.SB);
    const long long kc_max = ((1ll << 31) - 1) / ((1ll << (2 * I8_W - 2)) * terms_per_k);
    const long long kb_max = kc_max / 64;
    if (kb_max < 1) return set_err(MPCG_EUNSUPPORTED, "precision/spread too large for int32 slice accumulation");
    int ks = (int)((P.kblocks + kb_max - 1) / kb_max);
    int want = std::max(1, ceil_div(P.want_groups, groups));
    // the one-product form's three real products are work items too
    {
      const int np = P.mode3m ? 3 : 4;  // real products
      const int ks_one = std::max(ks, std::min(std::max(1, ceil_div(P.want_groups, np * groups)), P.kblocks));
      P.fused_items = (long long)groups * std::max(ks, std::min(want, P.kblocks));
      P.onepass_pays = onepass_pays(P, ks_one, P.fused_items);
    }
    if ((P.block == 0 || P.block <= 16) && onepass_form(P, (long long)groups * std::max(ks, std::min(want, P.kblocks))))
      want = std::max(1, ceil_div(P.want_groups, (P.mode3m ? 3 : 4) * groups));
    ks = std::max(ks, std::min(want, P.kblocks));
    P.ksplit = ks;
    if (P.block == 0) P.block = pick_band(P, (long long)groups * ks);
    if (P.block != 8 && P.block != 12 && P.block != 16 && P.block != 20)
      return set_err(MPCG_EINVAL, "block_override (band width) must be 8, 12, 16 or 20");
    P.SAp = P.SA;
    P.SBp = P.SB;
    // consecutive planes share their zero slices: a plane's upper pad is the
    // next plane's lower pad (the next tile's first plane after a tile's
    // last), and one more pad follows the last tile
    int alo, ahi, blo, bhi;
    gemm_i8_pads(P.block, &alo, &ahi, &blo, &bhi);
    P.xlo = std::max(alo, ahi);
    P.ylo = std::max(blo, bhi);
    P.xs = P.xlo + P.SA;
    P.ys = P.ylo + P.SB;
  } else {
    // DGEMMs of the stacked slice planes: A's slices in blocks of schunk
    // against B's first tcnt slices, the block's products within
    // F64_BLOCK_BYTES; one contraction chunk (the slice width keeps every
    // product entry below 2^53 over the whole contraction)
    P.block = 2;
    P.SAp = P.SA;
    P.SBp = P.SB;
    P.xs = P.SAp;
    P.ys = P.SBp;
    P.xlo = P.ylo = 0;
    P.kblocks = P.kpad / 64;
    P.ksplit = 1;
    P.ncombo = P.mode3m ? 3 : 4;
    P.tcnt = std::min(P.SB, P.Dmax + 1);
    const size_t per_s = (size_t)P.ncombo * P.mpad * (size_t)P.tcnt * P.npad * 8;
    P.schunk = (int)std::max<size_t>(1, std::min<size_t>(P.SA, F64_BLOCK_BYTES / per_s));
    // truncated: about five blocks, each against the B slices its first
    // slice reaches, so that few dropped pairs are computed
    if (P.trunc) P.schunk = std::min(P.schunk, std::max(1, ceil_div(std::min(P.SA, P.Dmax + 1), 5)));
  }
  if (opt && opt->ksplit_override > 0 && !P.f64) {
    if (!P.f64) {
      const long long terms_per_k = (long long)(P.mode3m || P.sep ? 1 : 2) * std::min(P.SA, P.SB);
      const long long kc_max = ((1ll << 31) - 1) / ((1ll << (2 * I8_W - 2)) * terms_per_k);
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
  // a product of few work items runs its bands in groups on workgroups of
  // their own (one digit stream per group, added up by the rounding kernel),
  // so its latency is a group's rather than all bands in turn; at most
  // BSPLIT_STREAMS streams in all
  P.bsplit = 1;
  P.psplit = 1;
  if (P.allow_bsplit && !P.f64 && (long long)groups * P.ksplit < BSPLIT_ITEMS) {
    const int nb = (P.Dmax + P.block) / P.block;
    const int bs = std::max(1, std::min(nb, BSPLIT_STREAMS / P.ksplit));
    P.bsplit = ceil_div(nb, ceil_div(nb, bs));  // no empty group
    // and the real products of a band group apart, when the rounding then
    // reads at most four streams per group and chunk
    const int np = P.mode3m ? 3 : 2;
    if (P.bsplit > 1 && !P.sep && P.ksplit * np <= 4) P.psplit = np;
  }
  // 3M with a band of at most 16 and no band groups: one real product per
  // work item, three streams per contraction chunk
  P.onepass = 0;
  if (P.bsplit == 1 && P.block <= 16 && onepass_form(P, (long long)groups * P.ksplit) &&
      onepass_pays(P, P.ksplit, P.fused_items)) {
    P.onepass = 1;
    P.psplit = P.mode3m ? 3 : 4;
  }
  const int streams = P.ksplit * P.bsplit * P.psplit;
  const size_t esz = P.f64 ? 8 : 1;
  const size_t tiles = (size_t)P.mt * P.nt;
  const size_t nd = (size_t)P.Dmax + 1;
  const size_t dig_bytes = P.f64 ? 4 : 1;
  size_t o = 0;
  P.off_G = o; o = align256(o + 4 * (size_t)P.mpad);
  P.off_H = o; o = align256(o + 4 * (size_t)P.npad);
  // (INT8: a slice of one 16-row tile is 16 kpad bytes; the pad after the last tile)
  P.off_X = o; o = align256(o + (size_t)P.nopsA * P.xs * P.mpad * (size_t)P.kpad * esz + (size_t)P.xlo * 16 * P.kpad);
  P.off_Y = o; o = align256(o + (size_t)P.nopsB * P.ys * P.npad * (size_t)P.kpad * esz + (size_t)P.ylo * 16 * P.kpad);
  if (P.f64) {
    P.off_C = o; o = align256(o + (size_t)P.ncombo * P.schunk * P.mpad * (size_t)P.tcnt * P.npad * 8);
    P.off_acc = o; o = align256(o + 2 * nd * (size_t)P.m * P.n * 8);
    P.off_dig = o; o = align256(o + (size_t)P.ksplit * tiles * nd * 512 * dig_bytes);
  } else {  // [ksplit][tiles][slot 8][chunk][lane 64][16] digit bytes
    P.nchunk = gemm_i8_digit_chunks(P.Dmax, P.block);
    P.off_dig = o; o = align256(o + (size_t)streams * tiles * 8 * P.nchunk * 1024);
  }
  P.off_top = o; o = align256(o + (size_t)streams * tiles * 512 * 8);
  P.off_lnz = o; o = align256(o + (size_t)streams * tiles * 512 * 4);
  P.off_scan = o; o = align256(o + scan_bytes(P.m, P.n));
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
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();  // the failed allocation is not an error of the next launch
      return set_err(MPCG_ENOMEM, "hipMalloc(%zu) failed: out of memory", bytes);
    }
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

// check_overlap = false is for the factorization's own calls, whose operands
// are element-disjoint views of one matrix (the scan and split read A and B
// before the rounding kernel writes C, in stream order) and whose arrays were
// checked once for the whole matrix: a view's ld x cols region can run past
// the end of its array.
int validate(int m, int n, int k, const mpcg_cmat* A, int lda, const mpcg_cmat* B, int ldb, mpcg_cmat* C,
             int ldc, int prec_bits, int mode, int scheme, const mpcg_options* opt, bool check_overlap = true) {
  if (m < 0 || n < 0 || k < 0) return set_err(MPCG_EINVAL, "negative dimension (m=%d n=%d k=%d)", m, n, k);
  if (prec_bits < MPCG_MIN_PREC || prec_bits > MPCG_MAX_PREC)
    return set_err(MPCG_EINVAL, "prec_bits %d outside [%d, %d]", prec_bits, MPCG_MIN_PREC, MPCG_MAX_PREC);
  if (mode != MPCG_4M && mode != MPCG_3M && mode != MPCG_AUTO) return set_err(MPCG_EINVAL, "bad mode %d", mode);
  if (scheme != MPCG_EXACT && scheme != MPCG_TRUNCATED) return set_err(MPCG_EINVAL, "bad scheme %d", scheme);
  if (opt) {
    if (opt->slice_type != MPCG_SLICE_INT8 && opt->slice_type != MPCG_SLICE_FP64)
      return set_err(MPCG_EINVAL, "bad slice_type %d", opt->slice_type);
    if (opt->cutoff_override < 0 || opt->ksplit_override < 0 || opt->block_override < 0 || opt->max_spread < 0)
      return set_err(MPCG_EINVAL, "negative option");
    if (opt->max_spread > (1 << 24)) return set_err(MPCG_EINVAL, "max_spread %d too large", opt->max_spread);
    if (opt->adaptive < 0 || (opt->adaptive > 1 && (opt->adaptive % 32 != 0 || opt->adaptive > (1 << 20))))
      return set_err(MPCG_EINVAL, "adaptive must be 0, 1 or a block size that is a multiple of 32");
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
  for (int a = 0; a < 6 && check_overlap; ++a)
    for (int b = a + 1; b < 6; ++b)
      if (overlap(rc[a], rc[b])) return set_err(MPCG_EINVAL, "C arrays overlap each other");
  if (k == 0) return MPCG_OK;
  if (!A || !B) return set_err(MPCG_EINVAL, "A or B is NULL");
  Region ra[12];
  if ((st = check_part(A->re, m, k, lda, L, "A.re", ra))) return st;
  if ((st = check_part(A->im, m, k, lda, L, "A.im", ra + 3))) return st;
  if ((st = check_part(B->re, k, n, ldb, L, "B.re", ra + 6))) return st;
  if ((st = check_part(B->im, k, n, ldb, L, "B.im", ra + 9))) return st;
  for (int a = 0; a < 6 && check_overlap; ++a)
    for (int b = 0; b < 12; ++b)
      if (overlap(rc[a], ra[b])) return set_err(MPCG_EINVAL, "C overlaps A or B");
  return MPCG_OK;
}

int run_batched(int count, const mpcg_problem* probs, int prec_bits, int mode, int scheme,
                const mpcg_options* opt, mpcg_info* info, int acc, bool check_overlap,
                size_t* size_query = nullptr);
mpcg_cmat view_at(const mpcg_cmat& M, int ld, int cols, int r, int c);

// Contiguous blocks of rows (of A) or columns (of B) for adaptive slicing:
// blocks of BLK, neighbours with the same slice count (and, truncated, the
// same hat spread in digits) merged.  Returns the block starts, plus the end.
std::vector<int> adaptive_blocks(const std::vector<RowStat>& st, int p, int x, bool trunc, int BLK) {
  const int R = (int)st.size();
  std::vector<int> starts;
  std::vector<std::pair<int, int>> keys;
  for (int r0 = 0; r0 < R; r0 += BLK) {
    int spread = -1, hat = -1;
    for (int r = r0; r < std::min(R, r0 + BLK); ++r)
      if (st[r].emax != EXP_ZERO) {
        spread = std::max(spread, st[r].emax - st[r].emin);
        hat = std::max(hat, st[r].emax - st[r].ehat);
      }
    std::pair<int, int> key{spread < 0 ? -1 : ceil_div(p + x + spread, I8_W),
                            trunc && hat >= 0 ? ceil_div(hat, I8_W) : 0};
    if (!starts.empty() && (key.first < 0 || keys.back() == key)) continue;  // all-zero blocks join a neighbour
    if (!starts.empty() && keys.back().first < 0) {
      keys.back() = key;  // a leading all-zero block takes the next block's key
      continue;
    }
    starts.push_back(r0);
    keys.push_back(key);
  }
  starts.push_back(R);
  return starts;
}

// acc = 0: C := AB; acc = +1 / -1: C := C + AB / C - AB, one rounding of the
// exact sum (C's current entries are the addend).
// Reads the tuning cache named by MPCG_TUNE_CACHE once per process (a
// missing file is not an error; a malformed one is ignored).
void tune_env_load() {
  if (g_tune_env_done) return;
  g_tune_env_done = true;
  const char* path = getenv("MPCG_TUNE_CACHE");
  if (path && *path) (void)tune_load(path);
}

// The slice count a request of MPCG_AUTO is keyed by: the 3M form's.
int auto_key_S(int p, int spreadA, int spreadB) { return ceil_div(p + 3 + std::max(spreadA, spreadB), I8_W); }

// The form for a request of MPCG_AUTO: the tuning cache's choice for the size
// class, else 3M.
int resolve_mode(int mode, int scheme, int m, int n, int k, int p, int spreadA, int spreadB) {
  if (mode != MPCG_AUTO) return mode;
  const int S = auto_key_S(p, spreadA, spreadB);
  TuneChoice tc;
  if (!g_tune_bypass && tune_find(tune_key(scheme, MPCG_AUTO, m, n, k, S), &tc)) return tc.mode3m ? MPCG_3M : MPCG_4M;
  return MPCG_3M;
}

// ---------------------------------------------------------------------------
// One level of Strassen's recursion (Algorithm 1) over the slice products.
// The operand quadrants' sums and differences are split exactly (one more
// bit of headroom in the folded row scales), the seven half-size products
// run as ordinary slice GEMMs, and each quadrant of C is the signed sum of
// two or four products' exact digit streams, formed in the rounding kernel
// before the single rounding: the same bits as the plain product.
// ---------------------------------------------------------------------------
constexpr int STRASSEN_DECLINED = 1;  // not applicable here: the plain product runs

DOperand quad(const DOperand& op, int br, int bk, int hR, int hK) {
  DOperand q = op;
  const int64_t off = (int64_t)br * hR * op.rs + (int64_t)bk * hK * op.ks;
  q.re.sign += off; q.re.exp += off; q.re.mant += off;
  q.im.sign += off; q.im.exp += off; q.im.mant += off;
  q.R = hR;
  q.K = hK;
  return q;
}

DOutPart quad_out(const DOutPart& c, int64_t off) {
  DOutPart q = c;
  q.sign += off; q.exp += off; q.mant += off;
  return q;
}

// Largest spread of the folded rows (r with r + half): -1 if all are zero.
int folded_spread(const std::vector<RowStat>& st, int half) {
  int spread = -1;
  for (int r = 0; r < half; ++r) {
    int32_t hi = INT32_MIN, lo = INT32_MAX;
    for (const RowStat& x : {st[r], st[r + half]})
      if (x.emax != EXP_ZERO) {
        hi = std::max(hi, x.emax);
        lo = std::min(lo, x.emin);
      }
    if (hi != INT32_MIN) spread = std::max(spread, hi - lo);
  }
  return spread;
}

int run_strassen(int m, int n, int k, const DOperand& opA, const DOperand& opB, int prec_bits, int mode3m,
                 int mode_req, const mpcg_options* opt, mpcg_info* info, const RowStat* statA, const RowStat* statB,
                 const DOutPart& cre, const DOutPart& cim, int64_t ldc) {
  const int hm = m / 2, hn = n / 2, hk = k / 2;
  const int L = (prec_bits + 63) / 64;
  std::vector<RowStat> hA(m), hB(n);
  HIP_TRY(hipMemcpyAsync(hA.data(), statA, sizeof(RowStat) * m, hipMemcpyDeviceToHost, g_stream));
  HIP_TRY(hipMemcpyAsync(hB.data(), statB, sizeof(RowStat) * n, hipMemcpyDeviceToHost, g_stream));
  HIP_TRY(hipStreamSynchronize(g_stream));
  const int spA = folded_spread(hA, hm), spB = folded_spread(hB, hn);
  if (spA < 0 || spB < 0) return STRASSEN_DECLINED;
  Plan Q{};
  Q.m = hm; Q.n = hn; Q.k = hk; Q.p = prec_bits;
  Q.mode_req = mode_req;
  Q.mode3m = mode3m;
  Q.trunc = 0;
  Q.f64 = 0;
  Q.want_groups = 512;
  Q.extra_x = 1;
  Q.allow_onepass = 1;
  int st;
  if ((st = plan_slices(Q, spA, spB, spA, spB, opt))) return st;
  if ((st = plan_layout(Q, opt))) return st;
  if (Q.onepass && 4 * Q.ksplit * Q.psplit > MAX_MERGE) {  // the real products together
    Q.allow_onepass = 0;
    if ((st = plan_layout(Q, opt))) return st;
  }
  const int qstreams = Q.ksplit * Q.psplit;  // digit streams of one product
  if (4 * qstreams > MAX_MERGE) return STRASSEN_DECLINED;
  const size_t stride = align256(Q.total);
  const size_t tiles = (size_t)Q.mt * Q.nt;
  const size_t qbytes = align256(tiles * 8 * Q.nchunk * 1024);  // one quadrant's recombined digits
  void* ws = nullptr;
  if ((st = ensure_workspace(7 * stride + 4 * qbytes + align256(sizeof(MergeSrc) * 8 * MAX_MERGE), &ws))) {
    if (st != MPCG_ENOMEM) return st;
    g_err.clear();  // seven plan layouts do not fit: the plain product runs
    return STRASSEN_DECLINED;
  }
  char* base = static_cast<char*>(ws);
  int32_t* G = reinterpret_cast<int32_t*>(base + Q.off_G);
  int32_t* H = reinterpret_cast<int32_t*>(base + Q.off_H);
  HIP_TRY(launch_fold_scales(statA, hm, Q.mpad, Q.x, G, g_stream));
  HIP_TRY(launch_fold_scales(statB, hn, Q.npad, Q.x, H, g_stream));
  // quadrants: A_ij = rows block i, k block j; B_ij = k block i, column block j
  auto Aq = [&](int i, int j) { return quad(opA, i, j, hm, hk); };
  auto Bq = [&](int i, int j) { return quad(opB, j, i, hn, hk); };
  struct Side { DOperand x, y; int sign; };
  struct Prod { Side a, b; };
  const Prod prods[7] = {
      {{Aq(0, 0), Aq(1, 1), +1}, {Bq(0, 0), Bq(1, 1), +1}},  // M1 = (A11 + A22)(B11 + B22)
      {{Aq(1, 0), Aq(1, 1), +1}, {Bq(0, 0), Bq(0, 0), 0}},   // M2 = (A21 + A22) B11
      {{Aq(0, 0), Aq(0, 0), 0}, {Bq(0, 1), Bq(1, 1), -1}},   // M3 = A11 (B12 - B22)
      {{Aq(1, 1), Aq(1, 1), 0}, {Bq(1, 0), Bq(0, 0), -1}},   // M4 = A22 (B21 - B11)
      {{Aq(0, 0), Aq(0, 1), +1}, {Bq(1, 1), Bq(1, 1), 0}},   // M5 = (A11 + A12) B22
      {{Aq(1, 0), Aq(0, 0), -1}, {Bq(0, 0), Bq(0, 1), +1}},  // M6 = (A21 - A11)(B11 + B12)
      {{Aq(0, 1), Aq(1, 1), -1}, {Bq(1, 0), Bq(1, 1), +1}},  // M7 = (A12 - A22)(B21 + B22)
  };
  const Third thirdA = Q.mode3m ? Third::SUM : Third::NONE;
  const Third thirdB = Q.mode3m ? Third::SUM : Third::NEG_IM;
  for (int j = 0; j < 7; ++j) {
    char* pb = base + j * stride;
    int8_t* X = reinterpret_cast<int8_t*>(pb + Q.off_X);
    int8_t* Y = reinterpret_cast<int8_t*>(pb + Q.off_Y);
    const Prod& P = prods[j];
    if (P.a.sign)
      HIP_TRY(launch_split2_i8(P.a.x, P.a.y, P.a.sign, prec_bits, L, Q.SA, Q.SAp, Q.xs, Q.xlo, thirdA, G, Q.mpad,
                               Q.kpad, X, g_status, g_stream));
    else
      HIP_TRY(launch_split_i8(P.a.x, prec_bits, L, Q.SA, Q.SAp, Q.xs, Q.xlo, thirdA, G, Q.mpad, Q.kpad, X, g_status,
                              g_stream));
    if (P.b.sign)
      HIP_TRY(launch_split2_i8(P.b.x, P.b.y, P.b.sign, prec_bits, L, Q.SB, Q.SBp, Q.ys, Q.ylo, thirdB, H, Q.npad,
                               Q.kpad, Y, g_status, g_stream));
    else
      HIP_TRY(launch_split_i8(P.b.x, prec_bits, L, Q.SB, Q.SBp, Q.ys, Q.ylo, thirdB, H, Q.npad, Q.kpad, Y, g_status,
                              g_stream));
  }
  if ((st = record(2))) return st;
  for (int j = 0; j < 7; ++j) {
    char* pb = base + j * stride;
    GemmArgs ga{};
    ga.X = reinterpret_cast<const int8_t*>(pb + Q.off_X);
    ga.Y = reinterpret_cast<const int8_t*>(pb + Q.off_Y);
    ga.mt = Q.mt; ga.nt = Q.nt; ga.kblocks = Q.kblocks; ga.ksplit = Q.ksplit; ga.psplit = Q.psplit;
    ga.SAp = Q.SAp; ga.SBp = Q.SBp; ga.Dmax = Q.Dmax;
    ga.form = Q.onepass ? (Q.mode3m ? F3P : F4P) : (Q.mode3m ? F3M : F4M);
    ga.digits = pb + Q.off_dig;
    ga.top = reinterpret_cast<int64_t*>(pb + Q.off_top);
    ga.lnz = reinterpret_cast<int32_t*>(pb + Q.off_lnz);
    ga.xs = Q.xs; ga.ys = Q.ys; ga.xlo = Q.xlo; ga.ylo = Q.ylo;
    HIP_TRY(launch_gemm_i8(ga, Q.block, g_stream));
  }
  if ((st = record(3))) return st;
  // C11 = M1 + M4 - M5 + M7, C12 = M3 + M5, C21 = M2 + M4, C22 = M1 - M2 + M3 + M6
  struct Term { int prod, sign; };
  const std::vector<Term> terms[4] = {{{0, +1}, {3, +1}, {4, -1}, {6, +1}},
                                      {{2, +1}, {4, +1}},
                                      {{1, +1}, {3, +1}},
                                      {{0, +1}, {1, -1}, {2, +1}, {5, +1}}};
  const size_t sstride = tiles * 8 * Q.nchunk * 1024;  // one stream's digits
  char* merged = base + 7 * stride;
  MergeSrc* srcdev = reinterpret_cast<MergeSrc*>(base + 7 * stride + 4 * qbytes);
  // per quadrant, the Re sources then the Im sources (in the one-product
  // form T3's streams hold no Re digits, a 4M product's only one component)
  MergeSrc srcs[4][2][MAX_MERGE] = {};
  int nsrc[4][2] = {};
  for (int qd = 0; qd < 4; ++qd)
    for (const Term& t : terms[qd])
      for (int c = 0; c < qstreams; ++c)  // contraction chunks (and real products)
        for (int comp = 0; comp < 2; ++comp) {
          if (Q.onepass && (Q.mode3m ? (comp == 0 && c % 3 == 2) : ((c % 4 < 2) != (comp == 0)))) continue;
          char* pb = base + t.prod * stride;
          MergeSrc& ms = srcs[qd][comp][nsrc[qd][comp]++];
          ms.dig = reinterpret_cast<const uint8_t*>(pb + Q.off_dig) + c * sstride;
          ms.top = reinterpret_cast<const int64_t*>(pb + Q.off_top) + (size_t)c * tiles * 512;
          ms.sign = t.sign;
        }
  HIP_TRY(launch_store_words(srcdev, srcs, sizeof(srcs), g_stream));
  for (int qd = 0; qd < 4; ++qd) {
    const int qr = qd >> 1, qc = qd & 1;
    RoundArgs ra{};
    ra.digits = merged + qd * qbytes;
    ra.digit_bytes = 1;
    ra.nchunk = Q.nchunk;
    ra.f64_layout = 0;
    ra.ksplit = 1; ra.mt = Q.mt; ra.nt = Q.nt; ra.Dmax = Q.Dmax; ra.w = Q.w;
    ra.G = G; ra.H = H; ra.m = hm; ra.n = hn; ra.prec = prec_bits; ra.L = L;
    const int64_t off = (int64_t)qc * hn * ldc + (int64_t)qr * hm;
    ra.cre = quad_out(cre, off);
    ra.cim = quad_out(cim, off);
    ra.ldc = ldc;
    ra.status = g_status;
    ra.acc = 0;
    ra.nsrc = nsrc[qd][0];
    ra.nsrc_im = nsrc[qd][1];
    ra.src = srcdev + qd * 2 * MAX_MERGE;
    ra.top = srcs[qd][0][0].top;  // not read when nsrc > 0
    ra.lnz = reinterpret_cast<const int32_t*>(base + Q.off_lnz);
    HIP_TRY(launch_round(ra, g_stream));
  }
  if ((st = record(4))) return st;
  if (info) {
    info->S_A = Q.SA; info->S_B = Q.SB; info->w = Q.w; info->cutoff = Q.cutoff;
    info->nprod = Q.mode3m ? 3 : 4; info->ksplit = Q.ksplit; info->block = Q.block; info->apart = Q.onepass;
    info->pairs = Q.pairs; info->algo_ops = 7 * Q.algo_ops; info->bound_bits = 0;
    info->strassen = 1;
  }
  g_timing_valid = g_timing;
  return MPCG_OK;
}

// ---------------------------------------------------------------------------
// FP64 form: the slice-plane products as DGEMMs (rocBLAS), accumulated
// exactly into the diagonals, then carried into digit streams.
// ---------------------------------------------------------------------------
std::map<int, rocblas_handle> g_blas;  // per device, created on first use

int blas_handle(rocblas_handle* h) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  auto it = g_blas.find(dev);
  if (it == g_blas.end()) {
    rocblas_handle nh;
    const rocblas_status bs = rocblas_create_handle(&nh);
    if (bs != rocblas_status_success) return set_err(MPCG_EHIP, "rocblas_create_handle: %s", rocblas_status_to_string(bs));
    it = g_blas.emplace(dev, nh).first;
  }
  const rocblas_status bs = rocblas_set_stream(it->second, g_stream);
  if (bs != rocblas_status_success) return set_err(MPCG_EHIP, "rocblas_set_stream: %s", rocblas_status_to_string(bs));
  *h = it->second;
  return MPCG_OK;
}

// X: nopsA planes of SA slices of mpad rows, column-major with leading
// dimension nopsA SA mpad; Y alike.  Products of plane pairs (4M: (0,0),
// (1,1), (0,1), (1,0); 3M: (0,0), (1,1), (2,2)), A's slices in blocks.
int f64_products(const Plan& P, char* base, int L) {
  (void)L;
  rocblas_handle h;
  int st;
  if ((st = blas_handle(&h))) return st;
  const double* X = reinterpret_cast<const double*>(base + P.off_X);
  const double* Y = reinterpret_cast<const double*>(base + P.off_Y);
  double* C = reinterpret_cast<double*>(base + P.off_C);
  int64_t* acc = reinterpret_cast<int64_t*>(base + P.off_acc);
  const int64_t ldx = (int64_t)P.nopsA * P.SAp * P.mpad, ldy = (int64_t)P.nopsB * P.SBp * P.npad;
  HIP_TRY(launch_fill_zero(acc, 2 * (size_t)(P.Dmax + 1) * P.m * P.n * 8, g_stream));
  static const int pairs4[4][2] = {{0, 0}, {1, 1}, {0, 1}, {1, 0}};
  static const int pairs3[3][2] = {{0, 0}, {1, 1}, {2, 2}};
  const double one = 1.0, zero = 0.0;
  const int smax = std::min(P.SA, P.Dmax + 1);  // slices of A that reach a kept diagonal
  for (int s0 = 0; s0 < smax; s0 += P.schunk) {
    const int s1 = std::min(smax, s0 + P.schunk);
    const int tcnt = std::min(P.tcnt, P.Dmax - s0 + 1);  // B slices reaching a kept diagonal
    const int M = (s1 - s0) * P.mpad, N = tcnt * P.npad;
    F64AccArgs fa{};
    for (int q = 0; q < P.ncombo; ++q) {
      const int oa = P.mode3m ? pairs3[q][0] : pairs4[q][0], ob = P.mode3m ? pairs3[q][1] : pairs4[q][1];
      double* Cq = C + (size_t)q * P.schunk * P.mpad * (size_t)P.tcnt * P.npad;
      const double* Xq = X + ((int64_t)oa * P.SAp + s0) * P.mpad;
      const double* Yq = Y + (int64_t)ob * P.SBp * P.npad;
      const rocblas_status bs = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, M, N, P.kpad,
                                              &one, Xq, ldx, Yq, ldy, &zero, Cq, M);
      if (bs != rocblas_status_success) return set_err(MPCG_EHIP, "rocblas_dgemm: %s", rocblas_status_to_string(bs));
      fa.C[q] = Cq;
    }
    fa.ldc = M;
    fa.s0 = s0; fa.s1 = s1; fa.tcnt = tcnt;
    fa.mpad = P.mpad; fa.npad = P.npad; fa.m = P.m; fa.n = P.n;
    fa.Dmax = P.Dmax; fa.mode3m = P.mode3m;
    fa.acc = acc;
    HIP_TRY(launch_f64_accumulate(fa, g_stream));
  }
  F64CarryArgs ca{};
  ca.acc = acc;
  ca.m = P.m; ca.n = P.n; ca.mt = P.mt; ca.nt = P.nt; ca.Dmax = P.Dmax; ca.w = P.w;
  ca.digits = reinterpret_cast<uint32_t*>(base + P.off_dig);
  ca.top = reinterpret_cast<int64_t*>(base + P.off_top);
  ca.lnz = reinterpret_cast<int32_t*>(base + P.off_lnz);
  HIP_TRY(launch_f64_carry(ca, g_stream));
  return MPCG_OK;
}

// ---------------------------------------------------------------------------
// Separate scales for the Re and Im parts (4M, exact): each part of a row of
// A (column of B) is scaled by its own maximum, so a part far below the
// other costs no slices; the four real products run as two GEMMs of two
// separate products each, and the rounding kernel merges each component's
// two streams, shifted by the whole digits between their scales, before the
// one rounding.  The scales of a row's two parts are made to agree modulo 8
// (at most 7 bits more headroom for one of them).
// ---------------------------------------------------------------------------
constexpr int PARTS_DECLINED = 1;  // no fewer slice pairs than one scale: the plain product runs
constexpr int PARTS_MAX_SHIFT = 4096;  // digits between the scales of one component's products

struct PartScales {
  std::vector<int32_t> Gre, Gim;  // scales of the Re and Im parts per row (column)
  int need = 0;                   // bits the slices must hold: max over parts of G - emin + p
  int maxq = 0;                   // max |G_re - G_im| / 8
  bool any = false;
};

PartScales part_scales(const std::vector<RowStat>& re, const std::vector<RowStat>& im, int x, int p) {
  PartScales ps;
  const size_t R = re.size();
  ps.Gre.assign(R, 0);
  ps.Gim.assign(R, 0);
  for (size_t r = 0; r < R; ++r) {
    const bool zr = re[r].emax == EXP_ZERO, zi = im[r].emax == EXP_ZERO;
    int64_t gr = 0, gi = 0;
    if (!zr && !zi) {
      gr = (int64_t)re[r].emax + x;
      const int64_t gi_nat = (int64_t)im[r].emax + x;
      const int64_t d = gr - gi_nat;
      const int64_t fl = d >= 0 ? d / I8_W : -((-d + I8_W - 1) / I8_W);  // floor(d / 8)
      gi = gr - (int64_t)I8_W * fl;  // >= gi_nat, within 7 bits of it
    } else if (!zr) {
      gr = gi = (int64_t)re[r].emax + x;
    } else if (!zi) {
      gr = gi = (int64_t)im[r].emax + x;
    }
    ps.Gre[r] = (int32_t)gr;
    ps.Gim[r] = (int32_t)gi;
    if (!zr) ps.need = std::max<int64_t>(ps.need, gr - re[r].emin + p);
    if (!zi) ps.need = std::max<int64_t>(ps.need, gi - im[r].emin + p);
    ps.any = ps.any || !zr || !zi;
    ps.maxq = std::max<int64_t>(ps.maxq, std::llabs(gr - gi) / I8_W);
  }
  return ps;
}

int run_parts(int m, int n, int k, const DOperand& opA, const DOperand& opB, int prec_bits,
              const mpcg_options* opt, mpcg_info* info, int SA_common, int SB_common, const DOutPart& cre,
              const DOutPart& cim, int64_t ldc) {
  const int L = (prec_bits + 63) / 64;
  // per-part statistics: the scan of a view whose two parts are the same part
  DOperand vAr = opA, vAi = opA, vBr = opB, vBi = opB;
  vAr.im = opA.re;
  vAi.re = opA.im;
  vBr.im = opB.re;
  vBi.re = opB.im;
  const size_t sA = align256(sizeof(RowStat) * (size_t)m), sB = align256(sizeof(RowStat) * (size_t)n);
  void* ws = nullptr;
  int st;
  if ((st = ensure_workspace(2 * sA + 2 * sB + 256, &ws))) return st;
  {
    char* b = static_cast<char*>(ws);
    RowStat* s0 = reinterpret_cast<RowStat*>(b);
    RowStat* s1 = reinterpret_cast<RowStat*>(b + sA);
    RowStat* s2 = reinterpret_cast<RowStat*>(b + 2 * sA);
    RowStat* s3 = reinterpret_cast<RowStat*>(b + 2 * sA + sB);
    ScanSummary* summ = reinterpret_cast<ScanSummary*>(b + 2 * sA + 2 * sB);
    HIP_TRY(launch_scan(vAr, s0, summ, 0, nullptr, g_stream));
    HIP_TRY(launch_scan(vAi, s1, summ + 1, 0, nullptr, g_stream));
    HIP_TRY(launch_scan(vBr, s2, summ + 2, 0, nullptr, g_stream));
    HIP_TRY(launch_scan(vBi, s3, summ + 3, 0, nullptr, g_stream));
  }
  std::vector<RowStat> aR(m), aI(m), bR(n), bI(n);
  {
    char* b = static_cast<char*>(ws);
    HIP_TRY(hipMemcpyAsync(aR.data(), b, sizeof(RowStat) * m, hipMemcpyDeviceToHost, g_stream));
    HIP_TRY(hipMemcpyAsync(aI.data(), b + sA, sizeof(RowStat) * m, hipMemcpyDeviceToHost, g_stream));
    HIP_TRY(hipMemcpyAsync(bR.data(), b + 2 * sA, sizeof(RowStat) * n, hipMemcpyDeviceToHost, g_stream));
    HIP_TRY(hipMemcpyAsync(bI.data(), b + 2 * sA + sB, sizeof(RowStat) * n, hipMemcpyDeviceToHost, g_stream));
    HIP_TRY(hipStreamSynchronize(g_stream));
  }
  const int x = 2;  // the 4M headroom of plan_slices
  const PartScales pa = part_scales(aR, aI, x, prec_bits), pb = part_scales(bR, bI, x, prec_bits);
  if (!pa.any || !pb.any) return PARTS_DECLINED;
  const int qmax = pa.maxq + pb.maxq;
  Plan Q{};
  Q.m = m; Q.n = n; Q.k = k; Q.p = prec_bits;
  Q.mode_req = MPCG_4M;
  Q.mode3m = 0;
  Q.sep = 1;
  Q.want_groups = 512;
  // plan_slices takes S = ceil((p + x + spread) / 8): pass the spread that gives `need` bits
  int spA = pa.need - prec_bits - x, spB = pb.need - prec_bits - x;
  if ((st = plan_slices(Q, spA, spB, spA, spB, opt))) return st;
  if ((long long)Q.SA * Q.SB >= (long long)SA_common * SB_common || qmax > PARTS_MAX_SHIFT)
    return PARTS_DECLINED;
  if ((st = plan_layout(Q, opt))) return st;
  const size_t tiles = (size_t)Q.mt * Q.nt;
  const size_t dig_b = align256((size_t)Q.ksplit * tiles * 8 * Q.nchunk * 1024);
  const size_t top_b = align256((size_t)Q.ksplit * tiles * 512 * 8);
  const size_t lnz_b = align256((size_t)Q.ksplit * tiles * 512 * 4);
  const int nchunk_m = (Q.Dmax + 1 + qmax + 15) / 16;
  const size_t mer_b = align256(tiles * 8 * (size_t)nchunk_m * 1024);
  const size_t sc_b = 2 * align256(4 * (size_t)Q.mpad) + 2 * align256(4 * (size_t)Q.npad);
  const size_t total = align256(Q.total) + dig_b + top_b + lnz_b + mer_b + sc_b + 256;
  if ((st = ensure_workspace(total, &ws))) {
    if (st != MPCG_ENOMEM) return st;
    g_err.clear();  // the two product layouts do not fit: one scale runs
    return PARTS_DECLINED;
  }
  char* base = static_cast<char*>(ws);
  char* p2 = base + align256(Q.total);
  uint8_t* dig2 = reinterpret_cast<uint8_t*>(p2);
  int64_t* top2 = reinterpret_cast<int64_t*>(p2 + dig_b);
  int32_t* lnz2 = reinterpret_cast<int32_t*>(p2 + dig_b + top_b);
  uint8_t* merged = reinterpret_cast<uint8_t*>(p2 + dig_b + top_b + lnz_b);
  char* scp = p2 + dig_b + top_b + lnz_b + mer_b;
  int32_t* dGr = reinterpret_cast<int32_t*>(scp);
  int32_t* dGi = reinterpret_cast<int32_t*>(scp + align256(4 * (size_t)Q.mpad));
  int32_t* dHr = reinterpret_cast<int32_t*>(scp + 2 * align256(4 * (size_t)Q.mpad));
  int32_t* dHi = reinterpret_cast<int32_t*>(scp + 2 * align256(4 * (size_t)Q.mpad) + align256(4 * (size_t)Q.npad));
  PartsMerge* dpm = reinterpret_cast<PartsMerge*>(scp + sc_b);
  // scales (padding rows take 0, as from the scale kernel)
  std::vector<int32_t> hG(Q.mpad, 0), hGi(Q.mpad, 0), hH(Q.npad, 0), hHi(Q.npad, 0);
  std::copy(pa.Gre.begin(), pa.Gre.end(), hG.begin());
  std::copy(pa.Gim.begin(), pa.Gim.end(), hGi.begin());
  std::copy(pb.Gre.begin(), pb.Gre.end(), hH.begin());
  std::copy(pb.Gim.begin(), pb.Gim.end(), hHi.begin());
  HIP_TRY(hipMemcpyAsync(dGr, hG.data(), 4 * (size_t)Q.mpad, hipMemcpyHostToDevice, g_stream));
  HIP_TRY(hipMemcpyAsync(dGi, hGi.data(), 4 * (size_t)Q.mpad, hipMemcpyHostToDevice, g_stream));
  HIP_TRY(hipMemcpyAsync(dHr, hH.data(), 4 * (size_t)Q.npad, hipMemcpyHostToDevice, g_stream));
  HIP_TRY(hipMemcpyAsync(dHi, hHi.data(), 4 * (size_t)Q.npad, hipMemcpyHostToDevice, g_stream));
  PartsMerge pm{};
  pm.dig[0] = reinterpret_cast<const uint8_t*>(base + Q.off_dig);
  pm.dig[1] = dig2;
  pm.top[0] = reinterpret_cast<const int64_t*>(base + Q.off_top);
  pm.top[1] = top2;
  pm.nchunk = Q.nchunk;
  pm.ksplit = Q.ksplit;
  pm.Gre = dGr; pm.Gim = dGi; pm.Hre = dHr; pm.Him = dHi;
  HIP_TRY(hipMemcpyAsync(dpm, &pm, sizeof(pm), hipMemcpyHostToDevice, g_stream));
  // the host arrays are pageable: wait for the copies before they go away
  HIP_TRY(hipStreamSynchronize(g_stream));
  int8_t* X = reinterpret_cast<int8_t*>(base + Q.off_X);
  int8_t* Y = reinterpret_cast<int8_t*>(base + Q.off_Y);
  HIP_TRY(launch_split_parts_i8(opA, prec_bits, L, Q.SA, Q.SAp, Q.xs, Q.xlo, Third::NONE, dGr, dGi, Q.mpad, Q.kpad,
                                X, g_status, g_stream));
  // B planes (Re, Im, Re): from the second plane on they read (Im, Re)
  HIP_TRY(launch_split_parts_i8(opB, prec_bits, L, Q.SB, Q.SBp, Q.ys, Q.ylo, Third::RE, dHr, dHi, Q.npad, Q.kpad, Y,
                                g_status, g_stream));
  if ((st = record(2))) return st;
  for (int pass = 0; pass < 2; ++pass) {
    GemmArgs ga{};
    ga.X = X;
    ga.Y = Y + (pass ? (size_t)Q.ys * Q.kblocks * 1024 : 0);
    ga.mt = Q.mt; ga.nt = Q.nt; ga.kblocks = Q.kblocks; ga.ksplit = Q.ksplit;
    ga.SAp = Q.SAp; ga.SBp = Q.SBp; ga.Dmax = Q.Dmax; ga.form = FSEP;
    ga.digits = pass ? static_cast<void*>(dig2) : static_cast<void*>(base + Q.off_dig);
    ga.top = pass ? top2 : reinterpret_cast<int64_t*>(base + Q.off_top);
    ga.lnz = pass ? lnz2 : reinterpret_cast<int32_t*>(base + Q.off_lnz);
    ga.xs = Q.xs; ga.ys = Q.ys; ga.xlo = Q.xlo; ga.ylo = Q.ylo;
    HIP_TRY(launch_gemm_i8(ga, Q.block, g_stream));
  }
  if ((st = record(3))) return st;
  RoundArgs ra{};
  ra.digits = merged;
  ra.digit_bytes = 1;
  ra.nchunk = nchunk_m;
  ra.f64_layout = 0;
  ra.top = pm.top[0];
  ra.lnz = reinterpret_cast<const int32_t*>(base + Q.off_lnz);
  ra.ksplit = 1; ra.mt = Q.mt; ra.nt = Q.nt; ra.Dmax = Q.Dmax; ra.w = Q.w;
  ra.G = dGr; ra.H = dHr; ra.m = m; ra.n = n; ra.prec = prec_bits; ra.L = L;
  ra.cre = cre; ra.cim = cim; ra.ldc = ldc; ra.status = g_status;
  ra.acc = 0;
  ra.parts = dpm;
  HIP_TRY(launch_round(ra, g_stream));
  if ((st = record(4))) return st;
  if (info) {
    info->S_A = Q.SA; info->S_B = Q.SB; info->w = Q.w; info->cutoff = Q.cutoff;
    info->nprod = 4; info->ksplit = Q.ksplit; info->block = Q.block;
    info->pairs = Q.pairs; info->algo_ops = 2.0 * m * (double)n * k * (double)Q.pairs * 4; info->bound_bits = 0;
    info->part_scales = 1;
  }
  g_timing_valid = g_timing;
  return MPCG_OK;
}

// Device memory of a call that must not allocate: the status word and one
// region that holds the exponent scan and then the workspace.
struct FixedBuffers {
  int* status;
  char* base;
  size_t bytes;
};

int run(int m, int n, int k, const mpcg_cmat* A, int lda, const mpcg_cmat* B, int ldb, mpcg_cmat* C, int ldc,
        int prec_bits, int mode, int scheme, const mpcg_options* opt, mpcg_info* info, int acc = 0,
        bool check_overlap = true, const FixedBuffers* fixed = nullptr) {
  g_err.clear();
  int st = validate(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, opt, check_overlap);
  if (st) return st;
  if (acc != 0 && acc != 1 && acc != -1) return set_err(MPCG_EINVAL, "accumulate sign must be +1 or -1");
  if (acc && opt && opt->slice_type == MPCG_SLICE_FP64)
    return set_err(MPCG_EUNSUPPORTED, "the accumulating form needs INT8 slices");
  if (info) memset(info, 0, sizeof(*info));
  if (fixed && opt && opt->slice_type == MPCG_SLICE_FP64)
    return set_err(MPCG_EUNSUPPORTED, "FP64 slices run their products through rocBLAS, which allocates");
  if (fixed && opt && opt->adaptive && opt->max_spread <= 0)
    return set_err(MPCG_EUNSUPPORTED, "adaptive slicing runs a batch, which this entry point cannot");
  if (m == 0 || n == 0) return MPCG_OK;
  std::unique_lock<std::mutex> lock(g_mu);
  g_timing_valid = false;
  const int L = (prec_bits + 63) / 64;
  const DOutPart cre = doutpart(C->re, (int64_t)ldc * n), cim = doutpart(C->im, (int64_t)ldc * n);
  if (!fixed && (st = ensure_status_and_pinned())) return st;
  int* const status = fixed ? fixed->status : g_status;
  // stage events need event objects: no timing without allocation
  auto stage = [&](int idx) { return fixed ? (int)MPCG_OK : record(idx); };
  if (k == 0) {  // empty contraction: AB = 0
    if (!acc) HIP_TRY(launch_zero(cre, cim, m, n, ldc, L, g_stream));
    return MPCG_OK;
  }

  // ---- exponent scan and plan ----------------------------------------------
  DOperand opA{dpart(A->re, (int64_t)lda * k), dpart(A->im, (int64_t)lda * k), m, k, 1, lda};
  DOperand opB{dpart(B->re, (int64_t)ldb * n), dpart(B->im, (int64_t)ldb * n), n, k, ldb, 1};
  Plan P{};
  P.m = m; P.n = n; P.k = k; P.p = prec_bits;
  P.mode_req = mode;
  P.mode3m = mode != MPCG_4M;  // MPCG_AUTO is resolved once the spreads are known
  P.trunc = scheme == MPCG_TRUNCATED;
  P.f64 = opt && opt->slice_type == MPCG_SLICE_FP64;
  P.want_groups = 512;
  P.allow_bsplit = 1;
  P.allow_onepass = 1;
  const int bound = opt ? opt->max_spread : 0;
  tune_env_load();
  const size_t sA = align256(sizeof(RowStat) * (size_t)m), sB = align256(sizeof(RowStat) * (size_t)n);
  void* ws = nullptr;
  RowStat *statA, *statB;
  if (bound > 0) {
    // planned from the caller's bound: no read-back, the scan lives in the workspace
    P.mode3m = resolve_mode(mode, scheme, m, n, k, prec_bits, bound, bound) == MPCG_3M;
    P.tune_S = mode == MPCG_AUTO ? auto_key_S(prec_bits, bound, bound) : 0;
    if ((st = plan_slices(P, bound, bound, bound, bound, opt))) return st;
    if ((st = plan_layout(P, opt))) return st;
    if (fixed && P.onepass && P.total > fixed->bytes) {  // the real products together: a third of the streams
      P.allow_onepass = 0;
      if ((st = plan_layout(P, opt))) return st;
    }
    if (fixed) {
      if (P.total > fixed->bytes)
        return set_err(MPCG_ENOMEM, "this product needs %zu bytes of workspace; the fixed buffer holds %zu",
                       P.total, fixed->bytes);
      ws = fixed->base;
    } else if ((st = ensure_workspace(P.total, &ws))) {
      return st;
    }
    char* sc = static_cast<char*>(ws) + P.off_scan;
    statA = reinterpret_cast<RowStat*>(sc);
    statB = reinterpret_cast<RowStat*>(sc + sA);
    ScanSummary* summ = reinterpret_cast<ScanSummary*>(sc + sA + sB);
    if ((st = stage(0))) return st;
    HIP_TRY(launch_scan_pair(opA, statA, opB, statB, summ, bound, status, g_stream));
    if ((st = stage(1))) return st;
  } else {
    // the scan's statistics: library-owned, or at the start of the fixed
    // buffer (the workspace then follows them)
    const size_t scan_bytes = sA + sB + 256;
    char* scan_base;
    if (fixed) {
      if (scan_bytes > fixed->bytes)
        return set_err(MPCG_ENOMEM, "the exponent scan needs %zu bytes; the fixed buffer holds %zu", scan_bytes,
                       fixed->bytes);
      scan_base = fixed->base;
    } else {
      if ((st = ensure_scan(scan_bytes))) return st;
      scan_base = static_cast<char*>(g_scan);
    }
    statA = reinterpret_cast<RowStat*>(scan_base);
    statB = reinterpret_cast<RowStat*>(scan_base + sA);
    ScanSummary* summ = reinterpret_cast<ScanSummary*>(scan_base + sA + sB);
    ScanSummary local[2];  // pageable read-back for calls that allocate nothing
    ScanSummary* host_summ = fixed ? local : g_host_summary;
    if ((st = stage(0))) return st;
    HIP_TRY(launch_scan_pair(opA, statA, opB, statB, summ, 0, nullptr, g_stream));
    HIP_TRY(hipMemcpyAsync(host_summ, summ, 2 * sizeof(ScanSummary), hipMemcpyDeviceToHost, g_stream));
    if ((st = stage(1))) return st;
    HIP_TRY(hipStreamSynchronize(g_stream));
    const ScanSummary sa = host_summ[0], sb = host_summ[1];
    if ((sa.status | sb.status) & ST_IN_RANGE)
      return set_err(MPCG_ERANGE, "input exponent outside [-2^30, 2^30]");
    if (sa.nonzero == 0 || sb.nonzero == 0) {  // AB = 0
      if (!acc) HIP_TRY(launch_zero(cre, cim, m, n, ldc, L, g_stream));
      return MPCG_OK;
    }
    if (opt && opt->adaptive && !P.f64) {
      // per-block slice counts: the row and column statistics of the scan
      std::vector<RowStat> hA(m), hB(n);
      HIP_TRY(hipMemcpyAsync(hA.data(), statA, sizeof(RowStat) * m, hipMemcpyDeviceToHost, g_stream));
      HIP_TRY(hipMemcpyAsync(hB.data(), statB, sizeof(RowStat) * n, hipMemcpyDeviceToHost, g_stream));
      HIP_TRY(hipStreamSynchronize(g_stream));
      const int xb = P.mode3m ? 3 : 2;  // the INT8 headroom of plan_slices
      const int blk = opt->adaptive == 1 ? 256 : opt->adaptive;
      const std::vector<int> rb = adaptive_blocks(hA, prec_bits, xb, P.trunc, blk);
      const std::vector<int> cb = adaptive_blocks(hB, prec_bits, xb, P.trunc, blk);
      const int nrb = (int)rb.size() - 1, ncb = (int)cb.size() - 1;
      if (nrb * ncb > 1) {
        std::vector<mpcg_cmat> va(nrb), vb(ncb), vc((size_t)nrb * ncb);
        std::vector<mpcg_problem> probs((size_t)nrb * ncb);
        for (int i = 0; i < nrb; ++i) va[i] = view_at(*A, lda, k, rb[i], 0);
        for (int j = 0; j < ncb; ++j) vb[j] = view_at(*B, ldb, n, 0, cb[j]);
        for (int i = 0; i < nrb; ++i)
          for (int j = 0; j < ncb; ++j) {
            const size_t t = (size_t)i * ncb + j;
            vc[t] = view_at(*C, ldc, n, rb[i], cb[j]);
            probs[t] = mpcg_problem{rb[i + 1] - rb[i], cb[j + 1] - cb[j], k, &va[i], lda, &vb[j], ldb, &vc[t], ldc};
          }
        mpcg_options o = *opt;
        o.adaptive = 0;
        lock.unlock();
        return run_batched((int)probs.size(), probs.data(), prec_bits, mode, scheme, &o, info, acc, false, nullptr);
      }
    }
    P.mode3m = resolve_mode(mode, scheme, m, n, k, prec_bits, sa.spread, sb.spread) == MPCG_3M;
    P.tune_S = mode == MPCG_AUTO ? auto_key_S(prec_bits, sa.spread, sb.spread) : 0;
    if (opt && opt->part_scales && mode == MPCG_4M && !P.f64 && !acc && !P.trunc && !fixed) {
      // the one-scale plan's slice counts, to compare with
      Plan C0 = P;
      if ((st = plan_slices(C0, sa.spread, sb.spread, sa.hat, sb.hat, opt))) return st;
      st = run_parts(m, n, k, opA, opB, prec_bits, opt, info, C0.SA, C0.SB, cre, cim, ldc);
      if (st != PARTS_DECLINED) return st;
    }
    if (opt && opt->strassen && !P.f64 && !acc && !P.trunc && !fixed && m % 2 == 0 && n % 2 == 0 && k % 2 == 0) {
      st = run_strassen(m, n, k, opA, opB, prec_bits, P.mode3m, mode, opt, info, statA, statB, cre, cim, ldc);
      if (st != STRASSEN_DECLINED) return st;
    }
    if ((st = plan_slices(P, sa.spread, sb.spread, sa.hat, sb.hat, opt))) return st;
    if ((st = plan_layout(P, opt))) return st;
    if (fixed && P.onepass && P.total > fixed->bytes - align256(scan_bytes)) {  // as above
      P.allow_onepass = 0;
      if ((st = plan_layout(P, opt))) return st;
    }
    if (fixed) {
      const size_t off = align256(scan_bytes);
      if (P.total > fixed->bytes - off)
        return set_err(MPCG_ENOMEM, "this product needs %zu bytes of workspace; the fixed buffer holds %zu",
                       P.total + off, fixed->bytes);
      ws = fixed->base + off;
    } else if ((st = ensure_workspace(P.total, &ws))) {
      return st;
    }
  }
  if (info) {
    info->S_A = P.SA; info->S_B = P.SB; info->w = P.w; info->cutoff = P.cutoff;
    info->nprod = P.mode3m ? 3 : 4; info->ksplit = P.ksplit; info->block = P.block; info->apart = P.onepass;
    info->pairs = P.pairs; info->algo_ops = P.algo_ops; info->bound_bits = P.bound_bits;
  }
  char* base = static_cast<char*>(ws);
  int32_t* G = reinterpret_cast<int32_t*>(base + P.off_G);
  int32_t* H = reinterpret_cast<int32_t*>(base + P.off_H);

  // ---- split ---------------------------------------------------------------
  const Third thirdA = P.mode3m ? Third::SUM : Third::NONE;
  const Third thirdB = P.mode3m ? Third::SUM : (P.f64 ? Third::NONE : Third::NEG_IM);
  if (!P.f64) {
    // both operands in one launch, which also stores the row scales G and H
    SplitPair sp{};
    sp.a = opA; sp.b = opB; sp.sa = statA; sp.sb = statB; sp.G = G; sp.H = H;
    sp.X = reinterpret_cast<int8_t*>(base + P.off_X);
    sp.Y = reinterpret_cast<int8_t*>(base + P.off_Y);
    sp.SA = P.SA; sp.SAp = P.SAp; sp.xs = P.xs; sp.xlo = P.xlo; sp.mpad = P.mpad;
    sp.SB = P.SB; sp.SBp = P.SBp; sp.ys = P.ys; sp.ylo = P.ylo; sp.npad = P.npad;
    sp.Kpad = P.kpad; sp.x = P.x; sp.prec = prec_bits; sp.L = L; sp.status = status;
    HIP_TRY(launch_split_pair_i8(sp, P.mode3m, g_stream));
  } else {
    HIP_TRY(launch_scales(statA, m, P.mpad, P.x, G, g_stream));
    HIP_TRY(launch_scales(statB, n, P.npad, P.x, H, g_stream));
    HIP_TRY(launch_split_f64(opA, prec_bits, L, P.SA, P.SAp, P.w, thirdA, G, P.mpad, P.kpad,
                             reinterpret_cast<double*>(base + P.off_X), status, g_stream));
    HIP_TRY(launch_split_f64(opB, prec_bits, L, P.SB, P.SBp, P.w, thirdB, H, P.npad, P.kpad,
                             reinterpret_cast<double*>(base + P.off_Y), status, g_stream));
  }
  if ((st = stage(2))) return st;

  // ---- slice GEMM + carry chain -------------------------------------------
  int64_t* top = reinterpret_cast<int64_t*>(base + P.off_top);
  int32_t* lnz = reinterpret_cast<int32_t*>(base + P.off_lnz);
  if (!P.f64) {
    GemmArgs ga{};
    ga.X = reinterpret_cast<const int8_t*>(base + P.off_X);
    ga.Y = reinterpret_cast<const int8_t*>(base + P.off_Y);
    ga.mt = P.mt; ga.nt = P.nt; ga.kblocks = P.kblocks; ga.ksplit = P.ksplit; ga.bsplit = P.bsplit;
    ga.psplit = P.psplit;
    ga.SAp = P.SAp; ga.SBp = P.SBp; ga.Dmax = P.Dmax;
    ga.form = P.onepass ? (P.mode3m ? F3P : F4P) : (P.mode3m ? F3M : F4M);
    ga.digits = base + P.off_dig; ga.top = top; ga.lnz = lnz;
    ga.xs = P.xs; ga.ys = P.ys; ga.xlo = P.xlo; ga.ylo = P.ylo;
    HIP_TRY(launch_gemm_i8(ga, P.block, g_stream));
  } else if ((st = f64_products(P, base, L))) {
    return st;
  }
  if ((st = stage(3))) return st;

  // ---- merge chunks, round, store -------------------------------------------
  RoundArgs ra{};
  ra.digits = base + P.off_dig;
  ra.digit_bytes = P.f64 ? 4 : 1;
  ra.nchunk = P.nchunk;
  ra.f64_layout = P.f64;
  ra.top = top; ra.lnz = lnz;
  ra.ksplit = P.ksplit; ra.mt = P.mt; ra.nt = P.nt; ra.Dmax = P.Dmax; ra.w = P.w;
  if (P.onepass) {  // every stream holds all digits of what it touches: a plain sum
    ra.ksplit = P.ksplit * P.psplit;
    ra.onepass = P.psplit;
  }
  if (P.bsplit > 1) {
    ra.seg_bs = P.bsplit;
    ra.seg_ps = P.psplit;
    ra.seg_w = P.block;
    ra.seg_bpg = ceil_div((P.Dmax + P.block) / P.block, P.bsplit);
  }
  ra.G = G; ra.H = H; ra.m = m; ra.n = n; ra.prec = prec_bits; ra.L = L;
  ra.cre = cre; ra.cim = cim; ra.ldc = ldc; ra.status = status;
  ra.acc = acc;
  HIP_TRY(launch_round(ra, g_stream));
  if ((st = stage(4))) return st;
  g_timing_valid = g_timing && !fixed;
  return MPCG_OK;
}


// ---------------------------------------------------------------------------
// Batches of independent products.
// ---------------------------------------------------------------------------

// Host-built job tables, copied to the device in one transfer through a
// pinned staging buffer.  A later call waits for the previous transfer before
// it rewrites the staging buffer.
void* g_stage = nullptr;
size_t g_stage_bytes = 0;
hipEvent_t g_stage_ev = nullptr;
bool g_stage_pending = false;
void* g_tab = nullptr;
size_t g_tab_bytes = 0;
ScanSummary* g_bsum = nullptr;  // pinned read-back of a batch's summaries
size_t g_bsum_count = 0;
int g_num_cu = 0;

struct Tables {
  std::vector<char> bytes;
  // room for `count` entries of T (at least one), 256-byte aligned
  template <typename T>
  size_t reserve(size_t count) {
    const size_t off = align256(bytes.size());
    bytes.resize(off + std::max<size_t>(1, count) * sizeof(T));
    return off;
  }
  template <typename T>
  void put(size_t off, const std::vector<T>& v) {
    if (!v.empty()) memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
  }
  template <typename T>
  size_t add(const std::vector<T>& v) {
    const size_t off = reserve<T>(v.size());
    put(off, v);
    return off;
  }
};

// Copy the tables to the device (asynchronously on the library stream), to
// `dst` if given, else to the library's table buffer; returns the device
// base address.
int upload_tables(const Tables& t, char** dev, char* dst = nullptr) {
  const size_t n = align256(t.bytes.size());
  if (g_stage_pending) {
    HIP_TRY(hipEventSynchronize(g_stage_ev));
    g_stage_pending = false;
  }
  if (n > g_stage_bytes) {
    if (g_stage) HIP_TRY(hipHostFree(g_stage));
    g_stage = nullptr;
    g_stage_bytes = 0;
    HIP_TRY(hipHostMalloc(&g_stage, n, 0));
    g_stage_bytes = n;
  }
  if (!dst && n > g_tab_bytes) {
    if (g_tab) {
      HIP_TRY(hipStreamSynchronize(g_stream));
      HIP_TRY(hipFree(g_tab));
    }
    g_tab = nullptr;
    g_tab_bytes = 0;
    HIP_TRY(hipMalloc(&g_tab, n));
    g_tab_bytes = n;
  }
  if (!dst) dst = static_cast<char*>(g_tab);
  if (!g_stage_ev) HIP_TRY(hipEventCreateWithFlags(&g_stage_ev, hipEventDisableTiming));
  memcpy(g_stage, t.bytes.data(), t.bytes.size());
  HIP_TRY(hipMemcpyAsync(dst, g_stage, t.bytes.size(), hipMemcpyHostToDevice, g_stream));
  HIP_TRY(hipEventRecord(g_stage_ev, g_stream));
  g_stage_pending = true;
  *dev = dst;
  return MPCG_OK;
}

int num_cu() {
  if (!g_num_cu) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    if (g_num_cu <= 0) g_num_cu = 256;
  }
  return MPCG_OK;
}

// Ring steps of one (pass, k-block) pass over all bands of the INT8 slice
// GEMM (the same geometry as the kernel's units).
long long band_steps(int W, int SA, int SB, int Dmax) {
  const int NS = (W % 8 == 0) ? 4 : 2;  // steps per queue entry; units are whole entry pairs
  const int nbands = (Dmax + W) / W;
  long long total = 0;
  for (int b = 0; b < nbands; ++b) {
    const int d0 = Dmax + 1 - W * (b + 1);
    const int s_lo = std::max(0, d0 - (SB - 1)), s_hi = std::min(SA - 1, d0 + W - 1);
    // bands reaching s = 0 and t = 0 are walked downward without a ring fill
    const bool down = d0 <= SB - 1 && d0 + W - 1 <= SA - 1;
    // downward and s_lo > 0 units need no ring fill
    const int n = down ? s_hi + 1 : (s_lo > 0 ? s_hi - s_lo + 1 : s_hi - (s_lo - W) + 1);
    total += (long long)ceil_div(n, 2 * NS) * 2 * NS;
  }
  return total;
}

struct BatchProblem {
  int idx;  // index in the caller's array
  Plan P;
  DOperand opA, opB;
  DOutPart cre, cim;
  size_t ws_off;      // problem's region in the workspace
  size_t scan_off;    // its statistics in the scan area
  int spread[4];      // spreads the plan was made for (A, B, hat A, hat B)
};

// acc = 0: C_i := A_i B_i; +1 / -1: C_i := C_i +- A_i B_i in place, one rounding.
// size_query != NULL (bound-planned batches only): plan, store the workspace
// the batch needs in *size_query and return before any device work.
int run_batched(int count, const mpcg_problem* probs, int prec_bits, int mode, int scheme,
                const mpcg_options* opt, mpcg_info* info, int acc, bool check_overlap, size_t* size_query) {
  g_err.clear();
  if (count < 0) return set_err(MPCG_EINVAL, "negative batch count %d", count);
  if (acc != 0 && acc != 1 && acc != -1) return set_err(MPCG_EINVAL, "accumulate sign must be +1 or -1");
  if (count > 0 && !probs) return set_err(MPCG_EINVAL, "problems is NULL");
  if (opt && opt->slice_type == MPCG_SLICE_FP64)
    return set_err(MPCG_EUNSUPPORTED, "batched products use INT8 slices");
  if (info) memset(info, 0, sizeof(*info));
  std::vector<Region> outs;
  for (int i = 0; i < count; ++i) {
    const mpcg_problem& q = probs[i];
    int st = validate(q.m, q.n, q.k, q.A, q.lda, q.B, q.ldb, q.C, q.ldc, prec_bits, mode, scheme, opt,
                      check_overlap);
    if (st) {
      const std::string e = g_err;
      return set_err(st, "problem %d: %s", i, e.c_str());
    }
    if (q.m > 0 && q.n > 0 && check_overlap) {
      const int L = (prec_bits + 63) / 64;
      Region r[6];
      check_part(q.C->re, q.m, q.n, q.ldc, L, "C.re", r);
      check_part(q.C->im, q.m, q.n, q.ldc, L, "C.im", r + 3);
      for (auto& x : r) outs.push_back(x);
    }
  }
  // outputs of different problems must not overlap each other or any input
  for (size_t a = 0; a < outs.size(); ++a)
    for (size_t b = a + 1; b < outs.size(); ++b)
      if (a / 6 != b / 6 && overlap(outs[a], outs[b]))
        return set_err(MPCG_EINVAL, "outputs of problems %zu and %zu overlap", a / 6, b / 6);
  if (check_overlap) {
    const int L = (prec_bits + 63) / 64;
    for (int i = 0; i < count; ++i) {
      const mpcg_problem& q = probs[i];
      if (q.m == 0 || q.n == 0 || q.k == 0) continue;
      Region ra[12];
      check_part(q.A->re, q.m, q.k, q.lda, L, "A.re", ra);
      check_part(q.A->im, q.m, q.k, q.lda, L, "A.im", ra + 3);
      check_part(q.B->re, q.k, q.n, q.ldb, L, "B.re", ra + 6);
      check_part(q.B->im, q.k, q.n, q.ldb, L, "B.im", ra + 9);
      for (size_t a = 0; a < outs.size(); ++a)
        for (auto& x : ra)
          if (overlap(outs[a], x)) return set_err(MPCG_EINVAL, "an output overlaps problem %d's inputs", i);
    }
  }
  bool any = false;
  for (int i = 0; i < count; ++i) any |= probs[i].m > 0 && probs[i].n > 0;
  if (!any) return MPCG_OK;
  std::lock_guard<std::mutex> lock(g_mu);
  g_timing_valid = false;
  int st;
  const int bound = opt ? opt->max_spread : 0;
  bool capturing = false;
  if (size_query) {
    if (bound <= 0) return set_err(MPCG_EINVAL, "the batch workspace query needs max_spread > 0");
  } else {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(g_stream, &cap));
    capturing = cap != hipStreamCaptureStatusNone;
    if (capturing && (bound <= 0 || !g_user_ws || !g_status || !g_host_summary || !g_num_cu))
      return set_err(MPCG_EUNSUPPORTED,
                     "a batch captured into a graph needs max_spread > 0, a workspace set by mpcg_set_workspace "
                     "and one batched call made before the capture");
    if ((st = ensure_status_and_pinned())) return st;
  }
  if ((st = num_cu())) return st;
  tune_env_load();
  const int L = (prec_bits + 63) / 64;

  std::vector<BatchProblem> bp;
  size_t scan_total = 0;
  for (int i = 0; i < count; ++i) {
    const mpcg_problem& q = probs[i];
    if (q.m == 0 || q.n == 0) continue;
    const DOutPart cre = doutpart(q.C->re, (int64_t)q.ldc * q.n), cim = doutpart(q.C->im, (int64_t)q.ldc * q.n);
    if (q.k == 0) {  // A B = 0: C := 0, or C unchanged when accumulating
      if (!acc && !size_query) HIP_TRY(launch_zero(cre, cim, q.m, q.n, q.ldc, L, g_stream));
      continue;
    }
    BatchProblem b{};
    b.idx = i;
    b.opA = DOperand{dpart(q.A->re, (int64_t)q.lda * q.k), dpart(q.A->im, (int64_t)q.lda * q.k), q.m, q.k, 1, q.lda};
    b.opB = DOperand{dpart(q.B->re, (int64_t)q.ldb * q.n), dpart(q.B->im, (int64_t)q.ldb * q.n), q.n, q.k, q.ldb, 1};
    b.cre = cre;
    b.cim = cim;
    b.scan_off = scan_total;
    scan_total += scan_bytes(q.m, q.n);
    bp.push_back(b);
  }
  if (bp.empty()) {
    if (size_query) *size_query = 0;
    return MPCG_OK;
  }
  const int np = (int)bp.size();

  // ---- plans (from the bound, or after the scan read-back) ------------------
  auto make_plan = [&](BatchProblem& b, int spA, int spB, int hA, int hB, int want) -> int {
    Plan& P = b.P;
    P = Plan{};
    P.m = b.opA.R; P.n = b.opB.R; P.k = b.opA.K; P.p = prec_bits;
    P.mode_req = mode;
    P.mode3m = resolve_mode(mode, scheme, P.m, P.n, P.k, prec_bits, spA, spB) == MPCG_3M;
    P.tune_S = mode == MPCG_AUTO ? auto_key_S(prec_bits, spA, spB) : 0;
    P.trunc = scheme == MPCG_TRUNCATED;
    P.f64 = 0;
    P.want_groups = want;
    b.spread[0] = spA; b.spread[1] = spB; b.spread[2] = hA; b.spread[3] = hB;
    int r = plan_slices(P, spA, spB, hA, hB, opt);
    if (r) return r;
    mpcg_options o = opt ? *opt : mpcg_options{};
    if (!o.block_override) {
      // the band width from the size class (needs S, which plan_slices set):
      // the tuning cache's, else the fixed rule; the contraction chunks stay
      // the batch's (balanced over the compute units below)
      TuneChoice tc;
      o.block_override = (!g_tune_bypass &&
                          tune_find(tune_key(P.trunc, mode, P.m, P.n, P.k,
                                             P.tune_S ? P.tune_S : std::max(P.SA, P.SB)),
                                    &tc) &&
                          tc.mode3m == P.mode3m)
                             ? tc.band
                             : pick_band(P, BSPLIT_ITEMS);  // the rule for many work items: a batch is one launch
    }
    return plan_layout(P, &o);
  };

  // scan area: library-owned, or (with a bound) at the end of the workspace
  std::vector<ScanJob> sjA(np), sjB(np);
  std::vector<int> fiA(np + 1), fsA(np + 1), fiB(np + 1), fsB(np + 1);
  // scan area: per problem the row statistics of A and B, then all summaries
  // (A and B of problem t at 2t, 2t + 1) for one read-back
  const size_t summ_at = align256(scan_total);
  scan_total = summ_at + align256(2 * sizeof(ScanSummary) * (size_t)np);
  auto fill_scan_jobs = [&](char* scan_base) {
    int ia = 0, sa = 0, ib = 0, sb = 0;
    for (int t = 0; t < np; ++t) {
      BatchProblem& b = bp[t];
      char* sc = scan_base + b.scan_off;
      const size_t sA = align256(sizeof(RowStat) * (size_t)b.opA.R);
      ScanSummary* summ = reinterpret_cast<ScanSummary*>(scan_base + summ_at) + 2 * t;
      int i0, n0, kc, rb;
      sjA[t].op = b.opA; sjA[t].stats = reinterpret_cast<RowStat*>(sc); sjA[t].summary = summ;
      scan_blocks(b.opA, &i0, &n0, &kc, &rb);
      sjA[t].kchunk = kc; sjA[t].rblocks = rb;
      fiA[t] = ia; ia += i0; fsA[t] = sa; sa += n0;
      sjB[t].op = b.opB; sjB[t].stats = reinterpret_cast<RowStat*>(sc + sA); sjB[t].summary = summ + 1;
      scan_blocks(b.opB, &i0, &n0, &kc, &rb);
      sjB[t].kchunk = kc; sjB[t].rblocks = rb;
      fiB[t] = ib; ib += i0; fsB[t] = sb; sb += n0;
    }
    fiA[np] = ia; fsA[np] = sa; fiB[np] = ib; fsB[np] = sb;
  };
  Tables scanT;
  size_t o_sjA = 0, o_sjB = 0, o_fiA = 0, o_fsA = 0, o_fiB = 0, o_fsB = 0;
  auto add_scan_tables = [&](Tables& T) {
    o_sjA = T.add(sjA); o_sjB = T.add(sjB);
    o_fiA = T.add(fiA); o_fsA = T.add(fsA); o_fiB = T.add(fiB); o_fsB = T.add(fsB);
  };
  auto launch_scans = [&](char* dev, int* status_word, int limit) -> int {
    HIP_TRY(launch_scan_batched(reinterpret_cast<ScanJob*>(dev + o_sjA), np, reinterpret_cast<int*>(dev + o_fiA),
                                fiA[np], reinterpret_cast<int*>(dev + o_fsA), fsA[np], true, limit, status_word,
                                g_stream));
    HIP_TRY(launch_scan_batched(reinterpret_cast<ScanJob*>(dev + o_sjB), np, reinterpret_cast<int*>(dev + o_fiB),
                                fiB[np], reinterpret_cast<int*>(dev + o_fsB), fsB[np], false, limit, status_word,
                                g_stream));
    return MPCG_OK;
  };

  // A batch with few output tile groups splits the contraction of every
  // problem in proportion, so that each compute unit gets about two items.
  auto balance_chunks = [&]() -> int {
    long long total = 0;
    for (auto& b : bp) total += (long long)(b.P.mt / 2) * (b.P.nt / 2) * b.P.ksplit;
    if (total >= 2ll * g_num_cu || (opt && opt->ksplit_override)) return MPCG_OK;
    const int f = (int)((2ll * g_num_cu + total - 1) / total);
    for (auto& b : bp) {
      const int groups = (b.P.mt / 2) * (b.P.nt / 2);
      const int r = make_plan(b, b.spread[0], b.spread[1], b.spread[2], b.spread[3], groups * b.P.ksplit * f);
      if (r) return r;
    }
    return MPCG_OK;
  };

  void* ws = nullptr;
  size_t ws_total = 0;
  auto layout_workspace = [&]() {
    ws_total = 0;
    for (auto& b : bp) {
      b.ws_off = ws_total;
      ws_total += align256(b.P.total);
    }
  };
  char* scan_base = nullptr;
  if (bound > 0) {
    // the workspace (problems, scan area, job tables) is sized once the
    // tables are laid out, below
    for (auto& b : bp)
      if ((st = make_plan(b, bound, bound, bound, bound, 1))) return st;
    if ((st = balance_chunks())) return st;
    layout_workspace();
  } else {
    if ((st = ensure_scan(align256(scan_total) + 256))) return st;
    scan_base = static_cast<char*>(g_scan);
    fill_scan_jobs(scan_base);
    add_scan_tables(scanT);
    char* dev = nullptr;
    if ((st = upload_tables(scanT, &dev))) return st;
    if ((st = record(0))) return st;
    if ((st = launch_scans(dev, nullptr, 0))) return st;
    if ((size_t)(2 * np) > g_bsum_count) {
      if (g_bsum) HIP_TRY(hipHostFree(g_bsum));
      g_bsum = nullptr;
      g_bsum_count = 0;
      HIP_TRY(hipHostMalloc((void**)&g_bsum, 2 * np * sizeof(ScanSummary), 0));
      g_bsum_count = 2 * np;
    }
    HIP_TRY(hipMemcpyAsync(g_bsum, scan_base + summ_at, 2 * np * sizeof(ScanSummary), hipMemcpyDeviceToHost,
                           g_stream));
    if ((st = record(1))) return st;
    HIP_TRY(hipStreamSynchronize(g_stream));
    std::vector<BatchProblem> live;
    for (int t = 0; t < np; ++t) {
      const ScanSummary sa = g_bsum[2 * t], sb = g_bsum[2 * t + 1];
      if ((sa.status | sb.status) & ST_IN_RANGE)
        return set_err(MPCG_ERANGE, "problem %d: input exponent outside [-2^30, 2^30]", bp[t].idx);
      if (sa.nonzero == 0 || sb.nonzero == 0) {
        if (!acc)
          HIP_TRY(launch_zero(bp[t].cre, bp[t].cim, bp[t].opA.R, bp[t].opB.R, probs[bp[t].idx].ldc, L, g_stream));
        continue;
      }
      if ((st = make_plan(bp[t], sa.spread, sb.spread, sa.hat, sb.hat, 1))) return st;
      live.push_back(bp[t]);
    }
    bp.swap(live);
    if (bp.empty()) return MPCG_OK;
    if ((st = balance_chunks())) return st;
    layout_workspace();
    if ((st = ensure_workspace(ws_total, &ws))) return st;
  }
  const int nl = (int)bp.size();
  if (g_tune_keys)
    for (const auto& b : bp)
      g_tune_keys->push_back({tune_key(scheme, mode, b.P.m, b.P.n, b.P.k,
                                       b.P.tune_S ? b.P.tune_S : std::max(b.P.SA, b.P.SB)),
                              b.P.block});

  // ---- work items: every 2x2 tile group of every contraction chunk ----------
  // (groups of equal cost: the tile groups of one chunk of one problem)
  struct Group { long long cost; int band, m3, t, sp, gm, gn; };
  std::vector<Group> groups;
  for (int t = 0; t < nl; ++t) {
    const Plan& P = bp[t].P;
    const long long steps = band_steps(P.block, P.SAp, P.SBp, P.Dmax);
    const int kbps = ceil_div(P.kblocks, P.ksplit);
    const int passes = P.mode3m ? 3 : 2;
    const int gm = P.mt / 2, gn = P.nt / 2;
    for (int sp = 0; sp < P.ksplit; ++sp) {
      const int kb = std::min(P.kblocks, (sp + 1) * kbps) - sp * kbps;
      const long long cost = steps * passes * kb * (P.mode3m ? 1 : 2) * P.block + 64;
      groups.push_back(Group{cost, P.block, P.mode3m, t, sp, gm, gn});
    }
    if (info) {
      info->S_A = std::max(info->S_A, P.SA); info->S_B = std::max(info->S_B, P.SB); info->w = P.w;
      info->cutoff = std::max(info->cutoff, P.cutoff); info->nprod = P.mode3m ? 3 : 4;
      info->ksplit = std::max(info->ksplit, P.ksplit); info->block = std::max(info->block, P.block);
      info->pairs += P.pairs; info->algo_ops += P.algo_ops;
      info->bound_bits = P.bound_bits;
    }
  }
  // longest processing time first onto one workgroup per compute unit, per
  // class of band width and form (sorting the groups orders their items the
  // same way)
  std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) {
    if (a.band != b.band) return a.band > b.band;
    if (a.m3 != b.m3) return a.m3 > b.m3;
    return a.cost > b.cost;
  });
  struct Launch { int band, m3, blocks; size_t o_items, o_first; };
  std::vector<Launch> launches;
  std::vector<std::vector<int4>> litems;
  std::vector<std::vector<int>> lfirst;
  for (size_t a = 0; a < groups.size();) {
    size_t e = a;
    long long nitems = 0;
    while (e < groups.size() && groups[e].band == groups[a].band && groups[e].m3 == groups[a].m3) {
      nitems += (long long)groups[e].gm * groups[e].gn;
      ++e;
    }
    const int nbins = (int)std::max(1ll, std::min(nitems, (long long)g_num_cu));
    // each item goes to the least loaded bin (lowest index on ties): a binary
    // min-heap of (load, bin), whose top is replaced and sifted down once per
    // item (all loads 0 with ascending bins is already a heap)
    struct LB { long long load; int bin; };
    auto lt = [](const LB& x, const LB& y) { return x.load != y.load ? x.load < y.load : x.bin < y.bin; };
    std::vector<LB> heap(nbins);
    for (int i = 0; i < nbins; ++i) heap[i] = LB{0, i};
    std::vector<std::vector<int4>> bins(nbins);
    for (auto& v : bins) v.reserve((size_t)(nitems / nbins) + 8);
    for (size_t g = a; g < e; ++g) {
      const Group& gr = groups[g];
      for (int gj = 0; gj < gr.gn; ++gj)
        for (int gi = 0; gi < gr.gm; ++gi) {
          LB top = heap[0];
          bins[top.bin].push_back(make_int4(gr.t, gi, gj, gr.sp));
          top.load += gr.cost;
          int i = 0;
          for (;;) {
            int c = 2 * i + 1;
            if (c >= nbins) break;
            if (c + 1 < nbins && lt(heap[c + 1], heap[c])) ++c;
            if (!lt(heap[c], top)) break;
            heap[i] = heap[c];
            i = c;
          }
          heap[i] = top;
        }
    }
    // bins in XCD-major order: bin i -> block (i % per) * 8 + i / per, so that
    // equally loaded bins fill one XCD before the next
    const int per = ceil_div(nbins, 8);
    std::vector<int> block_of(nbins);
    {
      // block b is dispatched to XCD b % 8; give XCD x the bins [x*per, (x+1)*per)
      std::vector<int> used(nbins, 0);
      for (int i = 0; i < nbins; ++i) {
        int blk = (i % per) * 8 + i / per;
        if (blk >= nbins || used[blk]) {  // ragged tail: first free block
          blk = 0;
          while (used[blk]) ++blk;
        }
        used[blk] = 1;
        block_of[i] = blk;
      }
    }
    std::vector<std::vector<int4>> by_block(nbins);
    for (int i = 0; i < nbins; ++i) by_block[block_of[i]] = std::move(bins[i]);
    std::vector<int4> flat;
    std::vector<int> first(1, 0);
    for (int bk = 0; bk < nbins; ++bk) {
      flat.insert(flat.end(), by_block[bk].begin(), by_block[bk].end());
      first.push_back((int)flat.size());
    }
    launches.push_back(Launch{groups[a].band, groups[a].m3, nbins, 0, 0});
    litems.push_back(std::move(flat));
    lfirst.push_back(std::move(first));
    a = e;
  }

  // ---- job tables: layout, then the workspace, then their contents ----------
  Tables T;
  if (bound > 0) {
    o_sjA = T.reserve<ScanJob>(np); o_sjB = T.reserve<ScanJob>(np);
    o_fiA = T.reserve<int>(np + 1); o_fsA = T.reserve<int>(np + 1);
    o_fiB = T.reserve<int>(np + 1); o_fsB = T.reserve<int>(np + 1);
  }
  const size_t o_scj = T.reserve<ScaleJob>(2 * (size_t)nl), o_fsc = T.reserve<int>(2 * (size_t)nl + 1);
  const size_t o_spA = T.reserve<SplitJob>(nl), o_fspA = T.reserve<int>(nl + 1);
  const size_t o_spB = T.reserve<SplitJob>(nl), o_fspB = T.reserve<int>(nl + 1);
  const size_t o_ga = T.reserve<GemmArgs>(nl), o_ra = T.reserve<RoundArgs>(nl), o_frd = T.reserve<int>(nl + 1);
  for (size_t l = 0; l < launches.size(); ++l) {
    launches[l].o_items = T.reserve<int4>(litems[l].size());
    launches[l].o_first = T.reserve<int>(lfirst[l].size());
  }
  T.bytes.resize(align256(T.bytes.size()));
  char* tab_dev = nullptr;  // bound-planned batches keep their tables in the workspace
  if (bound > 0) {
    const size_t scan_at = ws_total, tab_at = ws_total + align256(scan_total);
    if (size_query) {
      *size_query = tab_at + T.bytes.size();
      return MPCG_OK;
    }
    if ((st = ensure_workspace(tab_at + T.bytes.size(), &ws))) return st;
    scan_base = static_cast<char*>(ws) + scan_at;
    tab_dev = static_cast<char*>(ws) + tab_at;
    fill_scan_jobs(scan_base);
    T.put(o_sjA, sjA); T.put(o_sjB, sjB);
    T.put(o_fiA, fiA); T.put(o_fsA, fsA); T.put(o_fiB, fiB); T.put(o_fsB, fsB);
  }
  char* base = static_cast<char*>(ws);
  std::vector<ScaleJob> scj;
  std::vector<int> fsc(1, 0);
  std::vector<SplitJob> spA, spB;
  std::vector<int> fspA(1, 0), fspB(1, 0);
  std::vector<GemmArgs> gargs(nl);
  std::vector<RoundArgs> rargs(nl);
  std::vector<int> frd(1, 0);
  for (int t = 0; t < nl; ++t) {
    BatchProblem& b = bp[t];
    const Plan& P = b.P;
    const Third thirdA = P.mode3m ? Third::SUM : Third::NONE;
    const Third thirdB = P.mode3m ? Third::SUM : Third::NEG_IM;
    char* pb = base + b.ws_off;
    int32_t* G = reinterpret_cast<int32_t*>(pb + P.off_G);
    int32_t* H = reinterpret_cast<int32_t*>(pb + P.off_H);
    char* sc = scan_base + b.scan_off;
    const size_t sA = align256(sizeof(RowStat) * (size_t)P.m);
    scj.push_back(ScaleJob{reinterpret_cast<RowStat*>(sc), P.m, P.mpad, P.x, G});
    fsc.push_back(fsc.back() + ceil_div(P.mpad, 256));
    scj.push_back(ScaleJob{reinterpret_cast<RowStat*>(sc + sA), P.n, P.npad, P.x, H});
    fsc.push_back(fsc.back() + ceil_div(P.npad, 256));
    spA.push_back(SplitJob{b.opA, P.SA, P.SAp, P.xs, P.xlo, (int)thirdA, P.mpad, P.kpad, G,
                           reinterpret_cast<int8_t*>(pb + P.off_X)});
    fspA.push_back(fspA.back() + (P.kpad / 64) * (P.mpad / 16));
    spB.push_back(SplitJob{b.opB, P.SB, P.SBp, P.ys, P.ylo, (int)thirdB, P.npad, P.kpad, H,
                           reinterpret_cast<int8_t*>(pb + P.off_Y)});
    fspB.push_back(fspB.back() + (P.kpad / 64) * (P.npad / 16));
    GemmArgs& ga = gargs[t];
    ga = GemmArgs{};
    ga.X = reinterpret_cast<const int8_t*>(pb + P.off_X);
    ga.Y = reinterpret_cast<const int8_t*>(pb + P.off_Y);
    ga.mt = P.mt; ga.nt = P.nt; ga.kblocks = P.kblocks; ga.ksplit = P.ksplit;
    ga.SAp = P.SAp; ga.SBp = P.SBp; ga.Dmax = P.Dmax; ga.form = P.mode3m ? F3M : F4M;
    ga.digits = pb + P.off_dig;
    ga.top = reinterpret_cast<int64_t*>(pb + P.off_top);
    ga.lnz = reinterpret_cast<int32_t*>(pb + P.off_lnz);
    ga.xs = P.xs; ga.ys = P.ys; ga.xlo = P.xlo; ga.ylo = P.ylo;
    RoundArgs& ra = rargs[t];
    ra = RoundArgs{};
    ra.digits = pb + P.off_dig;
    ra.digit_bytes = 1;
    ra.nchunk = P.nchunk;
    ra.f64_layout = 0;
    ra.top = ga.top; ra.lnz = ga.lnz;
    ra.ksplit = P.ksplit; ra.mt = P.mt; ra.nt = P.nt; ra.Dmax = P.Dmax; ra.w = P.w;
    ra.G = G; ra.H = H; ra.m = P.m; ra.n = P.n; ra.prec = prec_bits; ra.L = L;
    ra.cre = b.cre; ra.cim = b.cim; ra.ldc = probs[b.idx].ldc; ra.status = g_status;
    ra.acc = acc;
    frd.push_back(frd.back() + P.mt * P.nt * 2);
  }
  T.put(o_scj, scj); T.put(o_fsc, fsc);
  T.put(o_spA, spA); T.put(o_fspA, fspA); T.put(o_spB, spB); T.put(o_fspB, fspB);
  T.put(o_ga, gargs); T.put(o_ra, rargs); T.put(o_frd, frd);
  for (size_t l = 0; l < launches.size(); ++l) {
    T.put(launches[l].o_items, litems[l]);
    T.put(launches[l].o_first, lfirst[l]);
  }
  char* dev = nullptr;
  if (capturing) {
    // the data travels in kernel arguments, which the graph keeps
    HIP_TRY(launch_store_words(tab_dev, T.bytes.data(), T.bytes.size(), g_stream));
    dev = tab_dev;
  } else if ((st = upload_tables(T, &dev, tab_dev))) {
    return st;
  }
  if (bound > 0) {
    if ((st = record(0))) return st;
    // the scan's status bits go to the status word; spreads are checked against the bound
    if ((st = launch_scans(dev, g_status, bound))) return st;
    if ((st = record(1))) return st;
  }
  HIP_TRY(launch_scales_batched(reinterpret_cast<ScaleJob*>(dev + o_scj), (int)scj.size(),
                                reinterpret_cast<int*>(dev + o_fsc), fsc.back(), g_stream));
  HIP_TRY(launch_split_i8_batched_pair(reinterpret_cast<SplitJob*>(dev + o_spA), reinterpret_cast<int*>(dev + o_fspA),
                                       fspA.back(), reinterpret_cast<SplitJob*>(dev + o_spB),
                                       reinterpret_cast<int*>(dev + o_fspB), fspB.back(), nl, prec_bits, L, g_status,
                                       g_stream));
  if ((st = record(2))) return st;
  for (const Launch& l : launches)
    HIP_TRY(launch_gemm_i8_batched(reinterpret_cast<GemmArgs*>(dev + o_ga), reinterpret_cast<int4*>(dev + l.o_items),
                                   reinterpret_cast<int*>(dev + l.o_first), l.blocks, l.band, l.m3,
                                   g_stream));
  if ((st = record(3))) return st;
  HIP_TRY(launch_round_batched(reinterpret_cast<RoundArgs*>(dev + o_ra), nl, reinterpret_cast<int*>(dev + o_frd),
                               frd.back(), L, acc, g_stream));
  if ((st = record(4))) return st;
  g_timing_valid = g_timing;
  return MPCG_OK;
}


// ---------------------------------------------------------------------------
// Blocked complex LU with partial pivoting (Sec. IV-B) and the solve with its
// factors.  Every product, update and reciprocal step is a call of `run` on
// views into the caller's matrix; the small kernels of lu.hip pick pivots,
// exchange rows, copy and seed.
// ---------------------------------------------------------------------------
std::mutex g_lu_mu;

// The view whose entry (0, 0) is entry (r, c) of M (leading dimension ld,
// `cols` columns); the limb stride is the whole matrix's.
mpcg_cmat view_at(const mpcg_cmat& M, int ld, int cols, int r, int c) {
  const int64_t o = (int64_t)c * ld + r;
  mpcg_cmat v{};
  for (int h = 0; h < 2; ++h) {
    const mpcg_part& s = h ? M.im : M.re;
    mpcg_part& d = h ? v.im : v.re;
    d.sign = s.sign + o;
    d.exp = s.exp + o;
    d.mant = s.mant + o;
    d.limb_stride = s.limb_stride ? s.limb_stride : (int64_t)ld * cols;
  }
  return v;
}

// Scratch of one factorization or solve: NCOL columns of R entries (R >= the
// longest column or row handled), plus the singularity word.
struct LuScratch {
  static constexpr int NCOL = 5;
  enum { ABS = 0, KEY, TMP, OMI, REC };
  void* buf = nullptr;
  mpcg_cmat M{};
  int R = 0;
  int* info = nullptr;
  mpcg_cmat at(int col, int row = 0) const { return view_at(M, R, NCOL, row, col); }
  ~LuScratch() {
    if (buf) {
      (void)hipStreamSynchronize(g_stream);
      (void)hipFree(buf);
    }
  }
};

int lu_scratch(LuScratch& W, int R, int L) {
  W.R = std::max(1, R);
  const size_t ne = (size_t)W.R * LuScratch::NCOL;
  const size_t part = align256(ne) + align256(4 * ne) + align256(8 * ne * L);
  HIP_TRY(hipMalloc(&W.buf, 2 * part + 256));
  char* b = static_cast<char*>(W.buf);
  for (int h = 0; h < 2; ++h) {
    mpcg_part& d = h ? W.M.im : W.M.re;
    char* q = b + h * part;
    d.sign = reinterpret_cast<uint8_t*>(q);
    d.exp = reinterpret_cast<int32_t*>(q + align256(ne));
    d.mant = reinterpret_cast<uint64_t*>(q + align256(ne) + align256(4 * ne));
    d.limb_stride = (int64_t)ne;
  }
  W.info = reinterpret_cast<int*>(b + 2 * part);
  HIP_TRY(launch_fill_zero(W.info, 256, g_stream));
  const mpcg_cmat omi = W.at(LuScratch::OMI);
  HIP_TRY(launch_lu_const(doutpart(omi.re, 0), doutpart(omi.im, 0), L, 1, -1, g_stream));
  return MPCG_OK;
}

// One rounded product or update of the factorization (exact scheme).
int lu_prod(int m, int n, int k, const mpcg_cmat& A, int lda, const mpcg_cmat& B, int ldb, mpcg_cmat C, int ldc,
            int prec, int mode, int acc) {
  return run(m, n, k, &A, lda, &B, ldb, &C, ldc, prec, mode, MPCG_EXACT, nullptr, nullptr, acc, false);
}

// W[REC .. REC + count) := the reciprocals of `count` entries of y, entry t
// at t * stride, each component correctly rounded (one kernel launch).  A
// zero entry gives zero.
int lu_recip(LuScratch& W, const mpcg_cmat& y, int64_t stride, int count, int prec) {
  const int L = (prec + 63) / 64;
  const mpcg_cmat rec = W.at(LuScratch::REC);
  HIP_TRY(launch_lu_recip(dpart(y.re, 0), dpart(y.im, 0), stride, doutpart(rec.re, 0), doutpart(rec.im, 0), prec, L,
                          count, g_stream));
  return MPCG_OK;
}

int check_square(int n, const mpcg_cmat* A, int lda, int prec_bits, int mode, Region out[6]) {
  if (n < 0) return set_err(MPCG_EINVAL, "negative dimension n=%d", n);
  if (prec_bits < MPCG_MIN_PREC || prec_bits > MPCG_MAX_PREC)
    return set_err(MPCG_EINVAL, "prec_bits %d outside [%d, %d]", prec_bits, MPCG_MIN_PREC, MPCG_MAX_PREC);
  if (mode != MPCG_4M && mode != MPCG_3M && mode != MPCG_AUTO) return set_err(MPCG_EINVAL, "bad mode %d", mode);
  if (lda < std::max(1, n)) return set_err(MPCG_EINVAL, "lda %d < max(1, n=%d)", lda, n);
  if (!A) return set_err(MPCG_EINVAL, "A is NULL");
  const int L = (prec_bits + 63) / 64;
  int st;
  if ((st = check_part(A->re, n, n, lda, L, "A.re", out))) return st;
  if ((st = check_part(A->im, n, n, lda, L, "A.im", out + 3))) return st;
  for (int a = 0; a < 6; ++a)
    for (int b = a + 1; b < 6; ++b)
      if (overlap(out[a], out[b])) return set_err(MPCG_EINVAL, "the arrays of A overlap each other");
  return MPCG_OK;
}

int lu_factor(int n, mpcg_cmat* A, int lda, int* ipiv, int nb, int prec, int mode) {
  g_err.clear();
  Region ra[6];
  int st = check_square(n, A, lda, prec, mode, ra);
  if (st) return st;
  if (nb < 0) return set_err(MPCG_EINVAL, "negative block width %d", nb);
  if (n == 0) return MPCG_OK;
  if (!ipiv) return set_err(MPCG_EINVAL, "ipiv is NULL");
  const Region rp{(uintptr_t)ipiv, (uintptr_t)ipiv + 4 * (uintptr_t)n};
  for (auto& r : ra)
    if (overlap(r, rp)) return set_err(MPCG_EINVAL, "ipiv overlaps A");
  if (nb == 0) nb = 64;
  std::lock_guard<std::mutex> lock(g_lu_mu);
  if ((st = ensure_status_and_pinned())) return st;
  const int L = (prec + 63) / 64;
  LuScratch W;
  if ((st = lu_scratch(W, n, L))) return st;
  const mpcg_cmat& M = *A;
  auto at = [&](int r, int c) { return view_at(M, lda, n, r, c); };
  const DOutPart are = doutpart(M.re, (int64_t)lda * n), aim = doutpart(M.im, (int64_t)lda * n);
  const mpcg_cmat T = W.at(LuScratch::ABS), K = W.at(LuScratch::KEY), tmp = W.at(LuScratch::TMP);
  for (int j = 0; j < n; j += nb) {
    const int jb = std::min(nb, n - j);
    for (int c = j; c < j + jb; ++c) {
      const int mr = n - c;  // rows c .. n-1 of column c
      const mpcg_cmat col = at(c, c);
      // pivot: the first row of the largest RNE(|Re| + |Im|) = Re((|Re| + i|Im|)(1 - i))
      HIP_TRY(launch_lu_copy(dpart(col.re, 0), dpart(col.im, 0), lda, doutpart(T.re, 0), doutpart(T.im, 0), W.R, mr,
                             1, L, 2, g_stream));
      if ((st = lu_prod(mr, 1, 1, T, W.R, W.at(LuScratch::OMI), 1, K, W.R, prec, mode, 0))) return st;
      HIP_TRY(launch_lu_pivot(dpart(K.re, 0), mr, L, c, ipiv + c, W.info, c, g_stream));
      HIP_TRY(launch_lu_swap(are, aim, lda, n, L, c, ipiv + c, g_stream));
      if ((st = lu_recip(W, col, 1, 1, prec))) return st;
      if (mr > 1) {
        // l := a r below the pivot, through the scratch column
        if ((st = lu_prod(mr - 1, 1, 1, at(c + 1, c), lda, W.at(LuScratch::REC), 1, tmp, W.R, prec, mode, 0)))
          return st;
        const mpcg_cmat dst = at(c + 1, c);
        HIP_TRY(launch_lu_copy(dpart(tmp.re, 0), dpart(tmp.im, 0), W.R, doutpart(dst.re, 0), doutpart(dst.im, 0), lda,
                               mr - 1, 1, L, 0, g_stream));
        // rank-1 update of the rest of the panel
        if (c + 1 < j + jb &&
            (st = lu_prod(mr - 1, j + jb - c - 1, 1, at(c + 1, c), lda, at(c, c + 1), lda, at(c + 1, c + 1), lda,
                          prec, mode, -1)))
          return st;
      }
    }
    const int nr = n - j - jb;
    if (nr > 0) {
      // U12 := L11^-1 A12 (unit lower, column by column of L11)
      for (int c = j; c + 1 < j + jb; ++c)
        if ((st = lu_prod(j + jb - c - 1, nr, 1, at(c + 1, c), lda, at(c, j + jb), lda, at(c + 1, j + jb), lda, prec,
                          mode, -1)))
          return st;
      // A22 := A22 - L21 U12, one rounding per entry
      if ((st = lu_prod(nr, nr, jb, at(j + jb, j), lda, at(j, j + jb), lda, at(j + jb, j + jb), lda, prec, mode, -1)))
        return st;
    }
  }
  int info = 0;
  HIP_TRY(hipMemcpyAsync(&info, W.info, sizeof(int), hipMemcpyDeviceToHost, g_stream));
  HIP_TRY(hipStreamSynchronize(g_stream));
  return info;
}

int lu_solve(int n, int nrhs, const mpcg_cmat* A, int lda, const int* ipiv, mpcg_cmat* B, int ldb, int prec,
             int mode) {
  g_err.clear();
  Region ra[6], rb[6];
  int st = check_square(n, A, lda, prec, mode, ra);
  if (st) return st;
  if (nrhs < 0) return set_err(MPCG_EINVAL, "negative nrhs %d", nrhs);
  if (ldb < std::max(1, n)) return set_err(MPCG_EINVAL, "ldb %d < max(1, n=%d)", ldb, n);
  if (n == 0 || nrhs == 0) return MPCG_OK;
  if (!ipiv || !B) return set_err(MPCG_EINVAL, "ipiv or B is NULL");
  const int L = (prec + 63) / 64;
  if ((st = check_part(B->re, n, nrhs, ldb, L, "B.re", rb))) return st;
  if ((st = check_part(B->im, n, nrhs, ldb, L, "B.im", rb + 3))) return st;
  const Region rp{(uintptr_t)ipiv, (uintptr_t)ipiv + 4 * (uintptr_t)n};
  for (int a = 0; a < 6; ++a) {
    if (overlap(rb[a], rp)) return set_err(MPCG_EINVAL, "ipiv overlaps B");
    for (int b = 0; b < 6; ++b)
      if ((b > a && overlap(rb[a], rb[b])) || overlap(rb[a], ra[b]))
        return set_err(MPCG_EINVAL, "B overlaps A or itself");
  }
  std::lock_guard<std::mutex> lock(g_lu_mu);
  if ((st = ensure_status_and_pinned())) return st;
  LuScratch W;
  if ((st = lu_scratch(W, std::max(n, nrhs), L))) return st;
  auto a_at = [&](int r, int c) { return view_at(*A, lda, n, r, c); };
  auto b_at = [&](int r, int c) { return view_at(*B, ldb, nrhs, r, c); };
  // the reciprocals of U's diagonal, all at once (entry c at c (lda + 1))
  if ((st = lu_recip(W, a_at(0, 0), (int64_t)lda + 1, n, prec))) return st;
  HIP_TRY(launch_lu_laswp(doutpart(B->re, (int64_t)ldb * nrhs), doutpart(B->im, (int64_t)ldb * nrhs), ldb, nrhs, n,
                          L, ipiv, g_stream));
  // forward: row c of Y := RNE(B_c - L(c, 0:c) Y(0:c, :)), unit diagonal
  for (int c = 1; c < n; ++c)
    if ((st = lu_prod(1, nrhs, c, a_at(c, 0), lda, b_at(0, 0), ldb, b_at(c, 0), ldb, prec, mode, -1))) return st;
  // backward: row c of X := RNE(RNE(Y_c - U(c, c+1:n) X(c+1:n, :)) * recip(U(c, c)))
  const mpcg_cmat tmp = W.at(LuScratch::TMP);  // a 1 x nrhs row, leading dimension 1
  for (int c = n - 1; c >= 0; --c) {
    if (c + 1 < n &&
        (st = lu_prod(1, nrhs, n - c - 1, a_at(c, c + 1), lda, b_at(c + 1, 0), ldb, b_at(c, 0), ldb, prec, mode, -1)))
      return st;
    if ((st = lu_prod(1, nrhs, 1, W.at(LuScratch::REC, c), 1, b_at(c, 0), ldb, tmp, 1, prec, mode, 0))) return st;
    const mpcg_cmat dst = b_at(c, 0);
    HIP_TRY(launch_lu_copy(dpart(tmp.re, 0), dpart(tmp.im, 0), 1, doutpart(dst.re, 0), doutpart(dst.im, 0), ldb, 1,
                           nrhs, L, 0, g_stream));
  }
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

int mp_cgemm_ex_noalloc(int m, int n, int k, const mpcg_cmat* A, int lda, const mpcg_cmat* B, int ldb,
                        mpcg_cmat* C, int ldc, int prec_bits, int mode, int scheme, const mpcg_options* opt,
                        mpcg_info* info) {
  g_err.clear();
  int st = validate(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, opt);
  if (st) return st;
  if (m == 0 || n == 0) {
    if (info) memset(info, 0, sizeof(*info));
    return MPCG_OK;
  }
  void* base = nullptr;
  size_t bytes = 0;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    HIP_TRY(noalloc_scratch(g_stream, &base, &bytes));
  }
  const FixedBuffers fb{static_cast<int*>(base), static_cast<char*>(base) + 256, bytes - 256};
  return run(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, opt, info, 0, true, &fb);
}

int mpcg_autotune(int m, int n, int k, const mpcg_cmat* A, int lda, const mpcg_cmat* B, int ldb, mpcg_cmat* C,
                  int ldc, int prec_bits, int mode, int scheme, int reps, mpcg_tune_report* report) {
  g_err.clear();
  int st = validate(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, nullptr);
  if (st) return st;
  if (report) memset(report, 0, sizeof(*report));
  if (m == 0 || n == 0 || k == 0) return set_err(MPCG_EINVAL, "nothing to tune for an empty product");
  reps = std::max(1, reps);
  {
    std::lock_guard<std::mutex> lock(g_mu);
    tune_env_load();
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  HIP_TRY(hipEventCreate(&ev[0]));
  hipError_t e = hipEventCreate(&ev[1]);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return set_err(MPCG_EHIP, "hipEventCreate failed: %s", hipGetErrorString(e));
  }
  struct Cand { int mode, band, groups; };
  std::vector<Cand> cands;
  const int forms[2] = {MPCG_3M, MPCG_4M};
  for (int f = 0; f < 2; ++f) {
    const int fm = forms[f];
    if (mode != MPCG_AUTO && fm != mode) continue;
    for (int band : {8, 12, 16, 20}) {
      if (fm == MPCG_4M && band > 16) continue;  // two rings per diagonal: 16 is the widest that fits registers
      for (int groups : {256, 512, 1024, 2048}) cands.push_back(Cand{fm, band, groups});
    }
  }
  // time `reps` calls of one plan (after one untimed call); -1 if it fails
  auto time_plan = [&](int fm, int band, int groups, mpcg_info* info) -> float {
    mpcg_options o{MPCG_SLICE_INT8, 0, 0, band, 0, 0};
    g_tune_forced_groups = groups;
    g_tune_bypass = true;
    int r = run(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, fm, scheme, band ? &o : nullptr, info);
    float ms = -1.f;
    if (!r && hipEventRecord(ev[0], g_stream) == hipSuccess) {
      for (int i = 0; i < reps && !r; ++i) r = run(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, fm, scheme,
                                                 band ? &o : nullptr, nullptr);
      if (!r && hipEventRecord(ev[1], g_stream) == hipSuccess && hipEventSynchronize(ev[1]) == hipSuccess &&
          hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess)
        ms /= reps;
      else
        ms = -1.f;
    }
    g_tune_forced_groups = 0;
    g_tune_bypass = false;
    return ms;
  };
  // the fixed rule's plan (3M unless 4M was asked for), which also gives S
  mpcg_info info{};
  const int base_mode = mode == MPCG_4M ? MPCG_4M : MPCG_3M;
  const float base_ms = time_plan(base_mode, 0, 512, &info);
  if (base_ms < 0) {
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return g_err.empty() ? set_err(MPCG_EHIP, "timing the untuned plan failed") : MPCG_EHIP;
  }
  float best_ms = base_ms;
  Cand best{base_mode, info.block, 512};
  int tried = 0;
  for (const Cand& c : cands) {
    const float ms = time_plan(c.mode, c.band, c.groups, nullptr);
    if (ms < 0) continue;  // a plan the limits reject (int32 headroom), or a failed call
    ++tried;
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  g_err.clear();
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  const int S = std::max(info.S_A, info.S_B);  // of the 3M plan for MPCG_AUTO and 3M requests
  tune_put(tune_key(scheme, mode, m, n, k, S), TuneChoice{best.band, best.groups, best.mode == MPCG_3M ? 1 : 0,
                                                          1000.f * best_ms});
  if (report) {
    report->band = best.band;
    report->groups = best.groups;
    report->mode = best.mode;
    report->S = S;
    report->candidates = tried;
    report->us = 1000.f * best_ms;
    report->untuned_us = 1000.f * base_ms;
  }
  return MPCG_OK;
}

int mpcg_autotune_batched(int count, const mpcg_problem* problems, int prec_bits, int mode, int scheme, int reps,
                          const mpcg_options* opt, mpcg_tune_report* report) {
  g_err.clear();
  if (report) memset(report, 0, sizeof(*report));
  if (mode != MPCG_4M && mode != MPCG_3M && mode != MPCG_AUTO) return set_err(MPCG_EINVAL, "bad mode %d", mode);
  if (opt && (opt->block_override || opt->slice_type != MPCG_SLICE_INT8 || opt->adaptive))
    return set_err(MPCG_EINVAL, "tuning a batch measures band widths itself (INT8 slices, no block or adaptive option)");
  reps = std::max(1, reps);
  {
    std::lock_guard<std::mutex> lock(g_mu);
    tune_env_load();
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  HIP_TRY(hipEventCreate(&ev[0]));
  hipError_t e = hipEventCreate(&ev[1]);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return set_err(MPCG_EHIP, "hipEventCreate failed: %s", hipGetErrorString(e));
  }
  std::vector<std::pair<TuneKey, int>> keys;
  auto time_batch = [&](int fm, int band, bool record_keys) -> float {
    mpcg_options o = opt ? *opt : mpcg_options{};
    o.block_override = band;
    g_tune_bypass = true;
    g_tune_keys = record_keys ? &keys : nullptr;
    int r = run_batched(count, problems, prec_bits, fm, scheme, &o, nullptr, 0, true);
    g_tune_keys = nullptr;
    float ms = -1.f;
    if (!r && hipEventRecord(ev[0], g_stream) == hipSuccess) {
      for (int i = 0; i < reps && !r; ++i) r = run_batched(count, problems, prec_bits, fm, scheme, &o, nullptr, 0, true);
      if (!r && hipEventRecord(ev[1], g_stream) == hipSuccess && hipEventSynchronize(ev[1]) == hipSuccess &&
          hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess)
        ms /= reps;
      else
        ms = -1.f;
    }
    g_tune_bypass = false;
    return ms;
  };
  // the fixed rule: 3M (unless 4M was asked for) with each problem's own band
  const int base_mode = mode == MPCG_4M ? MPCG_4M : MPCG_3M;
  const float base_ms = time_batch(base_mode, 0, true);
  if (base_ms < 0) {
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return g_err.empty() ? set_err(MPCG_EHIP, "timing the untuned batch failed") : MPCG_EHIP;
  }
  float best_ms = base_ms;
  int best_mode = -1, best_band = 0, tried = 0;  // -1: keep the fixed rule
  for (int fm : {MPCG_3M, MPCG_4M}) {
    if (mode != MPCG_AUTO && fm != mode) continue;
    for (int band : {8, 12, 16, 20}) {
      if (fm == MPCG_4M && band > 16) continue;
      const float ms = time_batch(fm, band, false);
      if (ms < 0) continue;
      ++tried;
      if (ms < best_ms) {
        best_ms = ms;
        best_mode = fm;
        best_band = band;
      }
    }
  }
  g_err.clear();
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  // every size class of the batch takes the winner: a uniform plan, or each
  // problem's own band in the base form.  Keyed by the requested form (the
  // classes were recorded by the base run, whose 3M or 4M slice counts are
  // the ones such requests are keyed by).
  for (auto kb : keys) {
    TuneKey k = kb.first;
    k.mode = mode;
    const int fm = best_mode >= 0 ? best_mode : base_mode;
    tune_put(k, TuneChoice{best_mode >= 0 ? best_band : kb.second, 512, fm == MPCG_3M ? 1 : 0, 1000.f * best_ms});
  }
  if (report) {
    report->band = best_mode >= 0 ? best_band : 0;
    report->groups = 512;
    report->mode = best_mode >= 0 ? best_mode : base_mode;
    report->S = 0;
    report->candidates = tried;
    report->us = 1000.f * best_ms;
    report->untuned_us = 1000.f * base_ms;
  }
  return MPCG_OK;
}

int mpcg_tune_load(const char* path) {
  g_err.clear();
  if (!path) path = getenv("MPCG_TUNE_CACHE");
  if (!path || !*path) return set_err(MPCG_EINVAL, "no tuning cache path (argument NULL and MPCG_TUNE_CACHE unset)");
  std::lock_guard<std::mutex> lock(g_mu);
  g_tune_env_done = true;
  const int r = tune_load(path);
  if (r < 0) return set_err(MPCG_EINVAL, "cannot read tuning cache %s (missing or malformed)", path);
  return r;
}

int mpcg_tune_save(const char* path) {
  g_err.clear();
  if (!path) path = getenv("MPCG_TUNE_CACHE");
  if (!path || !*path) return set_err(MPCG_EINVAL, "no tuning cache path (argument NULL and MPCG_TUNE_CACHE unset)");
  std::lock_guard<std::mutex> lock(g_mu);
  const int r = tune_save(path);
  if (r < 0) return set_err(MPCG_EINVAL, "cannot write tuning cache %s", path);
  return r;
}

int mpcg_tune_clear(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  tune_clear();
  g_tune_env_done = true;  // an explicit clear also stops the environment's cache from loading later
  return MPCG_OK;
}

int mp_cgemm_acc(int m, int n, int k, const mpcg_cmat* A, int lda, const mpcg_cmat* B, int ldb, mpcg_cmat* C,
                 int ldc, int prec_bits, int mode, int scheme, int sign, const mpcg_options* opt, mpcg_info* info) {
  if (sign != 1 && sign != -1) {
    g_err.clear();
    return set_err(MPCG_EINVAL, "accumulate sign must be +1 or -1");
  }
  return run(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, opt, info, sign);
}

int mp_cgemm_batched(int count, const mpcg_problem* problems, int prec_bits, int mode, int scheme,
                     const mpcg_options* opt, mpcg_info* info) {
  return run_batched(count, problems, prec_bits, mode, scheme, opt, info, 0, true);
}

size_t mpcg_workspace_size_batched(int count, const mpcg_problem* problems, int prec_bits, int mode, int scheme,
                                   const mpcg_options* opt) {
  size_t bytes = 0;
  if (run_batched(count, problems, prec_bits, mode, scheme, opt, nullptr, 0, true, &bytes)) return 0;
  return bytes;
}

int mp_cgemm_batched_acc(int count, const mpcg_problem* problems, int prec_bits, int mode, int scheme, int sign,
                         const mpcg_options* opt, mpcg_info* info) {
  if (sign != 1 && sign != -1) {
    g_err.clear();
    return set_err(MPCG_EINVAL, "accumulate sign must be +1 or -1");
  }
  return run_batched(count, problems, prec_bits, mode, scheme, opt, info, sign, true);
}

int mp_zgetrf(int n, mpcg_cmat* A, int lda, int* ipiv, int nb, int prec_bits, int mode) {
  return lu_factor(n, A, lda, ipiv, nb, prec_bits, mode);
}

int mp_zgetrs(int n, int nrhs, const mpcg_cmat* A, int lda, const int* ipiv, mpcg_cmat* B, int ldb, int prec_bits,
              int mode) {
  return lu_solve(n, nrhs, A, lda, ipiv, B, ldb, prec_bits, mode);
}

int mpcg_set_stream(void* hip_stream) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_stream = static_cast<hipStream_t>(hip_stream);
  return MPCG_OK;
}

int mpcg_set_workspace(void* dev_ptr, size_t bytes) {
  std::lock_guard<std::mutex> lock(g_mu);
  if ((dev_ptr == nullptr) != (bytes == 0)) return set_err(MPCG_EINVAL, "workspace pointer and size disagree");
  if (dev_ptr) {
    // allocate the status word now, so that later calls planned from a spread
    // bound allocate nothing
    const int st = ensure_status_and_pinned();
    if (st) return st;
  }
  g_user_ws = dev_ptr;
  g_user_ws_bytes = bytes;
  return MPCG_OK;
}

size_t mpcg_workspace_size(int m, int n, int k, int prec_bits, int mode, int scheme, const mpcg_options* opt,
                           int max_spread) {
  if (m <= 0 || n <= 0 || k <= 0 || prec_bits < MPCG_MIN_PREC || prec_bits > MPCG_MAX_PREC || max_spread < 0)
    return 0;
  if (mode != MPCG_4M && mode != MPCG_3M && mode != MPCG_AUTO) return 0;
  tune_env_load();  // the same plan as the call's, tuned size classes included
  Plan P{};
  P.m = m; P.n = n; P.k = k; P.p = prec_bits;
  P.mode_req = mode;
  P.mode3m = resolve_mode(mode, scheme, m, n, k, prec_bits, max_spread, max_spread) == MPCG_3M;
  P.tune_S = mode == MPCG_AUTO ? auto_key_S(prec_bits, max_spread, max_spread) : 0;
  P.trunc = scheme == MPCG_TRUNCATED;
  P.f64 = opt && opt->slice_type == MPCG_SLICE_FP64;
  P.want_groups = 512;
  P.allow_bsplit = 1;  // as the call plans it
  P.allow_onepass = 1;
  if (plan_slices(P, max_spread, max_spread, max_spread, max_spread, opt)) return 0;
  if (plan_layout(P, opt)) return 0;
  return P.total;
}

int mpcg_stream_status(void* hip_stream) {
  std::lock_guard<std::mutex> lock(g_mu);
  int* const fixed_status = noalloc_status_word();
  if (!g_status && !fixed_status) return MPCG_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  HIP_TRY(hipStreamSynchronize(s));
  int v = 0;
  for (int* word : {g_status, fixed_status}) {
    if (!word) continue;
    int w = 0;
    HIP_TRY(hipMemcpy(&w, word, sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(word, 0, sizeof(int)));
    v |= w;
  }
  if (v & ST_SPREAD) return set_err(MPCG_ESPREAD, "an operand's exponent spread exceeded max_spread");
  if (v & ST_IN_RANGE) return set_err(MPCG_ERANGE, "input exponent outside [-2^30, 2^30]");
  if (v & ST_OUT_RANGE) return set_err(MPCG_ERANGE, "output exponent outside int32 (or a double component beyond the largest double)");
  if (v & ST_DENORM) return set_err(MPCG_EDOMAIN, "nonzero input with clear significand top bit");
  if (v & ST_NONFINITE) return set_err(MPCG_EDOMAIN, "infinite or NaN double input");
  return MPCG_OK;
}

int mpcg_from_doubles(int rows, int cols, int ncomp, const double* src, int ld, long long plane, mpcg_part* dst,
                      int ldd, int prec_bits) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_err.clear();
  if (rows < 0 || cols < 0) return set_err(MPCG_EINVAL, "negative dimension");
  if (ncomp < 1 || ncomp > 4) return set_err(MPCG_EINVAL, "ncomp %d outside [1, 4]", ncomp);
  if (prec_bits < MPCG_MIN_PREC || prec_bits > MPCG_MAX_PREC)
    return set_err(MPCG_EINVAL, "prec_bits %d outside [%d, %d]", prec_bits, MPCG_MIN_PREC, MPCG_MAX_PREC);
  if (ld < std::max(1, rows) || ldd < std::max(1, rows)) return set_err(MPCG_EINVAL, "leading dimension < rows");
  if (!src || !dst) return set_err(MPCG_EINVAL, "NULL pointer");
  const int64_t n = (int64_t)ld * cols;
  const int64_t pl = plane ? (int64_t)plane : n;
  if (ncomp > 1 && pl < n) return set_err(MPCG_EINVAL, "plane stride %lld < ld*cols %lld", plane, (long long)n);
  const int L = (prec_bits + 63) / 64;
  Region rd[3];
  int st = check_part(*dst, rows, cols, ldd, L, "dst", rd);
  if (st) return st;
  const Region rs{(uintptr_t)src, (uintptr_t)src + (uintptr_t)(8 * (pl * (ncomp - 1) + n))};
  for (int a = 0; a < 3; ++a)
    if (overlap(rd[a], rs)) return set_err(MPCG_EINVAL, "dst overlaps the source doubles");
  if (rows == 0 || cols == 0) return MPCG_OK;
  if ((st = ensure_status_and_pinned())) return st;
  // the codec's pass flag lives in the status allocation, 64 bytes after the status word
  HIP_TRY(launch_from_doubles(src, rows, cols, ncomp, ld, pl, doutpart(*dst, (int64_t)ldd * cols), ldd, prec_bits, L,
                              g_status, g_status + 16, g_stream));
  return MPCG_OK;
}

int mpcg_to_doubles(int rows, int cols, const mpcg_part* src, int lds, int prec_bits, int ncomp, double* dst, int ld,
                    long long plane) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_err.clear();
  if (rows < 0 || cols < 0) return set_err(MPCG_EINVAL, "negative dimension");
  if (ncomp < 1 || ncomp > 4) return set_err(MPCG_EINVAL, "ncomp %d outside [1, 4]", ncomp);
  if (prec_bits < MPCG_MIN_PREC || prec_bits > MPCG_MAX_PREC)
    return set_err(MPCG_EINVAL, "prec_bits %d outside [%d, %d]", prec_bits, MPCG_MIN_PREC, MPCG_MAX_PREC);
  if (ld < std::max(1, rows) || lds < std::max(1, rows)) return set_err(MPCG_EINVAL, "leading dimension < rows");
  if (!src || !dst) return set_err(MPCG_EINVAL, "NULL pointer");
  const int64_t n = (int64_t)ld * cols;
  const int64_t pl = plane ? (int64_t)plane : n;
  if (ncomp > 1 && pl < n) return set_err(MPCG_EINVAL, "plane stride %lld < ld*cols %lld", plane, (long long)n);
  const int L = (prec_bits + 63) / 64;
  Region rs[3];
  int st = check_part(*src, rows, cols, lds, L, "src", rs);
  if (st) return st;
  const Region rd{(uintptr_t)dst, (uintptr_t)dst + (uintptr_t)(8 * (pl * (ncomp - 1) + n))};
  for (int a = 0; a < 3; ++a)
    if (overlap(rs[a], rd)) return set_err(MPCG_EINVAL, "the doubles overlap the source");
  if (rows == 0 || cols == 0) return MPCG_OK;
  if ((st = ensure_status_and_pinned())) return st;
  HIP_TRY(launch_to_doubles(dpart(*src, (int64_t)lds * cols), rows, cols, lds, prec_bits, L, ncomp, dst, ld, pl,
                            g_status, g_stream));
  return MPCG_OK;
}

const char* mpcg_last_error(void) { return g_err.c_str(); }

int mpcg_probe_mfma(int kind, int blocks, int iters, void* sink, double* ops, float* ms) {
  g_err.clear();
  if (kind != 0 && kind != 1) return set_err(MPCG_EINVAL, "probe kind must be 0 (INT8) or 1 (FP64)");
  if (blocks < 1 || blocks > (1 << 20)) return set_err(MPCG_EINVAL, "probe blocks must be in [1, 2^20]");
  if (iters < 1 || iters > (1 << 24)) return set_err(MPCG_EINVAL, "probe iterations must be in [1, 2^24]");
  if (!sink || !ops || !ms) return set_err(MPCG_EINVAL, "NULL pointer");
  std::lock_guard<std::mutex> lock(g_mu);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_err(MPCG_EHIP, "probe: hipEventCreate failed");
  }
  hipError_t e = hipEventRecord(e0, g_stream);
  if (e == hipSuccess) e = launch_mfma_probe(kind, blocks, iters, static_cast<int*>(sink), g_stream);
  if (e == hipSuccess) e = hipEventRecord(e1, g_stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return set_err(MPCG_EHIP, "probe: %s", hipGetErrorString(e));
  *ms = t;
  *ops = (double)blocks * 4.0 * (double)iters * 8.0 * (kind == 0 ? 32768.0 : 2048.0);
  return MPCG_OK;
}

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
