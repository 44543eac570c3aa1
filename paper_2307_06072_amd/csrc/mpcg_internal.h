// Internal declarations shared by the host planner and the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpcg {

constexpr int32_t EXP_ZERO = INT32_MIN;
// Bits per digit of the INT8 slices: balanced base-2^8 digits in [-128, 127],
// the full range of an int8 matrix-core operand.
constexpr int I8_W = 8;
constexpr int32_t EXP_LIMIT = 1 << 30;  // |exp| of a nonzero input

// Device status bits (OR-ed into a word in the workspace).
constexpr int ST_IN_RANGE = 1;   // input exponent outside [-2^30, 2^30]
constexpr int ST_DENORM = 2;     // nonzero input with clear top significand bit
constexpr int ST_OUT_RANGE = 4;  // output exponent does not fit int32
constexpr int ST_SPREAD = 8;     // exponent spread beyond the caller's bound (planning without read-back)
constexpr int ST_NONFINITE = 16;  // infinite or NaN double given to the multi-component codec

// One real component of a column-major matrix (read side).
struct DPart {
  const uint8_t* sign;
  const int32_t* exp;
  const uint64_t* mant;
  int64_t ls;  // limb stride (elements)
};

// One real component (write side).
struct DOutPart {
  uint8_t* sign;
  int32_t* exp;
  uint64_t* mant;
  int64_t ls;
};

// A real component viewed as an R x K operand: element (r, kk) at r*rs + kk*ks.
// For A (m x k, column-major) R = m, rs = 1, ks = lda; for B (k x n) R = n,
// rs = ldb, ks = 1 (B is read transposed, one "row" per output column).
struct DOperand {
  DPart re, im;
  int R, K;
  int64_t rs, ks;
};

// Per-row (A) or per-column (B) exponent statistics, filled by the scan.
struct RowStat {
  int32_t emax;   // largest exponent of any nonzero Re/Im component (INT32_MIN: all zero)
  int32_t emin;   // smallest such exponent
  int32_t ehat;   // min over the row of max(e_re, e_im) of nonzero entries
  int32_t pad;
};

// Whole-operand summary (device side, read back once by the host).
struct ScanSummary {
  int32_t spread;     // max over nonzero rows of emax - emin
  int32_t hat;        // max over nonzero rows of emax - ehat
  int32_t nonzero;    // number of rows with a nonzero entry
  int32_t status;     // ST_* bits from the scan
};

// ----------------------------------------------------------------------------
// Launchers (all asynchronous on `stream`).
// ----------------------------------------------------------------------------

// Exponent scan of one operand: stats[R], summary.  `stats` and `summary` are
// initialised by the launcher's own fill kernel.  With status_word != NULL the
// summary's status bits, and ST_SPREAD if the spread exceeds `limit`, are also
// OR-ed into *status_word (for calls that do not read the summary back).
hipError_t launch_scan(const DOperand& op, RowStat* stats, ScanSummary* summary, int limit, int* status_word,
                       hipStream_t stream);
// Both operands' scans (summary[0] for A, summary[1] for B), in one launch when both are small.
hipError_t launch_scan_pair(const DOperand& a, RowStat* sa, const DOperand& b, RowStat* sb, ScanSummary* summary,
                            int limit, int* status_word, hipStream_t stream);

// Digit planes of one operand.
//   nops       planes per slice index: 2 (Re, Im), 3 (Re, Im, Re+Im) or
//              3 with the third plane = -Im (neg_im_plane).
//   S          digits needed for exactness (frame size); Sp >= S planes are written
//              (planes s >= S are zero).
//   w          digit width in bits.
//   G          per-row scale exponents (int32 [Rpad]); digits represent
//              |x| / 2^G[r] = sum_s d_s 2^(-w(s+1)).
//   out        INT8: int8 planes [nops][Sp][Rpad/16][Kpad/64][64][16];
//              FP64: one column-major matrix of nops Sp Rpad rows (row
//              (o Sp + s) Rpad + r) and Kpad columns.
enum class Third { NONE = 0, SUM = 1, NEG_IM = 2, RE = 3 };
// INT8 planes hold Sstride slices each: pad_lo zero slices, the Sp digit
// slices, then zero slices up to Sstride (all written by the split); with
// Sstride = pad_lo + Sp the planes share their pads, and the last row tile's
// blocks also zero the pad_lo slices after its last plane (the region holds
// them).
hipError_t launch_split_i8(const DOperand& op, int prec, int L, int S, int Sp, int Sstride, int pad_lo,
                           Third third, const int32_t* G, int Rpad, int Kpad, int8_t* out, int* status,
                           hipStream_t stream);
// The split of op + sign2 * op2 (sign2 = +1 or -1; the same shape and
// strides), each entry's exact sum digitized with the row scales G, which must
// leave room for the sum (one more bit than either operand).
hipError_t launch_split2_i8(const DOperand& op, const DOperand& op2, int sign2, int prec, int L, int S, int Sp,
                            int Sstride, int pad_lo, Third third, const int32_t* G, int Rpad, int Kpad, int8_t* out,
                            int* status, hipStream_t stream);
// The split with separate row scales for the Re parts (G) and the Im parts
// (Gim); third NONE or RE (the Re plane again, as the third plane).
hipError_t launch_split_parts_i8(const DOperand& op, int prec, int L, int S, int Sp, int Sstride, int pad_lo,
                                 Third third, const int32_t* G, const int32_t* Gim, int Rpad, int Kpad, int8_t* out,
                                 int* status, hipStream_t stream);
hipError_t launch_split_f64(const DOperand& op, int prec, int L, int S, int Sp, int w, Third third,
                            const int32_t* G, int Rpad, int Kpad, double* out, int* status,
                            hipStream_t stream);

// Scales of the rows r < half of a one-level Strassen split: G[r] = max(emax
// of rows r and r + half) + x (0 where both are zero), G[r] = 0 up to Rpad.
hipError_t launch_fold_scales(const RowStat* stats, int half, int Rpad, int x, int32_t* G, hipStream_t stream);
// Scale exponents G[r] = emax + x (0 for all-zero rows), r < Rpad.
hipError_t launch_scales(const RowStat* stats, int R, int Rpad, int x, int32_t* G, hipStream_t stream);

// Slice GEMM + combination + carry chain (INT8 digits).
enum GemmForm { F4M = 0, F3M = 1, FSEP = 2, F3P = 3, F4P = 4 };
struct GemmArgs {
  const int8_t* X;   // A-side planes
  const int8_t* Y;   // B-side planes
  int mt, nt;        // 16-row tiles of A, 16-column tiles of B
  int kblocks;       // Kpad / 64 (INT8) or Kpad / 4 (FP64)
  int ksplit;        // contraction chunks
  int bsplit;        // > 1: the bands run in bsplit groups of ceil(bands / bsplit) consecutive
                     // bands on separate workgroups, one digit stream each, which holds the
                     // group's own digits only (zero to whole 16-digit chunks around them;
                     // other chunks unwritten) and leaves its carry into the next group's
                     // digits in `top`
  int psplit;        // > 1 (with bsplit > 1; 3M: 3, 4M: 2): each real product (pass) of a band
                     // group on a workgroup of its own, a stream each; stream
                     // (chunk c, group g, pass p) is (c bsplit + g) psplit + p.  Forms F3P
                     // and F4P (bsplit = 1): 3 or 4, stream c psplit + p
  int SAp, SBp;      // slice counts of the A and B operands
  int xs, ys;        // slices per A / B plane including the zero pads
  int xlo, ylo;      // zero slices below slice 0 of an A / B plane
  int Dmax;          // highest emitted diagonal
  int form;          // F4M: A planes (Re, Im), B (Re, Im, -Im), Re and Im of C out;
                     // F3M: planes (Re, Im, Re+Im) on both sides, Re and Im of C out;
                     // FSEP: A planes (X0, X1), B (Y0, Y1, ...), the two real products
                     //       X0 Y0 and X1 Y1 out in place of Re and Im;
                     // F3P: the planes of F3M, one real product per work item (psplit = 3,
                     //       bsplit = 1), its share of Re and Im out;
                     // F4P: the planes of F4M, one real product per work item (psplit = 4,
                     //       bsplit = 1: Re A Re B and Im A (-Im B) into Re, Re A Im B
                     //       and Im A Re B into Im), that component out
  void* digits;      // [ksplit][tiles][slot 8][chunk][lane 64][16] uint8 digits, q = Dmax - d
                     // (chunk = q / 16; gemm_i8_digit_chunks chunks per component)
  int64_t* top;      // [ksplit][tiles][64][8]
  int32_t* lnz;      // [ksplit][tiles][64][8]
};
// Zero slices the INT8 slice GEMM of band width `band` needs below (lo) and
// above (hi) the digits of the A and B planes.
void gemm_i8_pads(int band, int* alo, int* ahi, int* blo, int* bhi);
// 16-digit chunks per output component of the INT8 slice GEMM.
int gemm_i8_digit_chunks(int Dmax, int band);
hipError_t launch_gemm_i8(const GemmArgs& a, int band, hipStream_t stream);

// The FP64 form: the slice-plane products are DGEMMs (rocBLAS) of stacked
// column-major slice planes; these kernels accumulate them exactly.
// C[q]: the products of the block s0 .. s1 - 1 of A's slices with B's slices
// t = 0 .. tcnt - 1, row (s - s0) mpad + i, column t npad + j, leading
// dimension ldc: 4M (Re Re, Im Im, Re Im, Im Re), 3M (Re Re, Im Im,
// (Re+Im)(Re+Im)).  acc: int64 [2][Dmax + 1][n][m] diagonal sums of Re and Im.
struct F64AccArgs {
  const double* C[4];
  int64_t ldc;
  int s0, s1, tcnt, mpad, npad, m, n, Dmax, mode3m;
  int64_t* acc;
};
hipError_t launch_f64_accumulate(const F64AccArgs& a, hipStream_t stream);
// acc into the rounding kernel's FP64-order digit streams, tops and lowest
// nonzero digits (one contraction chunk).
struct F64CarryArgs {
  const int64_t* acc;
  int m, n, mt, nt, Dmax, w;
  uint32_t* digits;
  int64_t* top;
  int32_t* lnz;
};
hipError_t launch_f64_carry(const F64CarryArgs& a, hipStream_t stream);

// Merge chunk streams (if ksplit > 1), round to prec, write C.
constexpr int MAX_MERGE = 48;
struct MergeSrc {       // one signed digit stream of a merge
  const uint8_t* dig;   // one contraction chunk's digits, laid out like `digits`
  const int64_t* top;   // its tops
  int64_t sign;         // +1 or -1
};
struct RoundArgs {
  const void* digits;  // uint8 (w = 8, INT8 chunked layout) or uint32 (FP64 form) digits
  int digit_bytes;     // 1 or 4
  int nchunk;          // INT8: 16-digit chunks per component
  int f64_layout;      // 1: element (i, j) of a 16x16 tile sits in lane j + 16*(i%4), slot i/4
                       //    (fp64 matrix-core output order); 0: lane j + 16*(i/4), slot i%4
  const int64_t* top;
  const int32_t* lnz;
  int ksplit, mt, nt, Dmax, w;
  // 3 (4): the ksplit streams are (chunk, real product) pairs, stream q of
  // product q % 3 (q % 4); a 3M T3 stream (q % 3 == 2) holds no Re digits, a
  // 4M stream only Re (q % 4 < 2) or only Im digits (the others unwritten;
  // the tops of all are written)
  int onepass;
  // > 1: the streams are band groups (GemmArgs.bsplit, .psplit): stream
  // (chunk c, group g, pass p) = (c seg_bs + g) seg_ps + p holds group g's
  // digits, its top the carry into digit seg_w min(nbands, (g + 1) seg_bpg)
  int seg_bs, seg_ps, seg_w, seg_bpg;
  const int32_t* G;  // [m]
  const int32_t* H;  // [n]
  int m, n, prec, L;
  DOutPart cre, cim;
  int64_t ldc;
  int* status;
  int acc;  // 0: C := AB; +1 / -1: C := C + AB / C - AB (INT8 layout only), rounded once
  // INT8 only, nsrc > 0: the exact integer to round is the signed sum of the
  // nsrc (<= MAX_MERGE) streams of the device table src for Re and the
  // nsrc_im of src + MAX_MERGE for Im, formed into `digits` (ksplit must be
  // 1): the recombination of Strassen's products
  int nsrc, nsrc_im;
  const MergeSrc* src;
  // INT8 only, non-null: the four real products of separately scaled parts
  // (device pointer), merged into `digits` (nchunk chunks per component;
  // Dmax is the products' own)
  const struct PartsMerge* parts;
};
hipError_t launch_round(const RoundArgs& a, hipStream_t stream);
// Matrix-core rate probe: kind 0 INT8 16x16x64, 1 FP64 16x16x4; 256-thread blocks.
hipError_t launch_mfma_probe(int kind, int blocks, int iters, int* sink, hipStream_t stream);

// Separately scaled Re and Im parts (4M): the real products P_rr = Re A Re B,
// P_ii = Im A Im B, P_ri = Re A Im B and P_ir = Im A Re B are exact digit
// streams of one layout, each at the scale of its own parts, and
// Re C = P_rr - P_ii, Im C = P_ri + P_ir.  The scales of the two parts of a
// row (column) agree modulo 8, so the streams of one component are merged
// shifted by whole digits.
struct PartsMerge {
  const uint8_t* dig[2];  // streams of the pair (P_rr, P_ii) and (P_ri, P_ir): the first in the
                          // Re slots, the second in the Im slots of a GEMM digit layout
  const int64_t* top[2];  // their tops
  int nchunk;             // 16-digit chunks per component of those layouts
  int ksplit;             // contraction chunks of those layouts
  const int32_t* Gre;     // [m] row scales of Re A
  const int32_t* Gim;     // [m] row scales of Im A
  const int32_t* Hre;     // [n] column scales of Re B
  const int32_t* Him;     // [n] column scales of Im B
  char pad[256 - 2 * 8 - 2 * 8 - 2 * 4 - 4 * 8];  // a 256-byte record
};
static_assert(sizeof(PartsMerge) == 256, "PartsMerge is stored as 256 bytes");

// The fixed buffer of mp_cgemm_ex_noalloc on the current device (set up on
// first use: its device address looked up, its status word cleared on
// `stream`): *ptr, *bytes = MPCG_NOALLOC_BYTES.  The first 256 bytes hold the
// status word.
hipError_t noalloc_scratch(hipStream_t stream, void** ptr, size_t* bytes);
// That status word on the current device, or NULL if the buffer is not set up.
int* noalloc_status_word();

// dst[0, bytes) := src[0, bytes) by kernels that carry the data in their
// arguments (StoreWords::N words per launch): a captured graph replays its
// own copy, whatever becomes of src.
struct StoreWords {
  static constexpr uint32_t N = 760;
  uint32_t n;
  uint32_t v[N];
};
hipError_t launch_store_words(void* dst, const void* src, size_t bytes, hipStream_t stream);

// Size-class tuning cache (tune.cpp).
struct TuneKey {
  int scheme, mode;  // scheme, requested form (MPCG_4M, MPCG_3M or MPCG_AUTO)
  int lm, ln, lk;    // ceil(log2) of m, n, k
  int sb;            // ceil(S / 8), S the larger slice count of the two operands
};
struct TuneChoice {
  int band;    // INT8 slice GEMM band width
  int groups;  // work-item target that sets the contraction chunks
  int mode3m;  // the form chosen (for requests of MPCG_AUTO)
  float us;    // measured time of the class's tuning problem
};
bool operator<(const TuneKey& a, const TuneKey& b);
TuneKey tune_key(int scheme, int mode, int m, int n, int k, int S);
const char* tune_arch();
bool tune_find(const TuneKey& key, TuneChoice* out);
void tune_put(const TuneKey& key, const TuneChoice& c);
int tune_count();
void tune_clear();
int tune_load(const char* path);  // entries loaded, -1 on a read or parse error
int tune_save(const char* path);  // entries written, -1 on a write error

// bytes[0 .. n) := 0 (a kernel, so that the call stays capturable).
hipError_t launch_fill_zero(void* p, size_t n, hipStream_t stream);

// C := +0 everywhere.
hipError_t launch_zero(DOutPart cre, DOutPart cim, int m, int n, int64_t ldc, int L, hipStream_t stream);
// Blocked LU helpers (one stream-ordered launch each).
// copy: rows x cols block, mode 0 plain, 1 conjugate, 2 componentwise |.|.
hipError_t launch_lu_copy(DPart sre, DPart sim, int64_t lds, DOutPart dre, DOutPart dim, int64_t ldd, int rows,
                          int cols, int L, int mode, hipStream_t stream);
// *piv := base + first index of the largest of the m nonnegative keys; a
// zero maximum sets *info := col + 1 if *info is 0.
hipError_t launch_lu_pivot(DPart key, int m, int L, int base, int* piv, int* info, int col, hipStream_t stream);
// rows `row` and *piv exchanged over ncols columns.
hipError_t launch_lu_swap(DOutPart re, DOutPart im, int64_t ld, int ncols, int L, int row, const int* piv,
                          hipStream_t stream);
// interchanges ipiv[0..n) applied in order to an n x ncols block.
hipError_t launch_lu_laswp(DOutPart re, DOutPart im, int64_t ld, int ncols, int n, int L, const int* ipiv,
                           hipStream_t stream);
// entry 0 := vre + i vim, each in {-1, 0, 1}.
hipError_t launch_lu_const(DOutPart re, DOutPart im, int L, int vre, int vim, hipStream_t stream);
// entries 0 .. count-1 (consecutive) of (xre, xim) := the reciprocals of the
// entries t * stride of (yre, yim), each component rounded once to prec bits
// (nearest, ties to even); a zero entry gives zero.
hipError_t launch_lu_recip(DPart yre, DPart yim, int64_t stride, DOutPart xre, DOutPart xim, int prec, int L,
                           int count, hipStream_t stream);
hipError_t launch_to_doubles(DPart in, int rows, int cols, int64_t ldi, int prec, int L, int ncomp, double* dst,
                             int64_t ld, int64_t plane, int* status, hipStream_t stream);
hipError_t launch_from_doubles(const double* src, int rows, int cols, int ncomp, int64_t ld, int64_t plane,
                               DOutPart out, int64_t ldo, int prec, int L, int* status, int* pending,
                               hipStream_t stream);


// ----------------------------------------------------------------------------
// Batched launches.  Every stage of a batch of independent products is one
// launch: job j (an operand or a problem) owns the blocks
// [first[j], first[j+1]) of the grid, found by a binary search over `first`.
// The job tables live in device memory.
// ----------------------------------------------------------------------------
__device__ inline int job_of_block(const int* __restrict__ first, int njobs, int b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct ScanJob {
  DOperand op;
  RowStat* stats;
  ScanSummary* summary;
  int kchunk, rblocks;  // contraction chunk of one block, row blocks
};
// Block counts of the three scan launches for one operand (init, scan, summary).
void scan_blocks(const DOperand& op, int* init_blocks, int* scan_blocks, int* kchunk, int* rblocks);
// rows_contiguous: every job has rs == 1 (A operands); else ks == 1 (B operands).
hipError_t launch_scan_batched(const ScanJob* jobs, int njobs, const int* first_init, int init_blocks,
                               const int* first_scan, int scan_blocks_total, bool rows_contiguous, int limit,
                               int* status_word, hipStream_t stream);

struct ScaleJob {
  const RowStat* stats;
  int R, Rpad, x;
  int32_t* G;
};
hipError_t launch_scales_batched(const ScaleJob* jobs, int njobs, const int* first, int blocks, hipStream_t stream);

// Both operands of one product split in one launch (INT8): each row's scale
// is G = emax + x from the scan's statistics (0 for an empty or padding row),
// stored to G and H (Rpad entries) for the rounding by the blocks of the
// first contraction tile.
struct SplitPair {
  DOperand a, b;
  const RowStat *sa, *sb;
  int32_t *G, *H;
  int8_t *X, *Y;
  int SA, SAp, xs, xlo, mpad;
  int SB, SBp, ys, ylo, npad;
  int Kpad, x, prec, L;
  int* status;
};
// 3M: both third planes Re + Im; 4M: none for A, -Im for B.
hipError_t launch_split_pair_i8(const SplitPair& a, bool mode3m, hipStream_t stream);

struct SplitJob {
  DOperand op;
  int S, Sp, Sstride, pad_lo, third, Rpad, Kpad;
  const int32_t* G;
  int8_t* out;
};
// One block per 16 x 64 tile: job j has (Kpad/64) * (Rpad/16) blocks.

// Both sides of a batch in one launch: A's jobs (rows contiguous) in blocks
// [0, blocks_a), B's (contraction contiguous) after them; njobs jobs each.
hipError_t launch_split_i8_batched_pair(const SplitJob* ja, const int* fa, int blocks_a, const SplitJob* jb,
                                        const int* fb, int blocks_b, int njobs, int prec, int L, int* status,
                                        hipStream_t stream);

// Persistent slice GEMM: block b runs items[first[b] .. first[b+1]) in order;
// an item is (problem, tile-group row, tile-group column, contraction chunk).
hipError_t launch_gemm_i8_batched(const GemmArgs* probs, const int4* items, const int* first, int blocks,
                                  int band, int mode3m, hipStream_t stream);

// Round (INT8 digits): job j is problem j with 2 mt nt blocks (tile, component).
hipError_t launch_round_batched(const RoundArgs* jobs, int njobs, const int* first, int blocks, int L, int acc,
                                hipStream_t stream);

}  // namespace mpcg
