/*
 * mpcgemm.h - arbitrary-precision complex matrix multiplication C := A B on
 * AMD Instinct MI355X (gfx950) by the Ozaki scheme, 4M and 3M forms.
 *
 * The operation is eq. (1) of the paper (C := AB, A in C^{m x k}, B in
 * C^{k x n}), each entry being the sum of eq. (2) over complex products.
 * Each multi-precision matrix is split error-free into short signed-digit
 * slice matrices (the splitting idea of Algorithm 2), every slice-pair product
 * is formed exactly on the matrix cores, and the products are combined in an
 * exact multi-limb fixed-point accumulator (instead of the L-bit floating-point
 * accumulation of Algorithm 2) and rounded once to nearest-even.  The complex
 * product is assembled either from four real products (eq. 5, "4M") or from
 * three (eq. 6, "3M"); with exact slice products both give identical bits.
 *
 * NUMBER FORMAT (one real component of a matrix; column-major, leading
 * dimension ld >= rows):
 *   sign[c*ld + r]  uint8: 0 = +, 1 = -.
 *   exp [c*ld + r]  int32: value = (-1)^sign * M * 2^(exp - 64*L), where
 *                   L = ceil(prec_bits / 64) and M is the L-limb significand;
 *                   exp == MPCG_EXP_ZERO (INT32_MIN) marks an exact zero
 *                   (sign and limbs are then ignored).  Nonzero inputs need
 *                   |exp| <= 2^30.
 *   mant[l*limb_stride + c*ld + r]  uint64: limb l of M, limb 0 least
 *                   significant.  A nonzero entry has the top bit of limb L-1
 *                   set (significand in [1/2, 1), the MPFR convention of the
 *                   paper's F_bM, Section II).  Only the top prec_bits bits are
 *                   read; the lower bits of limb 0 are ignored on input and
 *                   written as zero on output.
 *   limb_stride >= (cols-1)*ld + rows (the entries addressed, so the limb
 *                   planes never share an entry); 0 means exactly ld*cols.
 *                   A strided view such as the diagonal of an n x n matrix
 *                   as a 1 x n row with ld = lda + 1 is therefore valid.
 * Outputs: each component of each entry of C is the exact value rounded to
 * prec_bits, round to nearest, ties to even.  An exact zero is written as
 * sign 0, exp MPCG_EXP_ZERO, limbs 0.
 *
 * MEMORY AND STREAMS: every matrix pointer is a DEVICE pointer owned by the
 * caller; the library never frees or retains it.  Work is issued on the
 * stream set by mpcg_set_stream (default: the null stream) and is
 * asynchronous, except that each multiplication synchronizes that stream once,
 * after its exponent scan, to size the slice planes (the number of slices
 * depends on the exponent spread of the data).  C must not overlap A or B.
 *
 * ERRORS: functions return MPCG_OK (0) or a negative code.  Argument errors
 * are detected on the host before any device work is issued.  The text of the
 * last error of the calling thread is returned by mpcg_last_error().
 *
 * THREADS AND DEVICES: the stream, the workspace (library-owned or set by
 * mpcg_set_workspace) and the host staging buffers are per process and shared
 * by all threads.  The library's own device buffers are allocated on the
 * device current at its first allocation, so every call must be made with
 * that device current (one GPU per process).  Calls from several threads are
 * safe: an internal lock serializes them (they do not issue work
 * concurrently), and a thread's mpcg_set_stream changes the stream for every
 * thread.  mp_zgetrf and mp_zgetrs hold a lock of their own for the whole
 * call (two of them never overlap); another thread's products may be issued
 * between their steps, on the same stream, which keeps both correct.  Calls on one stream use the workspace in stream order; before
 * switching to another stream while earlier calls may still be running, the
 * caller orders the new stream after the old one (for example an event
 * recorded on the old stream and waited on by the new), since both streams'
 * calls use the same workspace.
 */
#ifndef MPCGEMM_H
#define MPCGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPCG_EXP_ZERO INT32_MIN
#define MPCG_MIN_PREC 2
#define MPCG_MAX_PREC 4096

enum {
    MPCG_OK = 0,
    MPCG_EINVAL = -1,      /* bad dimension, leading dimension, precision, enum, NULL, aliasing */
    MPCG_ENOMEM = -2,      /* workspace too small / allocation failed */
    MPCG_ERANGE = -3,      /* input exponent outside [-2^30, 2^30], output exponent overflow, or a
                              double component beyond the largest double (mpcg_to_doubles) */
    MPCG_EHIP = -4,        /* HIP runtime error (text in mpcg_last_error) */
    MPCG_EUNSUPPORTED = -5,/* valid request this build cannot serve */
    MPCG_EDOMAIN = -6,     /* nonzero input whose significand top bit is clear; an infinite or NaN
                              double given to mpcg_from_doubles */
    MPCG_ESPREAD = -7      /* an operand's exponent spread exceeded mpcg_options.max_spread */
};

typedef struct {
    uint8_t *sign;
    int32_t *exp;
    uint64_t *mant;
    int64_t limb_stride;
} mpcg_part;

typedef struct {
    mpcg_part re, im;
} mpcg_cmat;

typedef enum { MPCG_4M = 0, MPCG_3M = 1, MPCG_AUTO = 2 } mpcg_mode;
typedef enum { MPCG_EXACT = 0, MPCG_TRUNCATED = 1 } mpcg_scheme;
typedef enum { MPCG_SLICE_INT8 = 0, MPCG_SLICE_FP64 = 1 } mpcg_slice;

/*
 * mp_cgemm - C := A B (eq. 1), A m x k (lda), B k x n (ldb), C m x n (ldc).
 *   mode   MPCG_4M: eq. (5), four real slice products per slice pair.
 *          MPCG_3M: eq. (6), three; (Re A + Im A) and (Re B + Im B) are formed
 *          exactly in fixed point, so no accuracy is lost.
 *          MPCG_AUTO: the form mpcg_autotune found faster for this size class
 *          (3M when the tuning cache has no entry); exact-scheme bits are the
 *          same either way.
 *   scheme MPCG_EXACT: every slice pair is kept; the result is the exact sum
 *          rounded once (bit-identical for 4M/3M and for both slice types).
 *          MPCG_TRUNCATED: slice pairs (s, t) with s + t above a cutoff are
 *          dropped (the triangular product loop of Algorithm 2); every
 *          component then satisfies
 *            |C~ - C*| <= 2^-(prec_bits-4) * sum_k |a_ik|_max |b_kj|_max,
 *          with C* the exact product and |z|_max = max(|Re z|, |Im z|).
 *   Slices are signed 8-bit digits (balanced base 2^8) on INT8 matrix cores.
 * Quick returns: m == 0 or n == 0 does nothing; k == 0 writes +0 to C.
 * Returns MPCG_OK, MPCG_EINVAL, MPCG_ENOMEM, MPCG_ERANGE (input exponents),
 * MPCG_EHIP.  Output exponent overflow and non-normalized inputs are reported
 * by mpcg_stream_status.
 */
int mp_cgemm(int m, int n, int k, const mpcg_cmat *A, int lda, const mpcg_cmat *B, int ldb,
             mpcg_cmat *C, int ldc, int prec_bits, int mode, int scheme);

/* Options for mp_cgemm_ex (NULL = defaults, all fields 0). */
typedef struct {
    int slice_type;       /* MPCG_SLICE_INT8 (default) or MPCG_SLICE_FP64: FP64 slices of
                             floor((53 - ceil(log2 k)) / 2) bits, the slice width rule of
                             Algorithm 2, their plane products as rocBLAS DGEMMs on the FP64
                             matrix cores, accumulated exactly */
    int cutoff_override;  /* truncated scheme: > 0 keeps pairs with s + t <= cutoff_override
                             (no error bound is then promised); 0 = derived cutoff */
    int ksplit_override;  /* > 0: number of contraction chunks; 0 = planner's choice */
    int block_override;   /* > 0: band width of the INT8 slice GEMM, the number of consecutive
                             anti-diagonals s + t a wavefront accumulates at once (8, 12, 16 or 20) */
    int max_spread;       /* > 0: size the slices for row/column exponent spreads of at most
                             max_spread (as for mpcg_workspace_size) instead of reading the
                             exponent scan back.  The call then never synchronizes, and with a
                             workspace set by mpcg_set_workspace it allocates nothing, so it may
                             be captured into a HIP graph (timing off).  The scales still come
                             from the data; an operand whose spread exceeds the bound makes
                             mpcg_stream_status return MPCG_ESPREAD (that result is invalid),
                             and input exponents beyond 2^30 are reported there as MPCG_ERANGE. */
    int adaptive;         /* 1: slice counts per block of rows of A and of columns of B (the
                             adaptive numbers of divisions the paper's concluding section asks
                             for).  After the exponent scan, rows of A and columns of B are
                             grouped into blocks of 256 (or of `adaptive` rows when it is a
                             multiple of 32 above 1), neighbouring blocks that need the same
                             slice count (and, truncated, the same cutoff share) are merged, and
                             if more than one block results the block products run as one
                             batched call, each planned from its own spreads (mp_cgemm_batched).
                             Exact-scheme bits are unchanged; the truncated bound holds per
                             block.  INT8 slices; ignored with max_spread > 0; 0 = off. */
    int strassen;         /* 1: one level of Strassen's recursion over the slice products
                             (Algorithm 1 applied to the exactly split operands): the seven
                             half-size products M1..M7 of the operand quadrants' sums and
                             differences, each sum formed exactly as it is split into digits,
                             and the quadrants of C recombined from the products' exact digit
                             streams before the one rounding, so the bits are those of the
                             plain product with 7/8 of its slice-pair work at equal slice
                             counts (the operand sums take one more bit of headroom, and the
                             rows folded together share a scale, which can add a slice).
                             Applies to C := AB in the exact scheme with INT8 slices, m, n and k
                             even, and no max_spread or adaptive option; elsewhere, in batches
                             and in mp_cgemm_ex_noalloc the plain product runs, as it does when
                             the half-size product would take more than 4 contraction chunks
                             or the seven products' workspace cannot be had (out of memory, or
                             beyond a workspace set by mpcg_set_workspace).
                             mpcg_info.strassen reports which ran.  0 = off. */
    int part_scales;      /* 1: separate scales for the Re and Im parts (MPCG_4M, exact scheme,
                             INT8 slices, C := AB; the adaptive numbers of divisions of the
                             paper's concluding section, per component).  Each part of a row of
                             A (column of B) is scaled by its own largest exponent, so a part far
                             below the other costs no slices; the four real products run as two
                             slice GEMMs and each component of C is the exact sum of its two
                             products, shifted by the whole digits between their scales, rounded
                             once: the bits of the one-scale product.  Runs only where it needs
                             fewer slice pairs than one scale per row (and the scales of a
                             component's two products lie within 4096 digits, and their
                             workspace can be had); otherwise, in batches and in
                             mp_cgemm_ex_noalloc the one-scale product runs.
                             mpcg_info.part_scales reports which ran.  0 = off. */
} mpcg_options;

/* Plan and timing report of one multiplication. */
typedef struct {
    int S_A, S_B;         /* slices per operand (A side, B side) */
    int w;                /* bits per slice digit */
    int cutoff;           /* highest kept diagonal s + t */
    int nprod;            /* real slice products per slice pair: 4 (4M) or 3 (3M) */
    int ksplit;           /* contraction chunks */
    int block;            /* band width of the INT8 slice GEMM (2 for FP64: pair block) */
    int strassen;         /* levels of Strassen's recursion run: 0 or 1 (the plan fields then
                             describe each of the seven half-size products) */
    long long pairs;      /* kept slice pairs (s, t) */
    double algo_ops;      /* 2*m*n*k*pairs*nprod: slice-product operations (all seven products
                             with Strassen's recursion) */
    double bound_bits;    /* truncated: error bound exponent (error <= 2^-bound_bits * sum|a||b|) */
    int part_scales;      /* 1 if the Re and Im parts were scaled separately (S_A, S_B then cover
                             each part's own spread) */
    int apart;            /* 1 if each 3M real product ran on workgroups of its own (a digit
                             stream per product and contraction chunk) */
} mpcg_info;

/* mp_cgemm with options; info (may be NULL) receives the plan. */
int mp_cgemm_ex(int m, int n, int k, const mpcg_cmat *A, int lda, const mpcg_cmat *B, int ldb,
                mpcg_cmat *C, int ldc, int prec_bits, int mode, int scheme,
                const mpcg_options *opt, mpcg_info *info);


/* Size in bytes of the fixed device buffer of mp_cgemm_ex_noalloc. */
#define MPCG_NOALLOC_BYTES (128u << 20)

/*
 * mp_cgemm_ex_noalloc - mp_cgemm_ex for callers that cannot allocate memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, layout, results (bit for bit) and errors as
 * mp_cgemm_ex, but every byte of device memory the call needs beyond A, B
 * and C (status word, exponent scan, digit planes, diagonal digits) comes
 * from a fixed buffer of MPCG_NOALLOC_BYTES inside the library, one per
 * device, held until the process ends; the call makes no hipMalloc, hipFree,
 * hipHostMalloc or event creation (timing is off for it).
 *   - A product whose scan and workspace exceed the buffer is rejected with
 *     MPCG_ENOMEM before any device work (mpcg_workspace_size with the same
 *     arguments gives the workspace part; the scan adds 16 (m + n) bytes
 *     plus 256, rounded up to 256).  Where mp_cgemm_ex would run the three
 *     real products of a 3M product on workgroups of their own (a digit
 *     stream each) and that workspace exceeds the buffer, this call runs
 *     them together (a third of the streams; info->block may then differ,
 *     the result does not).  256 x 256 x 256 at 256 bits (about 89 MiB
 *     with its real products apart), 64^3 at 1024 bits (43-90 MiB) and 32^3 at 4096 bits fit; 128^3
 *     at 1024 bits does not (138 MiB in 3M, 225 MiB in 4M, whose real
 *     products then run on workgroups of their own, a digit stream each).
 *   - adaptive slicing (opt->adaptive without max_spread) and FP64 slices
 *     (whose DGEMMs run through rocBLAS, which allocates) are rejected with
 *     MPCG_EUNSUPPORTED.
 *   - Without opt->max_spread the call reads its exponent scan back into host
 *     stack memory and synchronizes the stream once, as mp_cgemm_ex does; with
 *     max_spread > 0 it never synchronizes and may be captured into a HIP
 *     graph.
 *   - The buffer is shared by every call of this entry point on a device and
 *     keeps the last call's contents; each call initializes what it reads.
 *     Calls that overlap on one device (on different streams, or from
 *     several host threads whose stream work overlaps) race on it: the caller
 *     orders them.  mp_cgemm_ex and the other entry points do not use it.
 *   - Device-detected conditions are reported by mpcg_stream_status as for
 *     mp_cgemm_ex (the buffer's own status word is read and cleared too).
 * The buffer is set up on a device's first call: its device address is looked
 * up and its status word cleared (a kernel on the library stream).
 */
int mp_cgemm_ex_noalloc(int m, int n, int k, const mpcg_cmat *A, int lda, const mpcg_cmat *B, int ldb,
                        mpcg_cmat *C, int ldc, int prec_bits, int mode, int scheme,
                        const mpcg_options *opt, mpcg_info *info);

/*
 * mp_cgemm_acc - the accumulating product C := C + sign * A B (sign = +1 or
 * -1), the trailing update of the blocked complex LU (Sec. IV-B: the update
 * of the remaining block by the product of the panel's two factors).  Each
 * component of C becomes RNE_p of the exact sum of its current value and of
 * the exact component of sign * A B: one rounding, as for mp_cgemm (so with
 * C = 0 on entry the result equals mp_cgemm's, negated for sign = -1).
 * C (ldc) is read and written in place: its entries on entry are the
 * addend, read as their top prec_bits significand bits like every input.
 * Arguments, layout, ownership, validation, asynchrony and the truncated
 * scheme's bound (which then applies to the product term) are as for
 * mp_cgemm_ex; k = 0 or an all-zero A or B leaves C unchanged.  INT8 slices
 * only.  Returns MPCG_OK, MPCG_EINVAL (also for a sign other than +1 / -1),
 * MPCG_ENOMEM, MPCG_ERANGE, MPCG_EHIP, MPCG_EUNSUPPORTED (FP64 slices).
 */
int mp_cgemm_acc(int m, int n, int k, const mpcg_cmat *A, int lda, const mpcg_cmat *B, int ldb,
                 mpcg_cmat *C, int ldc, int prec_bits, int mode, int scheme, int sign,
                 const mpcg_options *opt, mpcg_info *info);

/*
 * One product of a batch: C := A B with A m x k (lda), B k x n (ldb), C m x n
 * (ldc).  The mpcg_cmat structs are host structs holding device pointers.
 */
typedef struct {
    int m, n, k;
    const mpcg_cmat *A;
    int lda;
    const mpcg_cmat *B;
    int ldb;
    mpcg_cmat *C;
    int ldc;
} mpcg_problem;

/*
 * mp_cgemm_batched - count independent products C_i := A_i B_i (eq. 1 for
 * each) sharing prec_bits, mode and scheme, INT8 slices.  `problems` is a host
 * array.  Each stage of the whole batch is one launch: one exponent scan per
 * side, one read-back of all the spreads (one stream synchronization; none
 * with opt->max_spread > 0), one split per side, one persistent slice-GEMM
 * launch per band-width class over all (problem, output tile group,
 * contraction chunk) items, balanced longest-first across the compute units,
 * and one rounding launch.  The band width and contraction chunks are chosen
 * per problem from its size class (opt->block_override / ksplit_override
 * force them).  Results are the same bits as mp_cgemm on each problem.
 * Every problem is validated as for mp_cgemm, and C_i must not overlap any
 * A_j, B_j or another C_j.  info (may be NULL) receives the largest S_A, S_B,
 * cutoff, ksplit and band width and the summed pairs and algo_ops.
 * Graph capture: with opt->max_spread > 0 and a workspace from
 * mpcg_set_workspace of at least mpcg_workspace_size_batched bytes, the
 * batch's job tables (problem descriptors and work items) live in that
 * workspace and, while the stream is capturing, are written by kernels that
 * carry them in their arguments, so a captured graph owns everything it
 * replays; later calls, batched or not, do not disturb it (the graph keeps
 * using the workspace, which the caller must not hand to other work the
 * replays overlap).  Capturing a batch without max_spread, without a caller
 * workspace, or before any batched call has run on the library (which sets
 * up its status word) returns MPCG_EUNSUPPORTED.
 * Returns MPCG_OK, MPCG_EINVAL, MPCG_ENOMEM, MPCG_ERANGE, MPCG_EHIP,
 * MPCG_EUNSUPPORTED (FP64 slices; capture as above).
 */
int mp_cgemm_batched(int count, const mpcg_problem *problems, int prec_bits, int mode, int scheme,
                     const mpcg_options *opt, mpcg_info *info);

/*
 * mpcg_workspace_size_batched - bytes of workspace a batch planned from
 * opt->max_spread (> 0, required) needs: every problem's slice planes and
 * digits, the exponent scans and the job tables (the same planning as
 * mp_cgemm_batched / mp_cgemm_batched_acc with these arguments; no device
 * work).  Returns 0 for invalid arguments or a batch with nothing to compute.
 */
size_t mpcg_workspace_size_batched(int count, const mpcg_problem *problems, int prec_bits, int mode, int scheme,
                                   const mpcg_options *opt);

/*
 * Size-class tuning (the planner's choices per size class, measured).  A size
 * class is (device architecture, scheme, requested form, ceil(log2 m),
 * ceil(log2 n), ceil(log2 k), ceil(S / 8)) with S the larger slice count of
 * the two operands.  For a class in the cache the planner takes its INT8
 * band width, its work-item target (which sets the contraction chunks of a
 * single product; batches keep balancing their chunks over the compute
 * units) and, for MPCG_AUTO, its form, unless the options override them.
 * None of these choices changes a bit of an exact-scheme result.  The cache
 * starts empty; if the environment variable MPCG_TUNE_CACHE names a file,
 * the first planning call reads it (a missing or malformed file is skipped).
 */
typedef struct {
    int band;         /* chosen band width (8, 12, 16 or 20) */
    int groups;       /* chosen work-item target (256 ... 2048) */
    int mode;         /* chosen form: MPCG_4M or MPCG_3M */
    int S;            /* slice count of the size class key */
    int candidates;   /* plans measured */
    float us;         /* time of one call with the chosen plan */
    float untuned_us; /* time of one call with the fixed rule's plan */
} mpcg_tune_report;

/*
 * mpcg_autotune - measures the plans of one product (the caller's operands:
 * A, B and C as for mp_cgemm, C overwritten) and stores the fastest in the
 * cache under the product's size class: band widths 8, 12, 16, 20 (4M: up to
 * 16), work-item targets 256, 512, 1024, 2048, and for mode MPCG_AUTO both
 * forms; reps timed calls per plan (at least 1) after one untimed call, on
 * the library stream, synchronously.  report (may be NULL) receives the
 * choice.  INT8 slices, no spread bound.  Returns MPCG_OK, MPCG_EINVAL (also
 * for an empty product), MPCG_ENOMEM, MPCG_ERANGE, MPCG_EHIP.
 */
int mpcg_autotune(int m, int n, int k, const mpcg_cmat *A, int lda, const mpcg_cmat *B, int ldb,
                  mpcg_cmat *C, int ldc, int prec_bits, int mode, int scheme, int reps,
                  mpcg_tune_report *report);

/*
 * mpcg_autotune_batched - the same for a batch (as for mp_cgemm_batched;
 * outputs overwritten): measures the whole batch with each problem's own
 * band width and 3M (4M if asked for), then with one band width (8, 12, 16,
 * 20; 4M up to 16) and form (both for MPCG_AUTO) for every problem, reps
 * timed calls each after one untimed call.  The winner is stored for the
 * size class of every problem of the batch (work-item target 512): the
 * uniform plan, or, if none beat the first, each problem's own band in the
 * first form (report->band is then 0).  opt may carry max_spread and ksplit_override (no block or adaptive
 * option).  Returns as mp_cgemm_batched, MPCG_EINVAL also for a bad option.
 */
int mpcg_autotune_batched(int count, const mpcg_problem *problems, int prec_bits, int mode, int scheme, int reps,
                          const mpcg_options *opt, mpcg_tune_report *report);

/*
 * mpcg_tune_load / mpcg_tune_save - read (merging the entries of this
 * device's architecture into the cache) or write the cache as JSON at path
 * (NULL: the path in MPCG_TUNE_CACHE).  Return the number of entries read or
 * written, or MPCG_EINVAL (no path, an unreadable or malformed file, a
 * failed write; the file is written whole or not at all).
 * mpcg_tune_clear empties the cache (and keeps MPCG_TUNE_CACHE from being
 * read later).
 */
int mpcg_tune_load(const char *path);
int mpcg_tune_save(const char *path);
int mpcg_tune_clear(void);

/*
 * mp_cgemm_batched_acc - the batched accumulating product: C_i := C_i +
 * sign * A_i B_i in place for every problem (sign = +1 or -1), each entry
 * rounded once as in mp_cgemm_acc, with the launches of mp_cgemm_batched.
 * The same validation and returns as mp_cgemm_batched (MPCG_EINVAL also for
 * a sign other than +1 / -1); a problem with k = 0 or an all-zero A_i or B_i
 * leaves its C_i unchanged.
 */
int mp_cgemm_batched_acc(int count, const mpcg_problem *problems, int prec_bits, int mode, int scheme, int sign,
                         const mpcg_options *opt, mpcg_info *info);

/*
 * mp_zgetrf - blocked complex LU factorization with partial pivoting, P A =
 * L U, in place (Sec. IV-B: the factorization whose trailing updates A22 -
 * L21 U12 are matrix products).  A is n x n (device arrays, leading
 * dimension lda >= max(1, n)); on return its strict lower triangle holds L
 * (unit diagonal not stored) and its upper triangle U.  ipiv (device int32
 * [n], caller-owned) receives the interchanges, 0-based: row c was exchanged
 * with row ipiv[c] >= c, in the order c = 0, 1, ...  nb is the block width
 * (the paper's K; 0 means 64).
 *
 * Order of operations (each product or update rounded once per component,
 * to nearest with ties to even, as in mp_cgemm_acc):
 *   for each block column j of width jb:
 *     for each column c of the block:
 *       pivot: the first row r >= c with the largest RNE(|Re a_rc| + |Im a_rc|)
 *       (LAPACK's |Re| + |Im| magnitude, rounded once); rows c and r
 *       exchanged over all n columns;
 *       reciprocal of the pivot y: Re y / |y|^2 and -Im y / |y|^2, each
 *       rounded once from its exact value (MPC's correctly rounded division,
 *       Sec. II); a zero y gives zero;
 *       column below the pivot := each entry times the reciprocal;
 *       rank-1 update of the rest of the block column;
 *     U12 := L11^-1 A12 by rank-1 updates; A22 := A22 - L21 U12 (k = jb).
 * A zero pivot column is multiplied by zero and reported in the return value.
 * mode (MPCG_4M / MPCG_3M) selects the product form, which does not change a
 * bit of the result.  Synchronous (returns after the device work); allocates
 * a scratch buffer of about 10 n (8L + 5) bytes.
 * Returns 0, c + 1 if the first exactly zero pivot was in column c (as
 * LAPACK's info), MPCG_EINVAL (bad n, lda, nb, precision, mode, NULL pointer,
 * overlapping arrays), MPCG_ERANGE, MPCG_EHIP.
 */
int mp_zgetrf(int n, mpcg_cmat *A, int lda, int *ipiv, int nb, int prec_bits, int mode);

/*
 * mp_zgetrs - solves A X = B with the factors of mp_zgetrf (same n, lda,
 * ipiv, prec_bits): B (n x nrhs, device, leading dimension ldb >= max(1, n))
 * is overwritten by X.  The interchanges are applied to B; then, row by row,
 * Y_c := RNE(B_c - L(c, 0:c) Y(0:c, :)) for c = 1 .. n-1 (one rounding per
 * entry) and, for c = n-1 down to 0, X_c := RNE(RNE(Y_c - U(c, c+1:n)
 * X(c+1:n, :)) * reciprocal of U(c, c)), the reciprocal formed as in
 * mp_zgetrf (Sec. IV-B: forward and backward substitution).  Synchronous.
 * ipiv must hold mp_zgetrf's interchanges; an entry outside [0, n) is skipped.
 * Returns 0, MPCG_EINVAL (also for B overlapping A or ipiv), MPCG_ERANGE,
 * MPCG_EHIP.
 */
int mp_zgetrs(int n, int nrhs, const mpcg_cmat *A, int lda, const int *ipiv, mpcg_cmat *B, int ldb, int prec_bits,
              int mode);

/*
 * Multi-component fixed-precision inputs (double-double, triple-double,
 * quad-double), the multi-component arithmetic the paper's concluding section
 * names for future work: converts them into the number format above, so that
 * they feed mp_cgemm unchanged.
 *
 * One real component (call once for Re and once for Im) of a rows x cols
 * column-major matrix whose entry (r, c) is the exact sum of ncomp doubles
 * (1 <= ncomp <= 4): component i at src[i * plane + c * ld + r], device
 * memory, plane >= ld * cols (0 means exactly ld * cols).  Each sum is formed
 * exactly (any finite doubles, subnormals included, any gaps between them)
 * and rounded once to prec_bits, to nearest with ties to even, into dst
 * (device arrays, leading dimension ldd, the layout of an mpcg_part); an
 * exactly zero sum is written as +0.  Host-side validation as for mp_cgemm
 * (MPCG_EINVAL for a bad dimension, ncomp, precision, NULL pointer or dst
 * overlapping src).  An infinite or NaN component writes +0 and is reported
 * as MPCG_EDOMAIN by mpcg_stream_status.  Asynchronous on the library's
 * stream; allocates nothing after the first call of the process.
 */
int mpcg_from_doubles(int rows, int cols, int ncomp, const double *src, int ld, long long plane, mpcg_part *dst,
                      int ldd, int prec_bits);

/*
 * The opposite conversion: each entry of one real component (the layout of
 * an mpcg_part, leading dimension lds, its top prec_bits significand bits)
 * written as ncomp doubles (1 <= ncomp <= 4), component i at
 * dst[i * plane + c * ld + r] (device memory, plane >= ld * cols, 0 means
 * exactly ld * cols).  Greedy: component i is the double nearest the value
 * minus the components before it (ties to even, gradual underflow, the sign
 * kept on a zero that underflows); an exactly zero remainder gives +0.  With
 * enough components (a normalised expansion needs one per 53 significant
 * bits) their sum is the entry exactly.  A component beyond the largest
 * double is written as +-infinity and reported as MPCG_ERANGE by
 * mpcg_stream_status (the later components then continue from the
 * unbounded rounding).  Host-side validation as for mpcg_from_doubles.
 */
int mpcg_to_doubles(int rows, int cols, const mpcg_part *src, int lds, int prec_bits, int ncomp, double *dst, int ld,
                    long long plane);

/* Issue subsequent work on this HIP stream (hipStream_t as void*; NULL = null
 * stream).  The setting is per process.  It does not order the new stream
 * after work still running on the old one; the caller does (see THREADS). */
int mpcg_set_stream(void *hip_stream);

/*
 * Use caller-owned device memory as workspace (NULL/0 = library-owned,
 * grown on demand with hipMalloc).  A multiplication whose plan needs more
 * than `bytes` fails with MPCG_ENOMEM.
 */
int mpcg_set_workspace(void *dev_ptr, size_t bytes);

/*
 * Workspace bytes needed for a multiplication whose operands have row/column
 * exponent spreads of at most max_spread (E_i - min exponent of the row),
 * e.g. 2R for exponents drawn from [-R, R].
 */
size_t mpcg_workspace_size(int m, int n, int k, int prec_bits, int mode, int scheme,
                           const mpcg_options *opt, int max_spread);

/*
 * Synchronize `hip_stream` and return (and clear) the device status of the
 * work issued so far: MPCG_OK, MPCG_ERANGE (an output exponent overflowed
 * int32 and that entry was written as zero, or, with max_spread, an input
 * exponent was beyond 2^30), MPCG_EDOMAIN (a nonzero input had its
 * significand top bit clear) or MPCG_ESPREAD (max_spread was too small).
 */
int mpcg_stream_status(void *hip_stream);

/* Text of the calling thread's last error ("" if none). */
const char *mpcg_last_error(void);

/* Device kernel time of the last multiplication, per stage, in microseconds
 * (scan, split, slice GEMM, round), measured with HIP events when enabled. */
int mpcg_enable_timing(int on);
int mpcg_last_timing(float us[4]);

/* Sum of the per-stage kernel times (us) over every multiplication issued
 * since timing was enabled or since the previous report, and their number;
 * synchronizes with the last recorded event and starts a new collection. */
int mpcg_timing_report(float us_sum[4], int *ncalls);

/*
 * Matrix-core rate probe (measurement support, no step of the method):
 * `blocks` workgroups of 4 wavefronts each issue `iters` x 8 back-to-back
 * matrix instructions from registers, no memory traffic; kind 0 is the INT8
 * slice products' v_mfma_i32_16x16x64_i8 (32768 integer ops each), kind 1
 * the FP64 plain form's v_mfma_f64_16x16x4_f64 (2048 flops each).  On the
 * library stream; synchronizes it.  `sink`: a device buffer of at least 4
 * bytes (one word is written).  Returns the operations issued in *ops and
 * the kernel time in *ms (HIP events).  MPCG_EINVAL for kind outside {0, 1},
 * blocks outside [1, 2^20], iters outside [1, 2^24] or a NULL pointer.
 */
int mpcg_probe_mfma(int kind, int blocks, int iters, void *sink, double *ops, float *ms);

#ifdef __cplusplus
}
#endif

#endif /* MPCGEMM_H */
