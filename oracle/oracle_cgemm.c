/*
 * CPU oracle for multi-precision complex matrix multiplication.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this library.  It shares no
 * code, header or table with the device path.
 *
 * What it computes (the plain definition, no Ozaki splitting at all):
 *   C := A B  (eq. 1), entry by entry as the triple loop of eq. 2, with each
 *   complex product expanded into real products (eq. 3, the 4M form):
 *     Re c_ij = sum_k ( Re a_ik Re b_kj - Im a_ik Im b_kj )
 *     Im c_ij = sum_k ( Re a_ik Im b_kj + Im a_ik Re b_kj )
 *   Both sums are formed EXACTLY in a long two's-complement fixed-point
 *   accumulator and then rounded ONCE to prec_bits, round to nearest, ties to
 *   even.  Exact evaluation followed by a single rounding is the reading this
 *   project takes of "MPFR arithmetic" for the result of the whole product.
 *
 *   A second evaluation form follows the 3M expansion (eq. 4 / eq. 6):
 *     Re c_ij = sum_k Re a Re b  -  sum_k Im a Im b
 *     Im c_ij = sum_k (Re a + Im a)(Re b + Im b) - sum_k Re a Re b - sum_k Im a Im b
 *   with the sums Re a + Im a formed exactly.  In exact arithmetic it equals
 *   the 4M form, so both forms must round to identical bits.
 *
 * Number format of one real component (column-major, leading dimension ld):
 *   sign[c*ld + r]  uint8, 0 = +, 1 = -
 *   exp [c*ld + r]  int32, value = (-1)^sign * M * 2^(exp - 64L); INT32_MIN = zero
 *   mant[l*limb_stride + c*ld + r]  uint64 limb l of M, limb 0 least significant
 * Only the top prec_bits bits of M are read (lower bits are ignored).
 * Outputs use the same format: left-aligned significand, low bits zero,
 * exact zero written as sign 0, exp INT32_MIN, limbs 0.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXP_ZERO INT32_MIN

typedef unsigned __int128 u128;

typedef struct {
    const uint8_t *sign;
    const int32_t *exp;
    const uint64_t *mant;
    int64_t limb_stride;
} orc_in_part;

typedef struct {
    orc_in_part re, im;
} orc_in_cmat;

typedef struct {
    uint8_t *sign;
    int32_t *exp;
    uint64_t *mant;
    int64_t limb_stride;
} orc_out_part;

typedef struct {
    orc_out_part re, im;
} orc_out_cmat;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ERANGE = -3 };
enum { ORC_FORM_4M = 0, ORC_FORM_3M = 1 };

/* ------------------------------------------------------------------------ */
/* A decoded real number: (-1)^neg * sig * 2^(e - p), sig a p-bit integer in  */
/* L limbs (top bit p-1 set), or zero.                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int zero;
    int neg;
    int64_t e;       /* MPFR exponent: |x| in [2^(e-1), 2^e) */
    uint64_t *sig;   /* L limbs */
} orc_real;

/* Read entry `idx` of a component and keep only its top p bits, shifted so that
 * the significand is the integer sig with value sig * 2^(e - p). */
static void decode_entry(const orc_in_part *P, int64_t idx, int L, int p, orc_real *out)
{
    int32_t e = P->exp[idx];
    if (e == ORC_EXP_ZERO) {
        out->zero = 1;
        out->neg = 0;
        out->e = 0;
        memset(out->sig, 0, sizeof(uint64_t) * (size_t)L);
        return;
    }
    out->zero = 0;
    out->neg = P->sign[idx] ? 1 : 0;
    out->e = e;
    int drop = 64 * L - p; /* 0..63 */
    for (int l = 0; l < L; ++l) {
        uint64_t lo = P->mant[(int64_t)l * P->limb_stride + idx];
        uint64_t hi = (l + 1 < L) ? P->mant[(int64_t)(l + 1) * P->limb_stride + idx] : 0;
        if (l == 0 && drop)
            lo &= ~((1ULL << drop) - 1ULL); /* ignore bits below the precision */
        out->sig[l] = drop ? ((lo >> drop) | (hi << (64 - drop))) : lo;
    }
}

/* ------------------------------------------------------------------------ */
/* Natural-number helpers on little-endian uint64 limb arrays.               */
/* ------------------------------------------------------------------------ */

/* out[0 .. na+nb) = a * b, schoolbook. */
static void mag_mul(const uint64_t *a, int na, const uint64_t *b, int nb, uint64_t *out)
{
    memset(out, 0, sizeof(uint64_t) * (size_t)(na + nb));
    for (int i = 0; i < na; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < nb; ++j) {
            u128 t = (u128)a[i] * b[j] + out[i + j] + carry;
            out[i + j] = (uint64_t)t;
            carry = (uint64_t)(t >> 64);
        }
        out[i + nb] = carry;
    }
}

/* acc (two's complement, nacc limbs) += (negate ? -1 : +1) * (v << sh), mod 2^(64 nacc). */
static void acc_add_shifted(uint64_t *acc, int nacc, const uint64_t *v, int nv, int64_t sh, int negate)
{
    int64_t lo = sh >> 6;
    int b = (int)(sh & 63);
    /* shifted value occupies limbs [lo, lo + nv] */
    uint64_t carry = 0; /* for add: carry; for sub: borrow */
    for (int64_t t = 0; t <= nv; ++t) {
        uint64_t cur = (t < nv) ? v[t] : 0;
        uint64_t prev = (t > 0) ? v[t - 1] : 0;
        uint64_t piece = b ? ((cur << b) | (prev >> (64 - b))) : cur;
        int64_t pos = lo + t;
        if (pos >= nacc)
            break;
        if (!negate) {
            u128 s = (u128)acc[pos] + piece + carry;
            acc[pos] = (uint64_t)s;
            carry = (uint64_t)(s >> 64);
        } else {
            u128 s = (u128)acc[pos] - piece - carry;
            acc[pos] = (uint64_t)s;
            carry = (uint64_t)((s >> 64) ? 1 : 0);
        }
    }
    for (int64_t pos = lo + nv + 1; carry && pos < nacc; ++pos) {
        if (!negate) {
            acc[pos] += 1;
            carry = (acc[pos] == 0);
        } else {
            carry = (acc[pos] == 0);
            acc[pos] -= 1;
        }
    }
}

static int mag_is_zero(const uint64_t *a, int n)
{
    for (int i = 0; i < n; ++i)
        if (a[i])
            return 0;
    return 1;
}

static void mag_negate(uint64_t *a, int n)
{
    uint64_t carry = 1;
    for (int i = 0; i < n; ++i) {
        uint64_t x = ~a[i];
        a[i] = x + carry;
        carry = (carry && a[i] == 0);
    }
}

static int mag_bit(const uint64_t *a, int n, int64_t pos)
{
    if (pos < 0 || pos >= 64LL * n)
        return 0;
    return (int)((a[pos >> 6] >> (pos & 63)) & 1ULL);
}

/* index of the highest set bit, or -1 */
static int64_t mag_top_bit(const uint64_t *a, int n)
{
    for (int i = n - 1; i >= 0; --i)
        if (a[i])
            return 64LL * i + 63 - __builtin_clzll(a[i]);
    return -1;
}

/* any bit set strictly below pos? */
static int mag_any_below(const uint64_t *a, int n, int64_t pos)
{
    if (pos <= 0)
        return 0;
    int64_t full = pos >> 6;
    for (int64_t i = 0; i < full && i < n; ++i)
        if (a[i])
            return 1;
    if (full < n) {
        int r = (int)(pos & 63);
        if (r && (a[full] & ((1ULL << r) - 1ULL)))
            return 1;
    }
    return 0;
}

/* bits [pos, pos + 64) of a (bits outside [0, 64n) read as zero) */
static uint64_t mag_field64(const uint64_t *a, int n, int64_t pos)
{
    uint64_t r = 0;
    for (int j = 0; j < 64; ++j)
        r |= (uint64_t)mag_bit(a, n, pos + j) << j;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Round |acc| * 2^base (acc two's complement, nacc limbs) to p bits, RNE,   */
/* and store it in L limbs.  Returns ORC_OK or ORC_ERANGE.                   */
/* ------------------------------------------------------------------------ */
static int round_store(uint64_t *acc, int nacc, int64_t base, int p, int L,
                       uint8_t *o_sign, int32_t *o_exp, uint64_t *o_mant, int64_t o_ls)
{
    int neg = (int)(acc[nacc - 1] >> 63);
    if (neg)
        mag_negate(acc, nacc);
    int64_t top = mag_top_bit(acc, nacc);
    if (top < 0) { /* exact zero -> +0 */
        *o_sign = 0;
        *o_exp = ORC_EXP_ZERO;
        for (int l = 0; l < L; ++l)
            o_mant[(int64_t)l * o_ls] = 0;
        return ORC_OK;
    }
    /* significand window: bits [top - p + 1, top] of |acc| */
    int64_t low = top - p + 1;
    int round_up = 0;
    if (low > 0) {
        int rbit = mag_bit(acc, nacc, low - 1);
        int sticky = mag_any_below(acc, nacc, low - 1);
        int lsb = mag_bit(acc, nacc, low);
        round_up = rbit && (sticky || lsb);
    }
    /* M bit j (0 <= j < 64L) <- |acc| bit (j - (64L - 1 - top)), zero below 64L - p */
    int64_t off = top + 1 - 64LL * L;
    int64_t keep_from = 64LL * L - p;
    uint64_t limbs_tmp[64 + 1];
    uint64_t *M = limbs_tmp;
    uint64_t *heap = NULL;
    if (L > 64) {
        heap = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)L);
        if (!heap)
            return ORC_ENOMEM;
        M = heap;
    }
    for (int l = 0; l < L; ++l) {
        uint64_t f = mag_field64(acc, nacc, off + 64LL * l);
        int64_t lo_bit = 64LL * l;
        if (keep_from > lo_bit) { /* clear M bits below keep_from */
            int64_t nclear = keep_from - lo_bit;
            if (nclear >= 64)
                f = 0;
            else
                f &= ~((1ULL << nclear) - 1ULL);
        }
        M[l] = f;
    }
    int64_t e_out = top + 1 + base;
    if (round_up) {
        /* add 2^(64L - p) */
        uint64_t carry = 1ULL << keep_from; /* keep_from in [0, 63] */
        for (int l = 0; l < L && carry; ++l) {
            uint64_t s = M[l] + carry;
            carry = (s < M[l]) ? 1 : 0;
            M[l] = s;
        }
        if (carry) { /* significand overflowed to 2^p: renormalize */
            for (int l = 0; l < L; ++l)
                M[l] = 0;
            M[L - 1] = 1ULL << 63;
            e_out += 1;
        }
    }
    int status = ORC_OK;
    if (e_out > INT32_MAX || e_out <= (int64_t)INT32_MIN)
        status = ORC_ERANGE;
    *o_sign = (uint8_t)neg;
    *o_exp = (status == ORC_OK) ? (int32_t)e_out : ORC_EXP_ZERO;
    for (int l = 0; l < L; ++l)
        o_mant[(int64_t)l * o_ls] = (status == ORC_OK) ? M[l] : 0;
    free(heap);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Exact signed sum of two decoded reals: (-1)^neg * mag * 2^base.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int zero;
    int neg;
    int64_t base;
    int n;
    uint64_t *mag; /* capacity given by caller */
    int64_t top;   /* |value| < 2^top */
} orc_sum;

static int exact_add(const orc_real *x, const orc_real *y, int p, int L, orc_sum *out, int cap)
{
    if (x->zero && y->zero) {
        out->zero = 1;
        return ORC_OK;
    }
    const orc_real *r[2] = {x, y};
    int64_t base = INT64_MAX, topv = INT64_MIN;
    for (int t = 0; t < 2; ++t) {
        if (r[t]->zero)
            continue;
        if (r[t]->e - p < base)
            base = r[t]->e - p;
        if (r[t]->e > topv)
            topv = r[t]->e;
    }
    int64_t width = topv + 2 - base; /* bits incl. sign */
    int n = (int)((width + 63) / 64) + 1;
    if (n > cap)
        return ORC_ENOMEM;
    memset(out->mag, 0, sizeof(uint64_t) * (size_t)n);
    for (int t = 0; t < 2; ++t) {
        if (r[t]->zero)
            continue;
        acc_add_shifted(out->mag, n, r[t]->sig, L, r[t]->e - p - base, r[t]->neg);
    }
    out->neg = (int)(out->mag[n - 1] >> 63);
    if (out->neg)
        mag_negate(out->mag, n);
    out->zero = mag_is_zero(out->mag, n);
    out->base = base;
    out->n = n;
    out->top = topv + 1;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Per-thread work: one output entry (both components).                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int m, n, k, p, L, form;
    const orc_in_cmat *A;
    int64_t lda;
    const orc_in_cmat *B;
    int64_t ldb;
    /* full-matrix output (mode 0) or per-entry output (mode 1) */
    int out_mode;
    orc_out_cmat *C;
    int64_t ldc;
    int64_t nent;
    const int32_t *ei, *ej;
    uint8_t *p_sign;   /* [nent*2] */
    int32_t *p_exp;    /* [nent*2] */
    uint64_t *p_mant;  /* [nent*2*L] */
    /* optional addend (eq. 1 extended to C := Cadd + sgn AB): NULL for C := AB */
    const orc_in_cmat *Cadd;
    int64_t ldcadd;
    int neg_prod;      /* 1: the products enter with a minus sign */
    /* exact (unrounded) output: one entry, one component */
    int nthreads;
    int tid;
    int status;
} orc_job;

typedef struct {
    /* decoded row of A and column of B */
    orc_real *ar, *ai, *br, *bi;
    orc_real cr, ci;   /* the addend's entry */
    uint64_t *sig_store;
    uint64_t *prod;    /* product scratch */
    uint64_t *acc;
    int acc_cap;
    orc_sum ua, ub;
    int sum_cap;
} orc_scratch;

static int scratch_init(orc_scratch *s, int k, int L, int64_t max_spread_limbs)
{
    memset(s, 0, sizeof(*s));
    s->ar = (orc_real *)calloc((size_t)k, sizeof(orc_real));
    s->ai = (orc_real *)calloc((size_t)k, sizeof(orc_real));
    s->br = (orc_real *)calloc((size_t)k, sizeof(orc_real));
    s->bi = (orc_real *)calloc((size_t)k, sizeof(orc_real));
    s->sig_store = (uint64_t *)calloc((size_t)(k + 1) * 4 * (size_t)L + 1, sizeof(uint64_t));
    s->sum_cap = (int)(max_spread_limbs + L + 4);
    s->ua.mag = (uint64_t *)calloc((size_t)s->sum_cap, sizeof(uint64_t));
    s->ub.mag = (uint64_t *)calloc((size_t)s->sum_cap, sizeof(uint64_t));
    s->prod = (uint64_t *)calloc((size_t)(2 * s->sum_cap), sizeof(uint64_t));
    if (!s->ar || !s->ai || !s->br || !s->bi || !s->sig_store || !s->ua.mag || !s->ub.mag || !s->prod)
        return ORC_ENOMEM;
    for (int t = 0; t < k; ++t) {
        s->ar[t].sig = s->sig_store + ((size_t)t * 4 + 0) * L;
        s->ai[t].sig = s->sig_store + ((size_t)t * 4 + 1) * L;
        s->br[t].sig = s->sig_store + ((size_t)t * 4 + 2) * L;
        s->bi[t].sig = s->sig_store + ((size_t)t * 4 + 3) * L;
    }
    s->cr.sig = s->sig_store + ((size_t)k * 4 + 0) * L;
    s->ci.sig = s->sig_store + ((size_t)k * 4 + 1) * L;
    s->cr.zero = s->ci.zero = 1;
    return ORC_OK;
}

static void scratch_free(orc_scratch *s)
{
    free(s->ar); free(s->ai); free(s->br); free(s->bi);
    free(s->sig_store); free(s->ua.mag); free(s->ub.mag); free(s->prod); free(s->acc);
}

static int ensure_acc(orc_scratch *s, int n)
{
    if (n <= s->acc_cap)
        return ORC_OK;
    uint64_t *a = (uint64_t *)realloc(s->acc, sizeof(uint64_t) * (size_t)n);
    if (!a)
        return ORC_ENOMEM;
    s->acc = a;
    s->acc_cap = n;
    return ORC_OK;
}

/* One real-product term x*y*sgn with x, y decoded reals. */
typedef struct {
    const orc_real *x, *y;
    int negate;
} term4;

/*
 * Exact sum of the real-product terms of one component, then RNE.
 * 4M form: two terms per k.  3M form (Im only): (ar+ai)(br+bi) - ar br - ai bi.
 * With an addend c (not NULL and nonzero) the exact sum is c + sgn * (products),
 * sgn = -1 when neg_prod, rounded once.
 */
static int eval_component(orc_scratch *s, int k, int p, int L, int comp, int form,
                          const orc_real *addend, int neg_prod,
                          uint8_t *o_sign, int32_t *o_exp, uint64_t *o_mant, int64_t o_ls,
                          int want_exact, int *x_neg, int64_t *x_base, uint64_t *x_mag, int x_cap, int *x_n)
{
    /* pass 1: weight range of all nonzero terms */
    int64_t base = INT64_MAX, topv = INT64_MIN;
    int64_t nterms = 0;
    for (int t = 0; t < k; ++t) {
        const orc_real *ar = &s->ar[t], *ai = &s->ai[t], *br = &s->br[t], *bi = &s->bi[t];
        term4 tm[3];
        int nt = 0;
        if (comp == 0) {
            tm[nt++] = (term4){ar, br, 0};
            tm[nt++] = (term4){ai, bi, 1};
        } else if (form == ORC_FORM_4M) {
            tm[nt++] = (term4){ar, bi, 0};
            tm[nt++] = (term4){ai, br, 0};
        } else {
            tm[nt++] = (term4){ar, br, 1};
            tm[nt++] = (term4){ai, bi, 1};
        }
        for (int q = 0; q < nt; ++q) {
            if (tm[q].x->zero || tm[q].y->zero)
                continue;
            int64_t b0 = tm[q].x->e + tm[q].y->e - 2LL * p;
            int64_t t0 = tm[q].x->e + tm[q].y->e;
            if (b0 < base) base = b0;
            if (t0 > topv) topv = t0;
            ++nterms;
        }
        if (comp == 1 && form == ORC_FORM_3M) {
            /* (ar + ai)(br + bi): magnitude < 2^(max(er,ei)+1 + max(er,ei)+1) */
            int ok_a = !(ar->zero && ai->zero), ok_b = !(br->zero && bi->zero);
            if (ok_a && ok_b) {
                int64_t ea_min = INT64_MAX, ea_max = INT64_MIN, eb_min = INT64_MAX, eb_max = INT64_MIN;
                if (!ar->zero) { ea_min = ar->e < ea_min ? ar->e : ea_min; ea_max = ar->e > ea_max ? ar->e : ea_max; }
                if (!ai->zero) { ea_min = ai->e < ea_min ? ai->e : ea_min; ea_max = ai->e > ea_max ? ai->e : ea_max; }
                if (!br->zero) { eb_min = br->e < eb_min ? br->e : eb_min; eb_max = br->e > eb_max ? br->e : eb_max; }
                if (!bi->zero) { eb_min = bi->e < eb_min ? bi->e : eb_min; eb_max = bi->e > eb_max ? bi->e : eb_max; }
                int64_t b0 = ea_min + eb_min - 2LL * p;
                int64_t t0 = ea_max + eb_max + 2;
                if (b0 < base) base = b0;
                if (t0 > topv) topv = t0;
                ++nterms;
            }
        }
    }
    const int have_add = addend && !addend->zero;
    if (have_add) {
        if (addend->e - p < base) base = addend->e - p;
        if (addend->e > topv) topv = addend->e;
        ++nterms;
    }
    if (nterms == 0) {
        if (want_exact) {
            *x_neg = 0; *x_base = 0; *x_n = 0;
            return ORC_OK;
        }
        *o_sign = 0;
        *o_exp = ORC_EXP_ZERO;
        for (int l = 0; l < L; ++l)
            o_mant[(int64_t)l * o_ls] = 0;
        return ORC_OK;
    }
    int lg = 0;
    while ((1LL << lg) < nterms + 1)
        ++lg;
    int64_t width = topv - base + lg + 2;
    int nacc = (int)((width + 63) / 64) + 1;
    int st = ensure_acc(s, nacc);
    if (st)
        return st;
    uint64_t *acc = s->acc;
    memset(acc, 0, sizeof(uint64_t) * (size_t)nacc);

    /* pass 2: exact accumulation */
    for (int t = 0; t < k; ++t) {
        const orc_real *ar = &s->ar[t], *ai = &s->ai[t], *br = &s->br[t], *bi = &s->bi[t];
        term4 tm[3];
        int nt = 0;
        if (comp == 0) {
            tm[nt++] = (term4){ar, br, 0};
            tm[nt++] = (term4){ai, bi, 1};
        } else if (form == ORC_FORM_4M) {
            tm[nt++] = (term4){ar, bi, 0};
            tm[nt++] = (term4){ai, br, 0};
        } else {
            tm[nt++] = (term4){ar, br, 1};
            tm[nt++] = (term4){ai, bi, 1};
        }
        for (int q = 0; q < nt; ++q) {
            const orc_real *x = tm[q].x, *y = tm[q].y;
            if (x->zero || y->zero)
                continue;
            mag_mul(x->sig, L, y->sig, L, s->prod);
            int neg = x->neg ^ y->neg ^ tm[q].negate ^ neg_prod;
            acc_add_shifted(acc, nacc, s->prod, 2 * L, x->e + y->e - 2LL * p - base, neg);
        }
        if (comp == 1 && form == ORC_FORM_3M) {
            if ((ar->zero && ai->zero) || (br->zero && bi->zero))
                continue;
            st = exact_add(ar, ai, p, L, &s->ua, s->sum_cap);
            if (st) return st;
            st = exact_add(br, bi, p, L, &s->ub, s->sum_cap);
            if (st) return st;
            if (s->ua.zero || s->ub.zero)
                continue;
            mag_mul(s->ua.mag, s->ua.n, s->ub.mag, s->ub.n, s->prod);
            int neg = s->ua.neg ^ s->ub.neg ^ neg_prod;
            acc_add_shifted(acc, nacc, s->prod, s->ua.n + s->ub.n, s->ua.base + s->ub.base - base, neg);
        }
    }
    if (have_add)
        acc_add_shifted(acc, nacc, addend->sig, L, addend->e - p - base, addend->neg);
    if (want_exact) {
        int neg = (int)(acc[nacc - 1] >> 63);
        if (neg)
            mag_negate(acc, nacc);
        if (nacc > x_cap)
            return ORC_ENOMEM;
        memcpy(x_mag, acc, sizeof(uint64_t) * (size_t)nacc);
        *x_neg = neg;
        *x_base = base;
        *x_n = nacc;
        return ORC_OK;
    }
    return round_store(acc, nacc, base, p, L, o_sign, o_exp, o_mant, o_ls);
}

static void load_row_col(orc_scratch *s, const orc_job *J, int i, int j)
{
    for (int t = 0; t < J->k; ++t) {
        int64_t ia = (int64_t)t * J->lda + i;
        int64_t ib = (int64_t)j * J->ldb + t;
        decode_entry(&J->A->re, ia, J->L, J->p, &s->ar[t]);
        decode_entry(&J->A->im, ia, J->L, J->p, &s->ai[t]);
        decode_entry(&J->B->re, ib, J->L, J->p, &s->br[t]);
        decode_entry(&J->B->im, ib, J->L, J->p, &s->bi[t]);
    }
}

static int64_t spread_limbs(const orc_job *J)
{
    /* the exact sum Re+Im of one entry spans at most (|e_re - e_im| + p + 2) bits */
    int64_t emin = INT64_MAX, emax = INT64_MIN;
    const orc_in_part *parts[4] = {&J->A->re, &J->A->im, &J->B->re, &J->B->im};
    int64_t counts[4] = {(int64_t)J->lda * J->k, (int64_t)J->lda * J->k, (int64_t)J->ldb * J->n,
                         (int64_t)J->ldb * J->n};
    for (int q = 0; q < 4; ++q)
        for (int64_t t = 0; t < counts[q]; ++t) {
            int32_t e = parts[q]->exp[t];
            if (e == ORC_EXP_ZERO) continue;
            if (e < emin) emin = e;
            if (e > emax) emax = e;
        }
    if (emin > emax)
        return 1;
    return (emax - emin + 2) / 64 + 2;
}

static void *worker(void *arg)
{
    orc_job *J = (orc_job *)arg;
    orc_scratch s;
    int64_t sp = spread_limbs(J);
    J->status = scratch_init(&s, J->k > 0 ? J->k : 1, J->L, sp);
    if (J->status) {
        scratch_free(&s);
        return NULL;
    }
    int64_t total = (J->out_mode == 0) ? (int64_t)J->m * J->n : J->nent;
    for (int64_t idx = J->tid; idx < total; idx += J->nthreads) {
        int i, j;
        if (J->out_mode == 0) {
            i = (int)(idx % J->m);
            j = (int)(idx / J->m);
        } else {
            i = J->ei[idx];
            j = J->ej[idx];
        }
        load_row_col(&s, J, i, j);
        if (J->Cadd) {
            int64_t ic = (int64_t)j * J->ldcadd + i;
            decode_entry(&J->Cadd->re, ic, J->L, J->p, &s.cr);
            decode_entry(&J->Cadd->im, ic, J->L, J->p, &s.ci);
        }
        for (int comp = 0; comp < 2; ++comp) {
            int st;
            const orc_real *add = J->Cadd ? (comp ? &s.ci : &s.cr) : NULL;
            if (J->out_mode == 0) {
                orc_out_part *C = comp ? &J->C->im : &J->C->re;
                int64_t o = (int64_t)j * J->ldc + i;
                st = eval_component(&s, J->k, J->p, J->L, comp, J->form, add, J->neg_prod, &C->sign[o],
                                    &C->exp[o], &C->mant[o], C->limb_stride, 0, NULL, NULL, NULL, 0, NULL);
            } else {
                int64_t o = idx * 2 + comp;
                st = eval_component(&s, J->k, J->p, J->L, comp, J->form, add, J->neg_prod, &J->p_sign[o],
                                    &J->p_exp[o], &J->p_mant[o * J->L], 1, 0, NULL, NULL, NULL, 0, NULL);
            }
            if (st && !J->status)
                J->status = st;
        }
    }
    scratch_free(&s);
    return NULL;
}

static int run_jobs(orc_job *proto, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 1024)
        nthreads = 1024;
    orc_job *jobs = (orc_job *)calloc((size_t)nthreads, sizeof(orc_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs); free(th);
        return ORC_ENOMEM;
    }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *proto;
        jobs[t].tid = t;
        jobs[t].nthreads = nthreads;
        jobs[t].status = 0;
    }
    char *started = (char *)calloc((size_t)nthreads, 1);
    if (!started) {
        free(jobs); free(th);
        return ORC_ENOMEM;
    }
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, worker, &jobs[t]) == 0)
            started[t] = 1;
        else
            jobs[t].status = ORC_ENOMEM; /* its entries stay uncomputed: report it */
    }
    worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t)
        if (started[t])
            pthread_join(th[t], NULL);
    free(started);
    int st = ORC_OK;
    for (int t = 0; t < nthreads; ++t)
        if (jobs[t].status && !st)
            st = jobs[t].status;
    free(jobs);
    free(th);
    return st;
}

static int check_common(int m, int n, int k, int p, int64_t lda, int64_t ldb, int form)
{
    if (m < 0 || n < 0 || k < 0 || p < 2 || p > 4096)
        return ORC_EINVAL;
    if (lda < (m > 1 ? m : 1) || ldb < (k > 1 ? k : 1))
        return ORC_EINVAL;
    if (form != ORC_FORM_4M && form != ORC_FORM_3M)
        return ORC_EINVAL;
    return ORC_OK;
}

/* Full product C = A B, every entry. */
int oracle_cgemm(int m, int n, int k, const orc_in_cmat *A, int64_t lda, const orc_in_cmat *B,
                 int64_t ldb, orc_out_cmat *C, int64_t ldc, int prec_bits, int form, int nthreads)
{
    int st = check_common(m, n, k, prec_bits, lda, ldb, form);
    if (st)
        return st;
    if (ldc < (m > 1 ? m : 1))
        return ORC_EINVAL;
    if (m == 0 || n == 0)
        return ORC_OK;
    orc_job J;
    memset(&J, 0, sizeof(J));
    J.m = m; J.n = n; J.k = k; J.p = prec_bits; J.L = (prec_bits + 63) / 64; J.form = form;
    J.A = A; J.lda = lda; J.B = B; J.ldb = ldb;
    J.out_mode = 0; J.C = C; J.ldc = ldc;
    return run_jobs(&J, nthreads);
}

/* Accumulating product C := Cadd + sgn A B (sgn = +1 or -1), every entry: the
 * exact sum of the addend and all real-product terms, one RNE per component.
 * C and Cadd may not share memory (the oracle reads Cadd while writing C). */
int oracle_cgemm_acc(int m, int n, int k, const orc_in_cmat *A, int64_t lda, const orc_in_cmat *B,
                     int64_t ldb, const orc_in_cmat *Cadd, int64_t ldcadd, orc_out_cmat *C, int64_t ldc,
                     int prec_bits, int form, int sgn, int nthreads)
{
    int st = check_common(m, n, k, prec_bits, lda, ldb, form);
    if (st)
        return st;
    if (ldc < (m > 1 ? m : 1) || ldcadd < (m > 1 ? m : 1) || (sgn != 1 && sgn != -1) || !Cadd)
        return ORC_EINVAL;
    if (m == 0 || n == 0)
        return ORC_OK;
    orc_job J;
    memset(&J, 0, sizeof(J));
    J.m = m; J.n = n; J.k = k; J.p = prec_bits; J.L = (prec_bits + 63) / 64; J.form = form;
    J.A = A; J.lda = lda; J.B = B; J.ldb = ldb;
    J.Cadd = Cadd; J.ldcadd = ldcadd; J.neg_prod = sgn < 0;
    J.out_mode = 0; J.C = C; J.ldc = ldc;
    return run_jobs(&J, nthreads);
}

/* The same for selected entries (ei[t], ej[t]); outputs packed as [t][comp]. */
int oracle_cgemm_acc_entries(int m, int n, int k, const orc_in_cmat *A, int64_t lda, const orc_in_cmat *B,
                             int64_t ldb, const orc_in_cmat *Cadd, int64_t ldcadd, int64_t nent,
                             const int32_t *ei, const int32_t *ej, uint8_t *o_sign, int32_t *o_exp,
                             uint64_t *o_mant, int prec_bits, int form, int sgn, int nthreads)
{
    int st = check_common(m, n, k, prec_bits, lda, ldb, form);
    if (st)
        return st;
    if (ldcadd < (m > 1 ? m : 1) || (sgn != 1 && sgn != -1) || !Cadd)
        return ORC_EINVAL;
    for (int64_t t = 0; t < nent; ++t)
        if (ei[t] < 0 || ei[t] >= m || ej[t] < 0 || ej[t] >= n)
            return ORC_EINVAL;
    if (nent == 0)
        return ORC_OK;
    orc_job J;
    memset(&J, 0, sizeof(J));
    J.m = m; J.n = n; J.k = k; J.p = prec_bits; J.L = (prec_bits + 63) / 64; J.form = form;
    J.A = A; J.lda = lda; J.B = B; J.ldb = ldb;
    J.Cadd = Cadd; J.ldcadd = ldcadd; J.neg_prod = sgn < 0;
    J.out_mode = 1; J.nent = nent; J.ei = ei; J.ej = ej;
    J.p_sign = o_sign; J.p_exp = o_exp; J.p_mant = o_mant;
    return run_jobs(&J, nthreads);
}

/* Selected entries (ei[t], ej[t]); outputs packed as [t][comp] (comp 0 = Re). */
int oracle_cgemm_entries(int m, int n, int k, const orc_in_cmat *A, int64_t lda, const orc_in_cmat *B,
                         int64_t ldb, int64_t nent, const int32_t *ei, const int32_t *ej, uint8_t *o_sign,
                         int32_t *o_exp, uint64_t *o_mant, int prec_bits, int form, int nthreads)
{
    int st = check_common(m, n, k, prec_bits, lda, ldb, form);
    if (st)
        return st;
    for (int64_t t = 0; t < nent; ++t)
        if (ei[t] < 0 || ei[t] >= m || ej[t] < 0 || ej[t] >= n)
            return ORC_EINVAL;
    if (nent == 0)
        return ORC_OK;
    orc_job J;
    memset(&J, 0, sizeof(J));
    J.m = m; J.n = n; J.k = k; J.p = prec_bits; J.L = (prec_bits + 63) / 64; J.form = form;
    J.A = A; J.lda = lda; J.B = B; J.ldb = ldb;
    J.out_mode = 1; J.nent = nent; J.ei = ei; J.ej = ej;
    J.p_sign = o_sign; J.p_exp = o_exp; J.p_mant = o_mant;
    return run_jobs(&J, nthreads);
}

/*
 * Exact (unrounded) value of one component of one entry:
 *   value = (-1)^(*neg) * mag * 2^(*base),  mag in *nmag little-endian limbs.
 * Returns ORC_ENOMEM when cap limbs are not enough (then *nmag holds the need).
 */
int oracle_exact_entry(int m, int n, int k, const orc_in_cmat *A, int64_t lda, const orc_in_cmat *B,
                       int64_t ldb, int i, int j, int comp, int prec_bits, int form, int *neg,
                       int64_t *base, uint64_t *mag, int cap, int *nmag)
{
    int st = check_common(m, n, k, prec_bits, lda, ldb, form);
    if (st)
        return st;
    if (i < 0 || i >= m || j < 0 || j >= n || (comp != 0 && comp != 1))
        return ORC_EINVAL;
    orc_job J;
    memset(&J, 0, sizeof(J));
    J.m = m; J.n = n; J.k = k; J.p = prec_bits; J.L = (prec_bits + 63) / 64; J.form = form;
    J.A = A; J.lda = lda; J.B = B; J.ldb = ldb;
    orc_scratch s;
    st = scratch_init(&s, k > 0 ? k : 1, J.L, spread_limbs(&J));
    if (st) {
        scratch_free(&s);
        return st;
    }
    load_row_col(&s, &J, i, j);
    st = eval_component(&s, k, prec_bits, J.L, comp, form, NULL, 0, NULL, NULL, NULL, 0, 1, neg, base, mag, cap,
                        nmag);
    if (st == ORC_ENOMEM && s.acc_cap > cap)
        *nmag = s.acc_cap;
    scratch_free(&s);
    return st;
}
