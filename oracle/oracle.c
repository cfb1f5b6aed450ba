/*
 * Sliding-window Pearson correlation: CPU reference ("oracle").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the GPU path.
 *
 * What it computes (Poyda & Zhizhin, arXiv 1807.06507):
 *   For every output position, the window of the two equal-shape arrays is
 *   drawn into two vectors (Introduction, problem statement), and the
 *   classical two-pass Pearson coefficient of the Introduction's formula is
 *   evaluated on them: first the two means, then the sums of products of
 *   deviations.  This is the paper's "basic version" (Section 3), i.e. the
 *   plain definition, evaluated window by window in FP64.  The paper's
 *   sliding-sum method (Section 1, steps 1-4) must reach the same value.
 *
 * Output conventions (Section 3, I/O paragraph):
 *   - the result for a window is written at the window's middle cell;
 *   - a value <= -999 anywhere in the window makes the result -2 (MISSING);
 *   - windows that cross the array border give -2 (BORDER) under the FILL
 *     policy; CLIP shrinks the window to the in-bounds part; VALID only
 *     visits windows that fit (output is compacted);
 *   - an all-equal window (zero denominator, Section 3 accuracy paragraph)
 *     gives -2 with the ZVAR_X / ZVAR_Y bit.
 *
 * Readings where the paper is silent (listed in the design notes):
 *   even k: l = floor(k/2) cells before the centre, k-1-l after;
 *   step s: output j is centred at j*s (FILL/CLIP), starts at j*s (VALID);
 *   NaN/Inf are missing too; integer inputs have no missing values;
 *   flag precedence BORDER > MISSING > ZVAR; |c| clamped to 1 (FP64 path).
 *
 * Integer inputs (u8/u16) additionally get the exactly rounded float32
 * result: the same two-pass formula in exact integer arithmetic (means
 * scaled by n so that every deviation is an integer), then round-to-nearest-
 * even of the real number P/sqrt(Q*R), decided by exact big-integer
 * comparisons against float32 midpoints.
 *
 * Parity pins: see tests/test_oracle_pins.py (exact rational brute force,
 * numpy/scipy/pandas special cases, closed-form invariants, golden files).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_U8 = 0, OR_U16 = 1, OR_F32 = 2 };
enum { OR_FILL = 0, OR_CLIP = 1, OR_VALID = 2 };
enum { FL_BORDER = 1, FL_MISSING = 2, FL_ZVAR_X = 4, FL_ZVAR_Y = 8 };

/* ------------------------------------------------------------------------ */
/* Output geometry                                                           */
/* ------------------------------------------------------------------------ */

/* Output length per dimension: ceil(N/s) for FILL and CLIP (same size as the
 * input at step 1), floor((N-k)/s)+1 for VALID.  Returns 0, or -1 on bad
 * arguments (including VALID with N < k). */
int oracle_output_shape(int ndim, const int64_t *shape, const int32_t *window,
                        const int32_t *step, int border, int64_t *out)
{
    if (ndim < 1 || ndim > 3) return -1;
    for (int d = 0; d < ndim; d++) {
        int64_t N = shape[d];
        int64_t k = window[d];
        int64_t s = step[d];
        if (N < 1 || k < 1 || s < 1) return -1;
        if (border == OR_VALID) {
            if (N < k) return -1;
            out[d] = (N - k) / s + 1;
        } else if (border == OR_FILL || border == OR_CLIP) {
            out[d] = (N + s - 1) / s;
        } else {
            return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Small unsigned big integers (little-endian 32-bit limbs), used only to    */
/* compare P^2 * 2^a against M^2 * Q * R * 2^b exactly.                      */
/* ------------------------------------------------------------------------ */

#define BN_LIMBS 24 /* 768 bits: ample for every product formed below */

typedef struct { uint32_t w[BN_LIMBS]; } bn_t;

static void bn_zero(bn_t *a) { memset(a, 0, sizeof(*a)); }

static void bn_from_u128(bn_t *a, unsigned __int128 v)
{
    bn_zero(a);
    for (int i = 0; i < 4; i++) { a->w[i] = (uint32_t)v; v >>= 32; }
}

/* r = a * b (schoolbook; r must not alias a or b) */
static void bn_mul(bn_t *r, const bn_t *a, const bn_t *b)
{
    bn_zero(r);
    for (int i = 0; i < BN_LIMBS; i++) {
        if (a->w[i] == 0) continue;
        uint64_t carry = 0;
        for (int j = 0; i + j < BN_LIMBS; j++) {
            uint64_t t = (uint64_t)a->w[i] * b->w[j] + r->w[i + j] + carry;
            r->w[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
    }
}

/* a <<= s */
static void bn_shl(bn_t *a, int s)
{
    int limbs = s / 32, bits = s % 32;
    for (int i = BN_LIMBS - 1; i >= 0; i--) {
        uint64_t v = 0;
        int src = i - limbs;
        if (src >= 0) {
            v = (uint64_t)a->w[src] << bits;
            if (bits && src - 1 >= 0) v |= (uint64_t)a->w[src - 1] >> (32 - bits);
        }
        a->w[i] = (uint32_t)v;
    }
}

static int bn_cmp(const bn_t *a, const bn_t *b)
{
    for (int i = BN_LIMBS - 1; i >= 0; i--) {
        if (a->w[i] != b->w[i]) return a->w[i] > b->w[i] ? 1 : -1;
    }
    return 0;
}

/* sign( aP / sqrt(Q*R) - m ) for aP >= 0, Q > 0, R > 0 and m > 0 a double.
 * Squares both (non-negative) sides: aP^2 vs m^2 * Q * R, with
 * m = M * 2^E exactly (M a 53-bit integer). */
static int cmp_ratio_vs(unsigned __int128 aP, unsigned __int128 Q,
                        unsigned __int128 R, double m)
{
    int ex;
    double fr = frexp(m, &ex);              /* m = fr * 2^ex, fr in [0.5,1) */
    uint64_t M = (uint64_t)ldexp(fr, 53);   /* exact */
    int E = ex - 53;                        /* m = M * 2^E */

    bn_t p, p2, q, rr, qr, mm, m2, rhs;
    bn_from_u128(&p, aP);
    bn_mul(&p2, &p, &p);
    bn_from_u128(&q, Q);
    bn_from_u128(&rr, R);
    bn_mul(&qr, &q, &rr);
    bn_from_u128(&mm, (unsigned __int128)M);
    bn_mul(&m2, &mm, &mm);
    bn_mul(&rhs, &m2, &qr);
    if (E < 0) bn_shl(&p2, -2 * E);
    else bn_shl(&rhs, 2 * E);
    return bn_cmp(&p2, &rhs);
}

static int f32_is_even(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return (u & 1u) == 0;
}

/* Round-to-nearest-even float32 of the real number P / sqrt(Q*R), where
 * Q, R > 0 and |P| <= sqrt(Q*R) (Cauchy-Schwarz).  Start from an FP64
 * estimate and move by one float32 ulp while the exact value lies outside the
 * rounding interval of the candidate. */
static float rn32_of_ratio(__int128 P, unsigned __int128 Q, unsigned __int128 R)
{
    if (P == 0) return 0.0f;
    int neg = P < 0;
    unsigned __int128 aP = neg ? (unsigned __int128)(-P) : (unsigned __int128)P;
    double est = (double)aP / sqrt((double)Q * (double)R);
    float f = (float)est;
    if (f > 1.0f) f = 1.0f;
    if (f < FLT_MIN) f = FLT_MIN;
    for (int iter = 0; iter < 64; iter++) {
        float up = nextafterf(f, INFINITY);
        double mid_hi = ((double)f + (double)up) * 0.5; /* exact in double */
        int s = cmp_ratio_vs(aP, Q, R, mid_hi);
        if (s > 0) { f = up; continue; }
        if (s == 0) { f = f32_is_even(f) ? f : up; break; }
        float dn = nextafterf(f, 0.0f);
        double mid_lo = ((double)dn + (double)f) * 0.5;
        int t = cmp_ratio_vs(aP, Q, R, mid_lo);
        if (t < 0) { f = dn; continue; }
        if (t == 0) { f = f32_is_even(f) ? f : dn; }
        break;
    }
    return neg ? -f : f;
}

/* ------------------------------------------------------------------------ */
/* One window                                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    int ndim;
    int64_t shape[3];
    int32_t window[3];
    int32_t step[3];
    int border;
    int dtype;
    double invalid;
    double missing_le;
    int64_t oshape[3];
    const void *x;
    const void *y;
} job_t;

static double load_as_double(const void *p, int dtype, int64_t i)
{
    switch (dtype) {
    case OR_U8: return (double)((const uint8_t *)p)[i];
    case OR_U16: return (double)((const uint16_t *)p)[i];
    default: return (double)((const float *)p)[i];
    }
}

static int64_t load_as_int(const void *p, int dtype, int64_t i)
{
    if (dtype == OR_U8) return ((const uint8_t *)p)[i];
    return ((const uint16_t *)p)[i];
}

/* Evaluate output flat index `o`.  xs/ys/ix are per-thread scratch of at
 * least prod(window) entries. */
static void eval_one(const job_t *J, int64_t o, double *xs, double *ys,
                     int64_t *ix, double *c64_out, float *c32_out,
                     uint8_t *flag_out)
{
    int nd = J->ndim;
    int64_t p[3] = {0, 0, 0};
    {
        int64_t rem = o;
        for (int d = nd - 1; d >= 0; d--) {
            p[d] = rem % J->oshape[d];
            rem /= J->oshape[d];
        }
    }

    /* Window range per dimension (inclusive). */
    int64_t lo[3], hi[3];
    int border_hit = 0;
    for (int d = 0; d < nd; d++) {
        int64_t k = J->window[d];
        int64_t s = J->step[d];
        if (J->border == OR_VALID) {
            lo[d] = p[d] * s;
            hi[d] = lo[d] + k - 1;
        } else {
            int64_t l = k / 2;
            int64_t r = k - 1 - l;
            lo[d] = p[d] * s - l;
            hi[d] = p[d] * s + r;
        }
        if (lo[d] < 0 || hi[d] > J->shape[d] - 1) {
            if (J->border == OR_FILL) border_hit = 1;
            if (lo[d] < 0) lo[d] = 0;
            if (hi[d] > J->shape[d] - 1) hi[d] = J->shape[d] - 1;
        }
    }
    if (border_hit) {
        *flag_out = FL_BORDER;
        *c64_out = J->invalid;
        *c32_out = (float)J->invalid;
        return;
    }

    /* Draw the window into vectors, C order. */
    int64_t n = 0;
    int64_t strides[3];
    strides[nd - 1] = 1;
    for (int d = nd - 2; d >= 0; d--) strides[d] = strides[d + 1] * J->shape[d + 1];
    int64_t a[3] = {0, 0, 0};
    for (int d = 0; d < 3; d++) a[d] = (d < nd) ? lo[d] : 0;
    for (;;) {
        int64_t flat = 0;
        for (int d = 0; d < nd; d++) flat += a[d] * strides[d];
        ix[n] = flat;
        xs[n] = load_as_double(J->x, J->dtype, flat);
        ys[n] = load_as_double(J->y, J->dtype, flat);
        n++;
        int d = nd - 1;
        while (d >= 0) {
            a[d]++;
            if (a[d] <= hi[d]) break;
            a[d] = lo[d];
            d--;
        }
        if (d < 0) break;
    }

    /* Missing values (float input only). */
    if (J->dtype == OR_F32) {
        for (int64_t i = 0; i < n; i++) {
            if (!isfinite(xs[i]) || !isfinite(ys[i]) ||
                xs[i] <= J->missing_le || ys[i] <= J->missing_le) {
                *flag_out = FL_MISSING;
                *c64_out = J->invalid;
                *c32_out = (float)J->invalid;
                return;
            }
        }
    }

    /* All-equal windows: the denominator vanishes. */
    uint8_t fl = 0;
    int eqx = 1, eqy = 1;
    for (int64_t i = 1; i < n; i++) {
        if (xs[i] != xs[0]) eqx = 0;
        if (ys[i] != ys[0]) eqy = 0;
    }
    if (eqx) fl |= FL_ZVAR_X;
    if (eqy) fl |= FL_ZVAR_Y;
    if (fl) {
        *flag_out = fl;
        *c64_out = J->invalid;
        *c32_out = (float)J->invalid;
        return;
    }

    /* Pass 1: means.  Pass 2: deviation products. */
    double sx = 0.0, sy = 0.0;
    for (int64_t i = 0; i < n; i++) { sx += xs[i]; sy += ys[i]; }
    double mx = sx / (double)n, my = sy / (double)n;
    double sxy = 0.0, sxx = 0.0, syy = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double dx = xs[i] - mx, dy = ys[i] - my;
        sxy += dx * dy;
        sxx += dx * dx;
        syy += dy * dy;
    }
    double c = sxy / sqrt(sxx * syy);
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    *flag_out = 0;
    *c64_out = c;

    if (J->dtype == OR_F32) {
        *c32_out = (float)c;
        return;
    }

    /* Integers: the same two passes in exact arithmetic.  With the sums
     * Sx, Sy, the scaled deviations d_i = n*x_i - Sx and e_i = n*y_i - Sy are
     * integers, and P/sqrt(Q*R) with P = sum d*e, Q = sum d^2, R = sum e^2 is
     * exactly the coefficient of the formula. */
    int64_t Sx = 0, Sy = 0;
    for (int64_t i = 0; i < n; i++) {
        Sx += load_as_int(J->x, J->dtype, ix[i]);
        Sy += load_as_int(J->y, J->dtype, ix[i]);
    }
    __int128 P = 0;
    unsigned __int128 Q = 0, R = 0;
    for (int64_t i = 0; i < n; i++) {
        __int128 d = (__int128)n * load_as_int(J->x, J->dtype, ix[i]) - Sx;
        __int128 e = (__int128)n * load_as_int(J->y, J->dtype, ix[i]) - Sy;
        P += d * e;
        Q += (unsigned __int128)(d * d);
        R += (unsigned __int128)(e * e);
    }
    *c32_out = rn32_of_ratio(P, Q, R);
}

/* ------------------------------------------------------------------------ */
/* Entry points                                                              */
/* ------------------------------------------------------------------------ */

static int setup(job_t *J, int ndim, const int64_t *shape, const int32_t *window,
                 const int32_t *step, int border, int dtype, double invalid,
                 double missing_le, const void *x, const void *y)
{
    if (!x || !y) return -1;
    if (dtype < OR_U8 || dtype > OR_F32) return -1;
    if (oracle_output_shape(ndim, shape, window, step, border, J->oshape) != 0) return -1;
    J->ndim = ndim;
    for (int d = 0; d < 3; d++) {
        J->shape[d] = d < ndim ? shape[d] : 1;
        J->window[d] = d < ndim ? window[d] : 1;
        J->step[d] = d < ndim ? step[d] : 1;
        if (d >= ndim) J->oshape[d] = 1;
    }
    J->border = border;
    J->dtype = dtype;
    J->invalid = invalid;
    J->missing_le = missing_le;
    J->x = x;
    J->y = y;
    return 0;
}

static int64_t window_cap(const job_t *J)
{
    int64_t cap = 1;
    for (int d = 0; d < J->ndim; d++) cap *= J->window[d];
    return cap;
}

/* Evaluate either every output (idx == NULL; count ignored; outputs in C
 * order of the output shape) or the listed flat output indices.  Outputs:
 * c64 (FP64 two-pass value, or `invalid`), c32 (float32: exact RN32 for
 * integer input, (float)c64 for float input) and flags.  Returns 0, -1 on bad
 * arguments, -2 on allocation failure. */
int oracle_corr(int ndim, const int64_t *shape, const int32_t *window,
                const int32_t *step, int border, int dtype, double invalid,
                double missing_le, const void *x, const void *y,
                const int64_t *idx, int64_t count, double *c64, float *c32,
                uint8_t *flags, int nthreads)
{
    job_t J;
    if (setup(&J, ndim, shape, window, step, border, dtype, invalid, missing_le, x, y))
        return -1;
    int64_t total = J.oshape[0] * J.oshape[1] * J.oshape[2];
    if (idx) {
        for (int64_t i = 0; i < count; i++)
            if (idx[i] < 0 || idx[i] >= total) return -1;
    } else {
        count = total;
    }
    int64_t cap = window_cap(&J);
    int failed = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double *xs = (double *)malloc(sizeof(double) * cap);
        double *ys = (double *)malloc(sizeof(double) * cap);
        int64_t *ix = (int64_t *)malloc(sizeof(int64_t) * cap);
        if (!xs || !ys || !ix) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < count; i++) {
                int64_t o = idx ? idx[i] : i;
                eval_one(&J, o, xs, ys, ix, &c64[i], &c32[i], &flags[i]);
            }
        }
        free(xs);
        free(ys);
        free(ix);
    }
    return failed ? -2 : 0;
}

/* Exact RN32 of P/sqrt(Q*R) for given 64-bit operands (exposed for tests of
 * the rounding step on constructed near-midpoint cases). */
float oracle_rn32_ratio(int64_t P, uint64_t Q, uint64_t R)
{
    return rn32_of_ratio((__int128)P, (unsigned __int128)Q, (unsigned __int128)R);
}

int oracle_has_openmp(void)
{
#ifdef _OPENMP
    return 1;
#else
    return 0;
#endif
}
