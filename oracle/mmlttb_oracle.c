/*
 * MinMaxLTTB reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar CPU statement of what the MinMaxLTTB downsampling
 * path computes (Van Der Donckt, Van Der Donckt, Rademaker, Van Hoecke,
 * "MinMaxLTTB: Leveraging MinMax-Preselection to Scale LTTB", 2023).
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library. The GPU library never links it, and the two share no
 * code, header, table or helper.
 *
 * Build: gcc -O2 -ffp-contract=off -std=c11 -shared -fPIC, no fast-math.
 * On x86-64 every `double` operation below is then one IEEE-754 binary64
 * operation rounded to nearest-even, with no fused multiply-add.
 *
 * What the paper fixes:
 *   - MinMax keeps, per bin, the points holding the minimum and the maximum
 *     of y (section 2.2.1, Table 1).
 *   - LTTB keeps, per bucket, the point spanning the largest triangle with
 *     the point kept in the previous bucket and the mean (x, y) of the next
 *     bucket; first and last points are kept (section 2.2.1, Fig. 3).
 *   - MinMaxLTTB preselects r_ps * n_out points with MinMax, r_ps >= 2 an
 *     integer, r_ps/2 min-max sub-buckets per LTTB bucket, adds the first and
 *     last points, and runs LTTB on that set only (section 3).
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes and pinned by a test):
 *   R1  number of MinMax bins nb = floor(n_out * r_ps / 2).
 *   R2  MinMax bins cover the interior [1, n-1) with equal-index integer
 *       boundaries 1 + floor(b * (n-2) / nb); empty bins are skipped.
 *   R3  min and max ties go to the lowest index; values compare as IEEE
 *       numbers (so -0.0 == +0.0); a bin whose min and max point coincide
 *       contributes one index.
 *   R4  the preselection P is the sorted distinct set {0, n-1} + all
 *       per-bin argmin/argmax indices; LTTB then runs as plain LTTB over P
 *       (sub-bucket alignment is not enforced).
 *   R5  LTTB buckets: n_out-2 interior buckets over positions [1, m-1) with
 *       boundaries 1 + floor(k * (m-2) / (n_out-2)).
 *   R6  next-bucket mean: exact sum of the raw x (integers) and of y
 *       (float32), each rounded once to binary64, then divided by the count
 *       with one binary64 division. The last interior bucket uses the last
 *       point alone.
 *   R7  area (doubled, the 1/2 is dropped):
 *         |(Xa - MX) * (Yj - Ya) - (Xa - Xj) * (MY - Ya)|
 *       in binary64, each operation rounded separately, in this order.
 *       X = x rounded to binary64 (x implicit: the index), Y = y widened.
 *   R8  area ties go to the lowest index.
 *   R9  n <= n_out returns every index; n < 1, n_out < 3 or r_ps < 2 is an
 *       argument error. No other short-circuit: P is always computed.
 *   R10 y must be finite; the oracle refuses non-finite input.
 *
 * The other downsamplers of Table 1, on the same building blocks:
 *   R11 MinMax alone is the preselection with r_ps = 1 (section 3 footnote:
 *       MinMaxLTTB with r_ps = 1 corresponds to MinMax aggregation):
 *       floor(n_out / 2) interior bins plus the first and last points.
 *   R12 M4 keeps per bin the first, the last, the lowest-index minimum and
 *       the lowest-index maximum (section 2.2.1); floor(n_out / 4)
 *       equal-index bins over all points, part b = [floor(b n / nb),
 *       floor((b+1) n / nb)); output sorted distinct; n <= n_out keeps
 *       every index; n < 1 or n_out < 4 is an argument error.
 *   R13 EveryNth keeps n_out evenly spaced indices floor(k n / n_out),
 *       k = 0..n_out-1 (section 2.2.1); n <= n_out keeps every index;
 *       n < 1 or n_out < 1 is an argument error.
 *
 * Bins equal in x (a variant for irregular timestamps; a bin has edges, Fig. 3):
 *   R14 x int64, strictly increasing. The interior points 1..n-2 fall into nb
 *       bins of equal x width: edges e_b = x_1 + floor(b (x_{n-1} - x_1) / nb),
 *       b = 0..nb, and point i is in bin b when e_b <= x_i < e_{b+1}. For
 *       x_i = i this is the equal-index binning of R2. Extrema, ties and P as
 *       R3-R4; bins may be empty (gaps in x), so P may hold n_out points or
 *       fewer; LTTB then keeps every point of P (R9 applied to P). The output
 *       count is min(m, n_out) when n > n_out, else n.
 *
 * Other value types (same definitions, other storage):
 *   R15 y may be float32, binary64 or int32; x may be implicit, int64 or
 *       binary64. Values compare as numbers (-0.0 == +0.0). Y = y converted
 *       to binary64 (exact for all three). X = x for binary64 x, x rounded to
 *       binary64 for int64 x. Next-bucket means: the exact sum of the raw
 *       values (x as stored; y as its exact binary64 value) rounded once to
 *       binary64, then one division by the count (R6); a sum beyond the
 *       binary64 range rounds to an infinity. binary64 x and y must be finite.
 *       An area that is not a number (possible only when such a sum
 *       overflowed) never wins; a bucket with no numeric area keeps its first
 *       point.
 *
 * MinMax preselection in front of other line simplifiers (section 4 names
 * Visvalingam-Whyatt, Douglas-Peucker and Longest-Line-Bucket as future work
 * without defining them; these are their standard forms, run on P exactly as
 * LTTB is, X and Y binary64 as in R7). m > n_out points in, n_out out; m <=
 * n_out keeps every point.
 *   R16 VW: while more than n_out points remain, remove the interior point
 *       whose doubled triangle area with its current neighbours a < j < b,
 *       |(Xa - Xb)(Yj - Ya) - (Xa - Xj)(Yb - Ya)|, is smallest (lowest index
 *       on ties), then recompute the areas of its two neighbours.
 *   R17 DP with a point budget: start from {first, last}; the farthest point
 *       of a segment a < j < b of consecutive kept points maximises
 *       |(Xb - Xa)(Yj - Ya) - (Xj - Xa)(Yb - Ya)| (lowest index on ties) and
 *       its key is c * c / ((Xb - Xa)^2 + (Yb - Ya)^2) for that value c, the
 *       squared distance to the chord, in this operation order (a key that
 *       is not a number, from a chord of zero length, counts as -1); while
 *       fewer than n_out points are kept, keep the farthest point of the
 *       segment with the largest key (the lowest such point on ties).
 *   R18 LLB: LTTB's buckets (R5); one point per bucket, first and last
 *       fixed, maximising the total length of the polyline, sum of
 *       sqrt((Xj - Xi)^2 + (Yj - Yi)^2) taken bucket by bucket in order; by
 *       dynamic programming over the buckets, each point keeping the lowest
 *       index among the predecessors that give the largest total (strict >).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOTFINITE (-5)
#define ORC_ENOMEM (-6)

#define XK_IMPLICIT 0
#define XK_INT64 1
#define XK_F64 2

#define YK_F32 0
#define YK_F64 1
#define YK_I32 2

/* ------------------------------------------------------------------------ */
/* Exact sums, rounded once to binary64 (reading R6).                        */
/* A big unsigned integer, 32-bit words, least significant word first.       */
/* ------------------------------------------------------------------------ */

/* float32 sums need < 2^(277+64): 16 words; binary64 sums need
 * < 2^(2098+64): 72 words. */
#define BIG_WORDS_F32 16
#define BIG_WORDS 72

typedef struct {
    uint32_t w[BIG_WORDS];
    int nw; /* words in use */
} big_t;

static void big_zero(big_t *a, int nw)
{
    memset(a, 0, sizeof(*a));
    a->nw = nw;
}

/* a += v << shift, for v < 2^32 */
static void big_add_u32_shifted(big_t *a, uint32_t v, int shift)
{
    int word = shift / 32;
    int bit = shift % 32;
    uint64_t wide = (uint64_t)v << bit; /* < 2^63 */
    uint64_t carry = 0;
    for (int i = word; i < a->nw; i++) {
        uint64_t add = 0;
        if (i == word)
            add = wide & 0xffffffffu;
        else if (i == word + 1)
            add = wide >> 32;
        uint64_t s = (uint64_t)a->w[i] + add + carry;
        a->w[i] = (uint32_t)s;
        carry = s >> 32;
    }
}

static int big_cmp(const big_t *a, const big_t *b)
{
    for (int i = a->nw - 1; i >= 0; i--) {
        if (a->w[i] != b->w[i])
            return a->w[i] < b->w[i] ? -1 : 1;
    }
    return 0;
}

/* r = a - b, requires a >= b */
static void big_sub(big_t *r, const big_t *a, const big_t *b)
{
    int64_t borrow = 0;
    r->nw = a->nw;
    for (int i = 0; i < a->nw; i++) {
        int64_t d = (int64_t)a->w[i] - (int64_t)b->w[i] - borrow;
        borrow = 0;
        if (d < 0) {
            d += (int64_t)1 << 32;
            borrow = 1;
        }
        r->w[i] = (uint32_t)d;
    }
}

static int big_bit(const big_t *a, int i) { return (int)((a->w[i / 32] >> (i % 32)) & 1u); }

/* The binary64 nearest to (negative ? -1 : 1) * a * 2^scale_exp, ties to
 * even. An a below 2^53 is converted exactly (with scale_exp = -1074 this
 * covers every subnormal result); larger ones keep 53 bits with round and
 * sticky bits, so the result is normal or overflows to an infinity. */
static double big_round_to_double(const big_t *a, int scale_exp, int negative)
{
    int top = -1;
    for (int i = a->nw * 32 - 1; i >= 0; i--) {
        if (big_bit(a, i)) {
            top = i;
            break;
        }
    }
    if (top < 0)
        return 0.0;
    uint64_t mant = 0;
    int low; /* weight (bit position) of the mantissa's last kept bit */
    if (top <= 52) {
        for (int i = top; i >= 0; i--)
            mant = (mant << 1) | (uint64_t)big_bit(a, i);
        low = 0;
    } else {
        low = top - 52;
        for (int i = top; i >= low; i--)
            mant = (mant << 1) | (uint64_t)big_bit(a, i);
        int round_bit = big_bit(a, low - 1);
        int sticky = 0;
        for (int i = low - 2; i >= 0; i--)
            sticky |= big_bit(a, i);
        if (round_bit && (sticky || (mant & 1u)))
            mant += 1; /* may reach 2^53: still exact in binary64 */
    }
    double r = ldexp((double)mant, low + scale_exp);
    return negative ? -r : r;
}

/* RN(sum of v[0..c-1]) with the sum taken exactly. Every finite float32 is
 * an integer multiple of 2^-149 of magnitude below 2^128, so the sum is an
 * integer count of 2^-149 units; positive and negative parts are kept apart. */
static double exact_sum_f32(const float *v, int64_t c)
{
    big_t pos, neg;
    big_zero(&pos, BIG_WORDS_F32);
    big_zero(&neg, BIG_WORDS_F32);
    for (int64_t i = 0; i < c; i++) {
        uint32_t bits;
        memcpy(&bits, &v[i], 4);
        uint32_t expo = (bits >> 23) & 0xffu;
        uint32_t frac = bits & 0x7fffffu;
        uint32_t mant;
        int shift;
        if (expo == 0) { /* zero or subnormal: frac * 2^-149 */
            mant = frac;
            shift = 0;
        } else { /* normal: (2^23 + frac) * 2^(expo - 150) */
            mant = frac | 0x800000u;
            shift = (int)expo - 1;
        }
        if (bits >> 31)
            big_add_u32_shifted(&neg, mant, shift);
        else
            big_add_u32_shifted(&pos, mant, shift);
    }
    big_t mag;
    int negative = 0;
    if (big_cmp(&pos, &neg) >= 0) {
        big_sub(&mag, &pos, &neg);
    } else {
        big_sub(&mag, &neg, &pos);
        negative = 1;
    }
    return big_round_to_double(&mag, -149, negative);
}

/* RN(sum of x[0..c-1]) with the sum taken exactly in 128-bit integers. */
static double exact_sum_i64(const int64_t *x, int64_t c)
{
    __int128 s = 0;
    for (int64_t i = 0; i < c; i++)
        s += (__int128)x[i];
    int negative = s < 0;
    unsigned __int128 mag = negative ? (unsigned __int128)(-s) : (unsigned __int128)s;
    big_t a;
    big_zero(&a, 4);
    for (int i = 0; i < 4; i++)
        a.w[i] = (uint32_t)(mag >> (32 * i));
    return big_round_to_double(&a, 0, negative);
}

/* RN(sum of v[0..c-1]) for finite binary64 values, the sum taken exactly.
 * Every finite binary64 is an integer multiple of 2^-1074 below 2^1024; the
 * significand (< 2^53) is added as two 32-bit pieces. A sum beyond the
 * binary64 range rounds to an infinity, as IEEE rounding to nearest does. */
static double exact_sum_f64(const double *v, int64_t c)
{
    big_t pos, neg;
    big_zero(&pos, BIG_WORDS);
    big_zero(&neg, BIG_WORDS);
    for (int64_t i = 0; i < c; i++) {
        uint64_t bits;
        memcpy(&bits, &v[i], 8);
        uint32_t expo = (uint32_t)((bits >> 52) & 0x7ffu);
        uint64_t frac = bits & 0xfffffffffffffull;
        uint64_t mant;
        int shift;
        if (expo == 0) { /* zero or subnormal: frac * 2^-1074 */
            mant = frac;
            shift = 0;
        } else { /* normal: (2^52 + frac) * 2^(expo - 1075) */
            mant = frac | (1ull << 52);
            shift = (int)expo - 1;
        }
        big_t *dst = (bits >> 63) ? &neg : &pos;
        big_add_u32_shifted(dst, (uint32_t)(mant & 0xffffffffu), shift);
        big_add_u32_shifted(dst, (uint32_t)(mant >> 32), shift + 32);
    }
    big_t mag;
    int negative = 0;
    if (big_cmp(&pos, &neg) >= 0) {
        big_sub(&mag, &pos, &neg);
    } else {
        big_sub(&mag, &neg, &pos);
        negative = 1;
    }
    return big_round_to_double(&mag, -1074, negative);
}

/* ------------------------------------------------------------------------ */
/* Boundaries                                                               */
/* ------------------------------------------------------------------------ */

/* floor(k * len / parts), exact */
static int64_t floor_frac(int64_t k, int64_t len, int64_t parts)
{
    return (int64_t)(((__int128)k * (__int128)len) / (__int128)parts);
}

static int is_finite_f32(float v) { return isfinite(v); }

/* ------------------------------------------------------------------------ */
/* MinMax preselection (section 2.2.1 MinMax; section 3 step (i); R1-R4).    */
/* ------------------------------------------------------------------------ */

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Writes the sorted distinct preselection into P (capacity 2*nb+2) and its
 * size into *m. r_ps = 1 gives the MinMax downsampler (R11). */
int oracle_minmax(const float *y, int64_t n, int64_t n_out, int32_t r_ps, int64_t *P, int64_t *m)
{
    if (n < 1 || n_out < 3 || r_ps < 1)
        return ORC_EINVAL;
    int64_t bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : bad)
#endif
    for (int64_t i = 0; i < n; i++)
        if (!is_finite_f32(y[i]))
            bad = 1;
    if (bad)
        return ORC_ENOTFINITE;
    int64_t cnt = 0;
    if (n <= 2) {
        for (int64_t i = 0; i < n; i++)
            P[cnt++] = i;
        *m = cnt;
        return ORC_OK;
    }
    int64_t nb = (int64_t)(((__int128)n_out * r_ps) / 2); /* R1 */
    int64_t L = n - 2;
    /* Per-bin argmin and argmax first (-1 marks an empty bin), then P in bin
     * order. The bins are independent: this is the loop the paper runs in
     * parallel (section 3.2); a build with -fopenmp spreads it over all cores,
     * with the same result. */
    int64_t *bmin = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
    int64_t *bmax = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
    if (!bmin || !bmax) {
        free(bmin);
        free(bmax);
        return ORC_ENOMEM;
    }
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t b = 0; b < nb; b++) {
        int64_t lo = 1 + floor_frac(b, L, nb); /* R2 */
        int64_t hi = 1 + floor_frac(b + 1, L, nb);
        int64_t imin = -1, imax = -1;
        if (lo < hi) {
            imin = lo;
            imax = lo;
            for (int64_t i = lo + 1; i < hi; i++) {
                if (y[i] < y[imin]) /* strict: lowest index wins ties (R3) */
                    imin = i;
                if (y[i] > y[imax])
                    imax = i;
            }
        }
        bmin[b] = imin;
        bmax[b] = imax;
    }
    P[cnt++] = 0;
    for (int64_t b = 0; b < nb; b++) {
        if (bmin[b] < 0) /* empty bin */
            continue;
        P[cnt++] = bmin[b];
        if (bmax[b] != bmin[b])
            P[cnt++] = bmax[b];
    }
    free(bmin);
    free(bmax);
    P[cnt++] = n - 1;
    qsort(P, (size_t)cnt, sizeof(int64_t), cmp_i64);
    int64_t d = 0;
    for (int64_t i = 0; i < cnt; i++)
        if (d == 0 || P[i] != P[d - 1])
            P[d++] = P[i];
    *m = d;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* LTTB over a point sequence (section 2.2.1 LTTB, Fig. 3; R5-R8).            */
/* xs: raw integer abscissae of the m points, ys: their ordinates.           */
/* ------------------------------------------------------------------------ */

/* Next-bucket means for every interior bucket k = 0..B-1 (R6). */
static void lttb_means(const int64_t *xs, const float *ys, int64_t m, int64_t n_out, double *MX, double *MY)
{
    int64_t B = n_out - 2;
    for (int64_t k = 0; k < B; k++) {
        int64_t g0, g1;
        if (k < B - 1) {
            g0 = 1 + floor_frac(k + 1, m - 2, B);
            g1 = 1 + floor_frac(k + 2, m - 2, B);
        } else {
            g0 = m - 1;
            g1 = m;
        }
        double c = (double)(g1 - g0);
        MX[k] = exact_sum_i64(xs + g0, g1 - g0) / c;
        MY[k] = exact_sum_f32(ys + g0, g1 - g0) / c;
    }
}

/* Selected positions (0..m-1) into out[0..min(m, n_out)-1]. */
static int lttb_positions(const int64_t *xs, const float *ys, int64_t m, int64_t n_out, int64_t *out)
{
    if (m <= n_out) {
        for (int64_t i = 0; i < m; i++)
            out[i] = i;
        return ORC_OK;
    }
    int64_t B = n_out - 2;
    double *MX = (double *)malloc(sizeof(double) * (size_t)B);
    double *MY = (double *)malloc(sizeof(double) * (size_t)B);
    if (!MX || !MY) {
        free(MX);
        free(MY);
        return ORC_ENOMEM;
    }
    lttb_means(xs, ys, m, n_out, MX, MY);
    int64_t a = 0;
    out[0] = 0;
    for (int64_t k = 0; k < B; k++) {
        int64_t s0 = 1 + floor_frac(k, m - 2, B); /* R5 */
        int64_t s1 = 1 + floor_frac(k + 1, m - 2, B);
        double Xa = (double)xs[a];
        double Ya = (double)ys[a];
        double best = -1.0; /* every area is >= 0 */
        int64_t sel = -1;
        for (int64_t j = s0; j < s1; j++) {
            double Xj = (double)xs[j];
            double Yj = (double)ys[j];
            double area = fabs((Xa - MX[k]) * (Yj - Ya) - (Xa - Xj) * (MY[k] - Ya)); /* R7 */
            if (area > best) { /* strict: lowest index wins ties (R8) */
                best = area;
                sel = j;
            }
        }
        out[k + 1] = sel;
        a = sel;
    }
    out[n_out - 1] = m - 1;
    free(MX);
    free(MY);
    return ORC_OK;
}

static int64_t *abscissae(int xk, const int64_t *x, int64_t n)
{
    int64_t *xs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!xs)
        return NULL;
    for (int64_t i = 0; i < n; i++)
        xs[i] = (xk == XK_INT64) ? x[i] : i;
    return xs;
}

static int check_x(int xk, const int64_t *x)
{
    if (xk == XK_IMPLICIT)
        return x == NULL ? ORC_OK : ORC_EINVAL;
    if (xk == XK_INT64)
        return x != NULL ? ORC_OK : ORC_EINVAL;
    return ORC_EINVAL;
}

/* Plain LTTB on all n points; out holds min(n, n_out) indices. */
int oracle_lttb(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int64_t *out)
{
    if (n < 1 || n_out < 3 || check_x(xk, x) != ORC_OK)
        return ORC_EINVAL;
    for (int64_t i = 0; i < n; i++)
        if (!is_finite_f32(y[i]))
            return ORC_ENOTFINITE;
    int64_t *xs = abscissae(xk, x, n);
    if (!xs)
        return ORC_ENOMEM;
    int rc = lttb_positions(xs, y, n, n_out, out);
    free(xs);
    return rc;
}

/* MinMaxLTTB (section 3): MinMax preselection, then LTTB on the preselected
 * points only; out holds min(n, n_out) indices into the original series. */
int oracle_minmaxlttb(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps, int64_t *out)
{
    if (n < 1 || n_out < 3 || r_ps < 2 || check_x(xk, x) != ORC_OK)
        return ORC_EINVAL;
    if (n <= n_out) {
        for (int64_t i = 0; i < n; i++)
            if (!is_finite_f32(y[i]))
                return ORC_ENOTFINITE;
        for (int64_t i = 0; i < n; i++)
            out[i] = i;
        return ORC_OK;
    }
    int64_t nb = (int64_t)(((__int128)n_out * r_ps) / 2);
    int64_t cap = 2 * nb + 2;
    int64_t *P = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    if (!P)
        return ORC_ENOMEM;
    int64_t m = 0;
    int rc = oracle_minmax(y, n, n_out, r_ps, P, &m);
    if (rc != ORC_OK) {
        free(P);
        return rc;
    }
    int64_t *xs = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    float *ys = (float *)malloc(sizeof(float) * (size_t)m);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_out);
    if (!xs || !ys || !pos) {
        free(P);
        free(xs);
        free(ys);
        free(pos);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < m; i++) {
        xs[i] = (xk == XK_INT64) ? x[P[i]] : P[i];
        ys[i] = y[P[i]];
    }
    rc = lttb_positions(xs, ys, m, n_out, pos);
    if (rc == ORC_OK) {
        int64_t cnt = m < n_out ? m : n_out;
        for (int64_t i = 0; i < cnt; i++)
            out[i] = P[pos[i]];
    }
    free(P);
    free(xs);
    free(ys);
    free(pos);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* MinMax bins equal in x (R14).                                              */
/* ------------------------------------------------------------------------ */

/* Edge b of nb equal x-width bins over [x1, xlast]. */
static int64_t x_edge(int64_t x1, int64_t xlast, int64_t b, int64_t nb)
{
    __int128 span = (__int128)xlast - (__int128)x1;
    return (int64_t)((__int128)x1 + (span * b) / nb);
}

int oracle_minmax_xbins(const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps, int64_t *P,
                        int64_t *m)
{
    if (n < 1 || n_out < 3 || r_ps < 1 || !x)
        return ORC_EINVAL;
    for (int64_t i = 0; i < n; i++)
        if (!is_finite_f32(y[i]))
            return ORC_ENOTFINITE;
    for (int64_t i = 1; i < n; i++)
        if (x[i] <= x[i - 1])
            return ORC_EINVAL;
    int64_t cnt = 0;
    if (n <= 2) {
        for (int64_t i = 0; i < n; i++)
            P[cnt++] = i;
        *m = cnt;
        return ORC_OK;
    }
    int64_t nb = (int64_t)(((__int128)n_out * r_ps) / 2); /* R1, R14 */
    P[cnt++] = 0;
    int64_t lo = 1; /* first interior point with x >= the current bin's left edge */
    for (int64_t b = 0; b < nb; b++) {
        int64_t right = x_edge(x[1], x[n - 1], b + 1, nb);
        int64_t hi = lo;
        while (hi < n - 1 && x[hi] < right)
            hi++;
        if (hi > lo) {
            int64_t imin = lo, imax = lo;
            for (int64_t i = lo + 1; i < hi; i++) {
                if (y[i] < y[imin]) /* lowest index on ties (R14, R3) */
                    imin = i;
                if (y[i] > y[imax]) /* lowest index on ties (R14, R3) */
                    imax = i;
            }
            P[cnt++] = imin;
            if (imax != imin)
                P[cnt++] = imax;
        }
        lo = hi;
    }
    P[cnt++] = n - 1;
    qsort(P, (size_t)cnt, sizeof(int64_t), cmp_i64);
    int64_t d = 0;
    for (int64_t i = 0; i < cnt; i++)
        if (d == 0 || P[i] != P[d - 1])
            P[d++] = P[i];
    *m = d;
    return ORC_OK;
}

/* out: capacity n_out (or n when n <= n_out); *count = entries written. */
int oracle_minmaxlttb_xbins(const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps, int64_t *out,
                            int64_t *count)
{
    if (n < 1 || n_out < 3 || r_ps < 2 || !x)
        return ORC_EINVAL;
    if (n <= n_out) {
        for (int64_t i = 0; i < n; i++)
            if (!is_finite_f32(y[i]))
                return ORC_ENOTFINITE;
        for (int64_t i = 1; i < n; i++)
            if (x[i] <= x[i - 1])
                return ORC_EINVAL;
        for (int64_t i = 0; i < n; i++)
            out[i] = i;
        *count = n;
        return ORC_OK;
    }
    int64_t nb = (int64_t)(((__int128)n_out * r_ps) / 2);
    int64_t *P = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * nb + 2));
    if (!P)
        return ORC_ENOMEM;
    int64_t m = 0;
    int rc = oracle_minmax_xbins(x, y, n, n_out, r_ps, P, &m);
    if (rc != ORC_OK) {
        free(P);
        return rc;
    }
    int64_t *xs = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    float *ys = (float *)malloc(sizeof(float) * (size_t)m);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m < n_out ? m : n_out));
    if (!xs || !ys || !pos) {
        free(P);
        free(xs);
        free(ys);
        free(pos);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < m; i++) {
        xs[i] = x[P[i]];
        ys[i] = y[P[i]];
    }
    rc = lttb_positions(xs, ys, m, n_out, pos);
    if (rc == ORC_OK) {
        int64_t c = m < n_out ? m : n_out;
        for (int64_t i = 0; i < c; i++)
            out[i] = P[pos[i]];
        *count = c;
    }
    free(P);
    free(xs);
    free(ys);
    free(pos);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Other value types (R15).                                                  */
/* ------------------------------------------------------------------------ */

static double y_value(int yk, const void *y, int64_t i)
{
    if (yk == YK_F32)
        return (double)((const float *)y)[i];
    if (yk == YK_F64)
        return ((const double *)y)[i];
    return (double)((const int32_t *)y)[i];
}

/* y_i < y_j as numbers; every y type fits binary64 exactly, so comparing the
 * binary64 values compares the stored ones. */
static int y_less(int yk, const void *y, int64_t i, int64_t j) { return y_value(yk, y, i) < y_value(yk, y, j); }

static int check_typed(int xk, const void *x, int yk, const void *y, int64_t n)
{
    if (yk != YK_F32 && yk != YK_F64 && yk != YK_I32)
        return ORC_EINVAL;
    if (xk == XK_IMPLICIT ? x != NULL : (xk == XK_INT64 || xk == XK_F64) ? x == NULL : 1)
        return ORC_EINVAL;
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(y_value(yk, y, i)))
            return ORC_ENOTFINITE;
    if (xk == XK_F64)
        for (int64_t i = 0; i < n; i++)
            if (!isfinite(((const double *)x)[i]))
                return ORC_ENOTFINITE;
    return ORC_OK;
}

int oracle_minmax_typed(int yk, const void *y, int64_t n, int64_t n_out, int32_t r_ps, int64_t *P, int64_t *m)
{
    if (n < 1 || n_out < 3 || r_ps < 1)
        return ORC_EINVAL;
    int rc = check_typed(XK_IMPLICIT, NULL, yk, y, n);
    if (rc != ORC_OK)
        return rc;
    int64_t cnt = 0;
    if (n <= 2) {
        for (int64_t i = 0; i < n; i++)
            P[cnt++] = i;
        *m = cnt;
        return ORC_OK;
    }
    int64_t nb = (int64_t)(((__int128)n_out * r_ps) / 2); /* R1, R15 */
    int64_t L = n - 2;
    P[cnt++] = 0;
    for (int64_t b = 0; b < nb; b++) {
        int64_t lo = 1 + floor_frac(b, L, nb);
        int64_t hi = 1 + floor_frac(b + 1, L, nb);
        if (lo == hi)
            continue;
        int64_t imin = lo, imax = lo;
        for (int64_t i = lo + 1; i < hi; i++) {
            if (y_less(yk, y, i, imin)) /* lowest index on ties (R15, R3) */
                imin = i;
            if (y_less(yk, y, imax, i)) /* lowest index on ties (R15, R3) */
                imax = i;
        }
        P[cnt++] = imin;
        if (imax != imin)
            P[cnt++] = imax;
    }
    P[cnt++] = n - 1;
    qsort(P, (size_t)cnt, sizeof(int64_t), cmp_i64);
    int64_t d = 0;
    for (int64_t i = 0; i < cnt; i++)
        if (d == 0 || P[i] != P[d - 1])
            P[d++] = P[i];
    *m = d;
    return ORC_OK;
}

/* Next-bucket means over m > n_out points (R6 with R15): exact sums of xi
 * (int64 x) or xf (binary64 x), and of Y. */
static void lttb_means_typed(const int64_t *xi, const double *xf, const double *Y, int64_t m, int64_t n_out,
                             double *MX, double *MY)
{
    int64_t B = n_out - 2;
    for (int64_t k = 0; k < B; k++) {
        int64_t g0, g1;
        if (k < B - 1) {
            g0 = 1 + floor_frac(k + 1, m - 2, B);
            g1 = 1 + floor_frac(k + 2, m - 2, B);
        } else {
            g0 = m - 1;
            g1 = m;
        }
        double c = (double)(g1 - g0);
        MX[k] = (xi ? exact_sum_i64(xi + g0, g1 - g0) : exact_sum_f64(xf + g0, g1 - g0)) / c;
        MY[k] = exact_sum_f64(Y + g0, g1 - g0) / c;
    }
}

/* LTTB positions over m points (R5-R8 with R15): X, Y are the binary64
 * coordinates; the means sum xi (int64 x) or xf (binary64 x) and Y exactly. */
static int lttb_positions_typed(const double *X, const int64_t *xi, const double *xf, const double *Y, int64_t m,
                                int64_t n_out, int64_t *out)
{
    if (m <= n_out) {
        for (int64_t i = 0; i < m; i++)
            out[i] = i;
        return ORC_OK;
    }
    int64_t B = n_out - 2;
    double *MX = (double *)malloc(sizeof(double) * (size_t)B);
    double *MY = (double *)malloc(sizeof(double) * (size_t)B);
    if (!MX || !MY) {
        free(MX);
        free(MY);
        return ORC_ENOMEM;
    }
    lttb_means_typed(xi, xf, Y, m, n_out, MX, MY);
    int64_t a = 0;
    out[0] = 0;
    for (int64_t k = 0; k < B; k++) {
        int64_t s0 = 1 + floor_frac(k, m - 2, B);
        int64_t s1 = 1 + floor_frac(k + 1, m - 2, B);
        double best = -1.0;
        int64_t sel = s0; /* kept when no area is a number (R15) */
        for (int64_t j = s0; j < s1; j++) {
            double area = fabs((X[a] - MX[k]) * (Y[j] - Y[a]) - (X[a] - X[j]) * (MY[k] - Y[a])); /* R7 */
            if (area > best) { /* lowest index on ties (R8) */
                best = area;
                sel = j;
            }
        }
        out[k + 1] = sel;
        a = sel;
    }
    out[n_out - 1] = m - 1;
    free(MX);
    free(MY);
    return ORC_OK;
}

int oracle_minmaxlttb_typed(int xk, const void *x, int yk, const void *y, int64_t n, int64_t n_out, int32_t r_ps,
                            int64_t *out)
{
    if (n < 1 || n_out < 3 || r_ps < 2)
        return ORC_EINVAL;
    int rc = check_typed(xk, x, yk, y, n);
    if (rc != ORC_OK)
        return rc;
    if (n <= n_out) {
        for (int64_t i = 0; i < n; i++)
            out[i] = i;
        return ORC_OK;
    }
    int64_t nb = (int64_t)(((__int128)n_out * r_ps) / 2);
    int64_t *P = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * nb + 2));
    if (!P)
        return ORC_ENOMEM;
    int64_t m = 0;
    rc = oracle_minmax_typed(yk, y, n, n_out, r_ps, P, &m);
    double *X = (double *)malloc(sizeof(double) * (size_t)m);
    double *Y = (double *)malloc(sizeof(double) * (size_t)m);
    int64_t *xi = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    double *xf = (double *)malloc(sizeof(double) * (size_t)m);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_out);
    if (rc == ORC_OK && (!X || !Y || !xi || !xf || !pos))
        rc = ORC_ENOMEM;
    if (rc == ORC_OK) {
        for (int64_t i = 0; i < m; i++) {
            int64_t p = P[i];
            if (xk == XK_F64) {
                xf[i] = ((const double *)x)[p];
                X[i] = xf[i];
            } else {
                xi[i] = (xk == XK_INT64) ? ((const int64_t *)x)[p] : p;
                X[i] = (double)xi[i];
            }
            Y[i] = y_value(yk, y, p);
        }
        rc = lttb_positions_typed(X, xk == XK_F64 ? NULL : xi, xf, Y, m, n_out, pos);
        if (rc == ORC_OK)
            for (int64_t i = 0; i < n_out; i++)
                out[i] = P[pos[i]];
    }
    free(P);
    free(X);
    free(Y);
    free(xi);
    free(xf);
    free(pos);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Other simplifiers on the preselected points (R16-R18).                    */
/* X, Y: binary64 coordinates of m points; out: n_out positions (m > n_out). */
/* ------------------------------------------------------------------------ */

static double vw_area(const double *X, const double *Y, int64_t a, int64_t j, int64_t b)
{
    return fabs((X[a] - X[b]) * (Y[j] - Y[a]) - (X[a] - X[j]) * (Y[b] - Y[a])); /* R16 */
}

static int vw_positions(const double *X, const double *Y, int64_t m, int64_t n_out, int64_t *out)
{
    int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    double *area = (double *)malloc(sizeof(double) * (size_t)m);
    char *alive = (char *)malloc((size_t)m);
    if (!prev || !next || !area || !alive) {
        free(prev);
        free(next);
        free(area);
        free(alive);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < m; i++) {
        prev[i] = i - 1;
        next[i] = i + 1;
        alive[i] = 1;
    }
    for (int64_t i = 1; i < m - 1; i++)
        area[i] = vw_area(X, Y, i - 1, i, i + 1);
    /* plain scan for the smallest area each time: slow and obviously right */
    for (int64_t left = m; left > n_out; left--) {
        int64_t sel = -1;
        for (int64_t i = 1; i < m - 1; i++)
            if (alive[i] && (sel < 0 || area[i] < area[sel])) /* lowest index on ties (R16) */
                sel = i;
        alive[sel] = 0;
        int64_t a = prev[sel], b = next[sel];
        next[a] = b;
        prev[b] = a;
        if (a > 0)
            area[a] = vw_area(X, Y, prev[a], a, b);
        if (b < m - 1)
            area[b] = vw_area(X, Y, a, b, next[b]);
    }
    int64_t c = 0;
    for (int64_t i = 0; i < m; i++)
        if (alive[i])
            out[c++] = i;
    free(prev);
    free(next);
    free(area);
    free(alive);
    return ORC_OK;
}

/* Farthest interior point of segment (a, b) and its key (R17); -1 if none. */
static int64_t dp_farthest(const double *X, const double *Y, int64_t a, int64_t b, double *key)
{
    int64_t sel = -1;
    double best = -1.0;
    for (int64_t j = a + 1; j < b; j++) {
        double c = fabs((X[b] - X[a]) * (Y[j] - Y[a]) - (X[j] - X[a]) * (Y[b] - Y[a]));
        if (c > best) { /* lowest index on ties (R17) */
            best = c;
            sel = j;
        }
    }
    if (sel >= 0) {
        double dx = X[b] - X[a], dy = Y[b] - Y[a];
        *key = best * best / (dx * dx + dy * dy);
        if (isnan(*key))
            *key = -1.0; /* R17 */
    }
    return sel;
}

static int dp_positions(const double *X, const double *Y, int64_t m, int64_t n_out, int64_t *out)
{
    char *kept = (char *)calloc((size_t)m, 1);
    if (!kept)
        return ORC_ENOMEM;
    kept[0] = kept[m - 1] = 1;
    /* plain rescan of every segment each time */
    for (int64_t count = 2; count < n_out; count++) {
        int64_t best_j = -1;
        double best_key = -2.0; /* below every key */
        int64_t a = 0;
        for (int64_t b = 1; b < m; b++) {
            if (!kept[b])
                continue;
            double key;
            int64_t j = dp_farthest(X, Y, a, b, &key);
            if (j >= 0 && key > best_key) { /* segments in index order: the lowest point wins ties */
                best_key = key;
                best_j = j;
            }
            a = b;
        }
        kept[best_j] = 1;
    }
    int64_t c = 0;
    for (int64_t i = 0; i < m; i++)
        if (kept[i])
            out[c++] = i;
    free(kept);
    return ORC_OK;
}

static int llb_positions(const double *X, const double *Y, int64_t m, int64_t n_out, int64_t *out)
{
    int64_t B = n_out - 2;
    double *L = (double *)malloc(sizeof(double) * (size_t)m);
    int64_t *pred = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    if (!L || !pred) {
        free(L);
        free(pred);
        return ORC_ENOMEM;
    }
    L[0] = 0.0;
    int64_t p0 = 0, p1 = 1; /* the previous bucket: point 0 alone */
    for (int64_t k = 0; k <= B; k++) {
        int64_t s0, s1;
        if (k < B) {
            s0 = 1 + floor_frac(k, m - 2, B); /* R5 */
            s1 = 1 + floor_frac(k + 1, m - 2, B);
        } else {
            s0 = m - 1;
            s1 = m;
        }
        for (int64_t j = s0; j < s1; j++) {
            double best = -1.0;
            int64_t bi = p0;
            for (int64_t i = p0; i < p1; i++) {
                double dx = X[j] - X[i], dy = Y[j] - Y[i];
                double t = L[i] + sqrt(dx * dx + dy * dy); /* R18 */
                if (t > best) { /* lowest index on ties */
                    best = t;
                    bi = i;
                }
            }
            L[j] = best;
            pred[j] = bi;
        }
        p0 = s0;
        p1 = s1;
    }
    int64_t j = m - 1;
    for (int64_t k = n_out - 1; k >= 0; k--) {
        out[k] = j;
        j = k > 0 ? pred[j] : 0;
    }
    free(L);
    free(pred);
    return ORC_OK;
}

/* MinMax preselection (R1-R4) then VW, DP or LLB on P (alg 1, 2, 3). */
int oracle_minmax_simplify(int alg, int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps,
                           int64_t *out)
{
    if (alg < 1 || alg > 3 || n < 1 || n_out < 3 || r_ps < 2 || check_x(xk, x) != ORC_OK)
        return ORC_EINVAL;
    if (n <= n_out) {
        for (int64_t i = 0; i < n; i++)
            if (!is_finite_f32(y[i]))
                return ORC_ENOTFINITE;
        for (int64_t i = 0; i < n; i++)
            out[i] = i;
        return ORC_OK;
    }
    int64_t nb = (int64_t)(((__int128)n_out * r_ps) / 2);
    int64_t *P = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * nb + 2));
    if (!P)
        return ORC_ENOMEM;
    int64_t m = 0;
    int rc = oracle_minmax(y, n, n_out, r_ps, P, &m);
    double *X = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *Y = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_out);
    if (rc == ORC_OK && (!X || !Y || !pos))
        rc = ORC_ENOMEM;
    if (rc == ORC_OK) {
        for (int64_t i = 0; i < m; i++) {
            X[i] = (double)((xk == XK_INT64) ? x[P[i]] : P[i]);
            Y[i] = (double)y[P[i]];
        }
        if (alg == 1)
            rc = vw_positions(X, Y, m, n_out, pos);
        else if (alg == 2)
            rc = dp_positions(X, Y, m, n_out, pos);
        else
            rc = llb_positions(X, Y, m, n_out, pos);
        if (rc == ORC_OK)
            for (int64_t i = 0; i < n_out; i++)
                out[i] = P[pos[i]];
    }
    free(P);
    free(X);
    free(Y);
    free(pos);
    return rc;
}

/* The simplifier alone over m > n_out given points (test hook). */
int oracle_simplify_points(int alg, const double *X, const double *Y, int64_t m, int64_t n_out, int64_t *out)
{
    if (alg < 1 || alg > 3 || n_out < 3 || m <= n_out)
        return ORC_EINVAL;
    if (alg == 1)
        return vw_positions(X, Y, m, n_out, out);
    if (alg == 2)
        return dp_positions(X, Y, m, n_out, out);
    return llb_positions(X, Y, m, n_out, out);
}

/* ------------------------------------------------------------------------ */
/* M4 and EveryNth (section 2.2.1, Table 1; R12, R13).                       */
/* ------------------------------------------------------------------------ */

/* out: capacity 4 * floor(n_out / 4) (or n when n <= n_out); *count = size. */
int oracle_m4(const float *y, int64_t n, int64_t n_out, int64_t *out, int64_t *count)
{
    if (n < 1 || n_out < 4)
        return ORC_EINVAL;
    for (int64_t i = 0; i < n; i++)
        if (!is_finite_f32(y[i]))
            return ORC_ENOTFINITE;
    int64_t cnt = 0;
    if (n <= n_out) {
        for (int64_t i = 0; i < n; i++)
            out[cnt++] = i;
        *count = cnt;
        return ORC_OK;
    }
    int64_t nb = n_out / 4;
    for (int64_t b = 0; b < nb; b++) {
        int64_t lo = floor_frac(b, n, nb);
        int64_t hi = floor_frac(b + 1, n, nb);
        if (lo == hi)
            continue;
        int64_t imin = lo, imax = lo;
        for (int64_t i = lo + 1; i < hi; i++) {
            if (y[i] < y[imin]) /* lowest index on ties (R12) */
                imin = i;
            if (y[i] > y[imax]) /* lowest index on ties (R12) */
                imax = i;
        }
        out[cnt++] = lo;
        out[cnt++] = imin;
        out[cnt++] = imax;
        out[cnt++] = hi - 1;
    }
    qsort(out, (size_t)cnt, sizeof(int64_t), cmp_i64);
    int64_t d = 0;
    for (int64_t i = 0; i < cnt; i++)
        if (d == 0 || out[i] != out[d - 1])
            out[d++] = out[i];
    *count = d;
    return ORC_OK;
}

/* out: capacity min(n, n_out). */
/* Threads the parallel loops of this build may use: 1 unless built with
 * -fopenmp (then OpenMP's limit, e.g. OMP_NUM_THREADS). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int oracle_everynth(int64_t n, int64_t n_out, int64_t *out)
{
    if (n < 1 || n_out < 1)
        return ORC_EINVAL;
    if (n <= n_out) {
        for (int64_t i = 0; i < n; i++)
            out[i] = i;
        return ORC_OK;
    }
    for (int64_t k = 0; k < n_out; k++)
        out[k] = floor_frac(k, n, n_out);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Entry points exposed only so that tests can pin the pieces one by one.    */
/* ------------------------------------------------------------------------ */

/* Next-bucket means of LTTB over m points (R6); MX, MY hold n_out-2 values. */
int oracle_lttb_means(int xk, const int64_t *x, const float *y, int64_t m, int64_t n_out, double *MX, double *MY)
{
    if (m <= n_out || n_out < 3 || check_x(xk, x) != ORC_OK)
        return ORC_EINVAL;
    int64_t *xs = abscissae(xk, x, m);
    if (!xs)
        return ORC_ENOMEM;
    lttb_means(xs, y, m, n_out, MX, MY);
    free(xs);
    return ORC_OK;
}

int oracle_exact_sum_f32(const float *v, int64_t c, double *out)
{
    *out = exact_sum_f32(v, c);
    return ORC_OK;
}

/* The next-bucket means LTTB takes over m > n_out points of any value type. */
int oracle_lttb_means_typed(int xk, const void *x, int yk, const void *y, int64_t m, int64_t n_out, double *MX,
                            double *MY)
{
    if (m <= n_out || n_out < 3)
        return ORC_EINVAL;
    int rc = check_typed(xk, x, yk, y, m);
    if (rc != ORC_OK)
        return rc;
    int64_t *xi = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    double *xf = (double *)malloc(sizeof(double) * (size_t)m);
    double *Y = (double *)malloc(sizeof(double) * (size_t)m);
    if (xi && xf && Y) {
        for (int64_t i = 0; i < m; i++) {
            xi[i] = (xk == XK_INT64) ? ((const int64_t *)x)[i] : i;
            xf[i] = (xk == XK_F64) ? ((const double *)x)[i] : 0.0;
            Y[i] = y_value(yk, y, i);
        }
        lttb_means_typed(xk == XK_F64 ? NULL : xi, xf, Y, m, n_out, MX, MY);
    } else {
        rc = ORC_ENOMEM;
    }
    free(xi);
    free(xf);
    free(Y);
    return rc;
}

int oracle_exact_sum_f64(const double *v, int64_t c, double *out)
{
    *out = exact_sum_f64(v, c);
    return ORC_OK;
}

int oracle_exact_sum_i64(const int64_t *v, int64_t c, double *out)
{
    *out = exact_sum_i64(v, c);
    return ORC_OK;
}
