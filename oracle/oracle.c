/*
 * Oracle for the exact k-means hot path: plain, slow, obviously correct FP64
 * Lloyd iteration on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; the tests, the smoke check and the benchmark's CPU-baseline
 * leg are its only users.  It shares no code with the GPU library.
 *
 * What it computes (paper: problem definition, Eq. (1) and the description of
 * Lloyd's algorithm right after it; the exactness claim for index-based
 * acceleration in the related-work subsection on accelerated Lloyd's
 * algorithms; Algorithm 1's outer loop and its centroid refinement step):
 *
 *   for t = 1..T:
 *     a_t(i) = argmin_j D(x_i, c_j)          ties -> lowest j
 *     c_j    = RN(exact sum of x_i in S_j) / |S_j|,  or the old c_j if S_j is empty
 *     stop early once a_t == a_{t-1} (t >= 2) when asked to
 *
 * Readings of points the paper leaves open (each stated where used):
 *  - D is the squared Euclidean distance, compared without sqrt.
 *  - D is evaluated canonically: dx_i = fl(x_i - c_i), then
 *    fl(...fl(fl(dx_0^2) + fl(dx_1^2)) + ...), left to right, no fused
 *    multiply-add (this file must be compiled with -ffp-contract=off).
 *  - cluster sums are exact (a fixed-point super-accumulator), rounded once
 *    to nearest-even double, then divided by the count in IEEE double.
 *  - an empty cluster keeps its previous centroid.
 *
 * Build: gcc -O2 -fPIC -shared -fopenmp -ffp-contract=off -fno-fast-math
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Canonical squared distance (problem definition, Eq. (1)).                 */
/* ------------------------------------------------------------------------ */
static double dist64(const double *x, const double *c, int d)
{
    double t = x[0] - c[0];
    double s = t * t;
    for (int i = 1; i < d; ++i) {
        t = x[i] - c[i];
        s = s + t * t;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Exact summation of doubles.                                               */
/*                                                                           */
/* Every finite double is an integer multiple of 2^-1074 below 2^1024, so    */
/* a sum of doubles is an integer number of 2^-1074 units.  The accumulator  */
/* keeps that integer as base-2^32 digits, each held in a signed 64-bit limb  */
/* so that up to 2^30 additions need no carry propagation.                   */
/* ------------------------------------------------------------------------ */
#define ACC_LIMBS 70 /* 70*32 = 2240 bits > 1074 + 1024 + 64 bits of headroom */

typedef struct {
    int64_t limb[ACC_LIMBS];
    int64_t pending; /* additions since the last carry propagation */
} exact_acc;

static void acc_clear(exact_acc *A) { memset(A, 0, sizeof(*A)); }

static void acc_normalize(exact_acc *A)
{
    for (int i = 0; i < ACC_LIMBS - 1; ++i) {
        int64_t carry = A->limb[i] >> 32; /* floor division by 2^32 */
        A->limb[i] -= carry * ((int64_t)1 << 32);
        A->limb[i + 1] += carry;
    }
    A->pending = 0;
}

static void acc_add(exact_acc *A, double v)
{
    if (v == 0.0)
        return;
    int e;
    double m = frexp(v, &e);             /* v = m * 2^e, 0.5 <= |m| < 1 */
    int64_t M = (int64_t)ldexp(m, 53);   /* exact: |M| < 2^53          */
    int64_t sh = (int64_t)e - 53 + 1074; /* v = M * 2^(sh - 1074)      */
    int neg = M < 0;
    uint64_t mag = (uint64_t)(neg ? -M : M);
    if (sh < 0) {                        /* subnormal: dropped bits are zero */
        mag >>= -sh;
        sh = 0;
    }
    int q = (int)(sh / 32), r = (int)(sh % 32);
    unsigned __int128 w = (unsigned __int128)mag << r; /* at most 85 bits */
    for (int j = 0; j < 3 && q + j < ACC_LIMBS; ++j) {
        int64_t digit = (int64_t)(uint64_t)(w & 0xffffffffu);
        A->limb[q + j] += neg ? -digit : digit;
        w >>= 32;
    }
    if (++A->pending >= ((int64_t)1 << 30))
        acc_normalize(A);
}

/* Bit b of a non-negative multi-digit magnitude. */
static int mag_bit(const uint32_t *dig, int64_t b) { return (dig[b / 32] >> (b % 32)) & 1u; }

/* Round the exact sum to the nearest double, ties to even. */
static double acc_round(exact_acc *A)
{
    acc_normalize(A);
    uint32_t dig[ACC_LIMBS];
    int neg = A->limb[ACC_LIMBS - 1] < 0;
    /* two's-complement negate across digits when negative */
    int64_t borrow = 0;
    for (int i = 0; i < ACC_LIMBS; ++i) {
        int64_t v = A->limb[i];
        if (neg) {
            v = -v - borrow;
            borrow = 0;
            if (v < 0) {
                v += (int64_t)1 << 32;
                borrow = 1;
            }
        }
        dig[i] = (uint32_t)v;
    }
    int64_t top = -1;
    for (int i = ACC_LIMBS - 1; i >= 0 && top < 0; --i)
        if (dig[i])
            for (int b = 31; b >= 0; --b)
                if ((dig[i] >> b) & 1u) {
                    top = (int64_t)i * 32 + b;
                    break;
                }
    if (top < 0)
        return 0.0;
    double out;
    if (top < 53) { /* fewer than 54 significant bits: exactly representable */
        uint64_t M = 0;
        for (int64_t b = top; b >= 0; --b)
            M = (M << 1) | (uint64_t)mag_bit(dig, b);
        out = ldexp((double)M, -1074);
    } else {
        uint64_t M = 0;
        for (int64_t b = top; b > top - 53; --b)
            M = (M << 1) | (uint64_t)mag_bit(dig, b);
        int round = mag_bit(dig, top - 53);
        int sticky = 0;
        for (int64_t b = top - 54; b >= 0 && !sticky; --b)
            sticky = mag_bit(dig, b);
        int64_t ex = top - 52 - 1074;
        if (round && (sticky || (M & 1u))) {
            ++M;
            if (M == ((uint64_t)1 << 53)) {
                M >>= 1;
                ++ex;
            }
        }
        out = ldexp((double)M, (int)ex);
    }
    return neg ? -out : out;
}

double oracle_exact_sum(const double *v, int64_t n)
{
    exact_acc *A = (exact_acc *)malloc(sizeof(exact_acc));
    acc_clear(A);
    for (int64_t i = 0; i < n; ++i)
        acc_add(A, v[i]);
    double s = acc_round(A);
    free(A);
    return s;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Assignment step: brute force over all k centroids, lowest index on ties.  */
/* ------------------------------------------------------------------------ */
void oracle_assign(const double *x, int64_t n, int d, const double *c, int64_t k,
                   int32_t *a_out, double *dmin_out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double *xi = x + i * d;
        double best = dist64(xi, c, d);
        int64_t bj = 0;
        for (int64_t j = 1; j < k; ++j) {
            double D = dist64(xi, c + j * d, d);
            if (D < best) { /* strict: an equal distance keeps the lower index */
                best = D;
                bj = j;
            }
        }
        a_out[i] = (int32_t)bj;
        if (dmin_out)
            dmin_out[i] = best;
    }
}

/* Point indices grouped by cluster (stable counting sort). */
static void group_by_cluster(const int32_t *a, int64_t n, int64_t k, int64_t *start, int64_t *idx)
{
    memset(start, 0, sizeof(int64_t) * (size_t)(k + 1));
    for (int64_t i = 0; i < n; ++i)
        start[a[i] + 1]++;
    for (int64_t j = 0; j < k; ++j)
        start[j + 1] += start[j];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    memcpy(fill, start, sizeof(int64_t) * (size_t)k);
    for (int64_t i = 0; i < n; ++i)
        idx[fill[a[i]]++] = i;
    free(fill);
}

/* ------------------------------------------------------------------------ */
/* Update step (Algorithm 1, centroid refinement): exact per-cluster sums.   */
/* ------------------------------------------------------------------------ */
void oracle_update(const double *x, int64_t n, int d, const int32_t *a, int64_t k,
                   const double *c_prev, double *c_out, int64_t *cnt_out)
{
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k + 1));
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    group_by_cluster(a, n, k, start, idx);
#pragma omp parallel
    {
        exact_acc *A = (exact_acc *)malloc(sizeof(exact_acc));
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < k; ++j) {
            int64_t cnt = start[j + 1] - start[j];
            if (cnt_out)
                cnt_out[j] = cnt;
            for (int dim = 0; dim < d; ++dim) {
                if (cnt == 0) { /* empty cluster keeps its centroid */
                    c_out[j * d + dim] = c_prev[j * d + dim];
                    continue;
                }
                acc_clear(A);
                for (int64_t p = start[j]; p < start[j + 1]; ++p)
                    acc_add(A, x[idx[p] * d + dim]);
                c_out[j * d + dim] = acc_round(A) / (double)cnt;
            }
        }
        free(A);
    }
    free(start);
    free(idx);
}

/* ------------------------------------------------------------------------ */
/* Lloyd loop (Algorithm 1's outer loop).                                    */
/*   sse_hist[t] = RN(exact sum_i D(x_i, C_{t-1}[a_t(i)])): the objective of */
/*   the assignment made in iteration t, with the centroids it was made to.  */
/* ------------------------------------------------------------------------ */
int oracle_lloyd(const double *x, int64_t n, int d, const double *c0, int64_t k,
                 int max_iter, int stop_when_stable,
                 int32_t *a_hist, double *c_hist, double *sse_hist,
                 double *c_final, int32_t *a_final)
{
    double *c = (double *)malloc(sizeof(double) * (size_t)(k * d));
    double *cn = (double *)malloc(sizeof(double) * (size_t)(k * d));
    int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *ap = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *dm = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(c, c0, sizeof(double) * (size_t)(k * d));
    int t = 0;
    while (t < max_iter) {
        oracle_assign(x, n, d, c, k, a, dm);
        if (sse_hist)
            sse_hist[t] = oracle_exact_sum(dm, n);
        oracle_update(x, n, d, a, k, c, cn, NULL);
        int same = 0;
        if (t >= 1) {
            same = 1;
            for (int64_t i = 0; i < n && same; ++i)
                same = (a[i] == ap[i]);
        }
        memcpy(c, cn, sizeof(double) * (size_t)(k * d));
        if (a_hist)
            memcpy(a_hist + (int64_t)t * n, a, sizeof(int32_t) * (size_t)n);
        if (c_hist)
            memcpy(c_hist + (int64_t)t * k * d, c, sizeof(double) * (size_t)(k * d));
        memcpy(ap, a, sizeof(int32_t) * (size_t)n);
        ++t;
        if (stop_when_stable && same)
            break;
    }
    if (c_final)
        memcpy(c_final, c, sizeof(double) * (size_t)(k * d));
    if (a_final)
        memcpy(a_final, a, sizeof(int32_t) * (size_t)n);
    free(c);
    free(cn);
    free(a);
    free(ap);
    free(dm);
    return t;
}

/* ------------------------------------------------------------------------ */
/* Distortion loss (Eq. (1) for fixed centroids) and its gradient.           */
/*   L_b = RN(exact sum_i D(x_i, c_{a(i)})), a = lowest-index argmin.        */
/*   dL/dx_i = 2 g (x_i - c_{a(i)})                                          */
/*   dL/dc_j = 2 g RN(exact sum_{i in S_j} (c_j - x_i))                      */
/* The assignment is piecewise constant, so it carries no gradient.          */
/* ------------------------------------------------------------------------ */
void oracle_distortion_fwd(const double *x, const double *c, int64_t B, int64_t n, int64_t k, int d,
                           int32_t *a_out, double *loss_out)
{
    double *dm = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t b = 0; b < B; ++b) {
        oracle_assign(x + b * n * d, n, d, c + b * k * d, k, a_out + b * n, dm);
        loss_out[b] = oracle_exact_sum(dm, n);
    }
    free(dm);
}

void oracle_distortion_bwd(const double *x, const double *c, const int32_t *a, const double *g,
                           int64_t B, int64_t n, int64_t k, int d, double *gx, double *gc)
{
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k + 1));
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t b = 0; b < B; ++b) {
        const double *xb = x + b * n * d, *cb = c + b * k * d;
        const int32_t *ab = a + b * n;
        double two_g = 2.0 * g[b];
        if (gx)
            for (int64_t i = 0; i < n; ++i)
                for (int dim = 0; dim < d; ++dim)
                    gx[(b * n + i) * d + dim] = two_g * (xb[i * d + dim] - cb[(int64_t)ab[i] * d + dim]);
        if (gc) {
            group_by_cluster(ab, n, k, start, idx);
#pragma omp parallel
            {
                exact_acc *A = (exact_acc *)malloc(sizeof(exact_acc));
#pragma omp for schedule(dynamic, 16)
                for (int64_t j = 0; j < k; ++j)
                    for (int dim = 0; dim < d; ++dim) {
                        acc_clear(A);
                        for (int64_t p = start[j]; p < start[j + 1]; ++p)
                            acc_add(A, cb[j * d + dim] - xb[idx[p] * d + dim]);
                        gc[(b * k + j) * d + dim] = two_g * acc_round(A);
                    }
                free(A);
            }
        }
    }
    free(start);
    free(idx);
}
