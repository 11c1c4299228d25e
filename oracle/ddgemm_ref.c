/*
 * TEST INFRASTRUCTURE -- not part of the product path.
 *
 * Plain FP64x2 (double-double) GEMM, C := op(A) op(B) + C, as a triple loop.
 * This is the plain FP64x2 triple loop that the paper compares the cascade's
 * accuracy with (Sec. 5.2, accuracy experiments; FP64x2 format
 * of Sec. 3.1, eq. (doubledouble)).  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may call it.
 *
 * Arithmetic (published error-free transforms, written out here):
 *   TwoSum       (Knuth):  s = a+b, e = exact error of that addition
 *   QuickTwoSum  (Dekker): same for |a| >= |b|
 *   TwoProd      (FMA):    p = a*b, e = fma(a, b, -p)
 * DD product of a and b:
 *   (p, e) = TwoProd(a.hi, b.hi); e += (a.hi*b.lo + a.lo*b.hi); QuickTwoSum(p, e)
 * DD sum (the "accurate" double-double add):
 *   (s, e) = TwoSum(x.hi, y.hi); (t, f) = TwoSum(x.lo, y.lo);
 *   e += t; (s, e) = QuickTwoSum(s, e); e += f; QuickTwoSum(s, e)
 * Every output entry: acc = 0; for p = 0..k-1 ascending: acc = acc + a_ip*b_pj;
 * then C_ij = C_ij + acc (C added last).  k == 0 leaves C untouched.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 * Matrices are column-major with leading dimensions (BLAS convention).
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

typedef struct { double hi, lo; } dd_t;

static inline dd_t two_sum(double a, double b) {
    dd_t r;
    double s = a + b;
    double bb = s - a;
    r.hi = s;
    r.lo = (a - (s - bb)) + (b - bb);
    return r;
}

static inline dd_t quick_two_sum(double a, double b) {
    dd_t r;
    double s = a + b;
    r.hi = s;
    r.lo = b - (s - a);
    return r;
}

static inline dd_t two_prod(double a, double b) {
    dd_t r;
    double p = a * b;
    r.hi = p;
    r.lo = fma(a, b, -p);
    return r;
}

static inline dd_t dd_mul(dd_t a, dd_t b) {
    dd_t p = two_prod(a.hi, b.hi);
    double t = a.hi * b.lo;
    double u = a.lo * b.hi;
    double v = t + u;
    p.lo = p.lo + v;
    return quick_two_sum(p.hi, p.lo);
}

static inline dd_t dd_add(dd_t x, dd_t y) {
    dd_t s = two_sum(x.hi, y.hi);
    dd_t t = two_sum(x.lo, y.lo);
    s.lo = s.lo + t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo = s.lo + t.lo;
    return quick_two_sum(s.hi, s.lo);
}

/* element (i, p) of op(X) for a column-major X with leading dimension ld */
static inline int64_t at(int trans, int64_t r, int64_t c, int64_t ld) {
    return trans ? (c + r * ld) : (r + c * ld);
}

static dd_t dot_entry(int64_t i, int64_t j, int64_t k, int transa, int transb,
                      const double *Ahi, const double *Alo, int64_t lda,
                      const double *Bhi, const double *Blo, int64_t ldb) {
    dd_t acc = {0.0, 0.0};
    for (int64_t p = 0; p < k; ++p) {
        int64_t ia = at(transa, i, p, lda);
        int64_t ib = at(transb, p, j, ldb);
        dd_t a = {Ahi[ia], Alo[ia]};
        dd_t b = {Bhi[ib], Blo[ib]};
        acc = dd_add(acc, dd_mul(a, b));
    }
    return acc;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* z = x + y entry by entry with the accurate FP64x2 addition above (the one
 * the triple loop accumulates with).  z may be x or y. */
void oracle_dd_add_vec(int64_t n, const double *xh, const double *xl, const double *yh, const double *yl,
                       double *zh, double *zl) {
    for (int64_t i = 0; i < n; ++i) {
        dd_t x = {xh[i], xl[i]}, y = {yh[i], yl[i]};
        dd_t z = dd_add(x, y);
        zh[i] = z.hi;
        zl[i] = z.lo;
    }
}

/* C := op(A) op(B) + C over the whole m x n output. Returns the threads used. */
int oracle_dd_gemm(int64_t m, int64_t n, int64_t k, int transa, int transb,
                   const double *Ahi, const double *Alo, int64_t lda,
                   const double *Bhi, const double *Blo, int64_t ldb,
                   double *Chi, double *Clo, int64_t ldc, int nthreads) {
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    if (m <= 0 || n <= 0 || k <= 0) return nthreads;
    int used = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t j = 0; j < n; ++j) {
        if (j == 0) used = omp_get_num_threads();
        for (int64_t i = 0; i < m; ++i) {
            dd_t acc = dot_entry(i, j, k, transa, transb, Ahi, Alo, lda, Bhi, Blo, ldb);
            dd_t c = {Chi[i + j * ldc], Clo[i + j * ldc]};
            c = dd_add(c, acc);
            Chi[i + j * ldc] = c.hi;
            Clo[i + j * ldc] = c.lo;
        }
    }
    return used;
}

/* The same computation for a list of output positions (I[t], J[t]):
 * out[t] = C(I[t], J[t]) + sum_p op(A)(I[t], p) op(B)(p, J[t]).
 * C is read only.  Returns the threads used. */
int oracle_dd_gemm_entries(int64_t count, const int64_t *I, const int64_t *J, int64_t k,
                           int transa, int transb,
                           const double *Ahi, const double *Alo, int64_t lda,
                           const double *Bhi, const double *Blo, int64_t ldb,
                           const double *Chi, const double *Clo, int64_t ldc,
                           double *out_hi, double *out_lo, int nthreads) {
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    int used = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t t = 0; t < count; ++t) {
        if (t == 0) used = omp_get_num_threads();
        int64_t i = I[t], j = J[t];
        dd_t c = {Chi[i + j * ldc], Clo[i + j * ldc]};
        if (k > 0) {
            dd_t acc = dot_entry(i, j, k, transa, transb, Ahi, Alo, lda, Bhi, Blo, ldb);
            c = dd_add(c, acc);
        }
        out_hi[t] = c.hi;
        out_lo[t] = c.lo;
    }
    return used;
}

/*
 * Exact reference for accuracy workloads (the role the paper's FP128x2
 * results play in Sec. 5.2): for each requested entry (i, j), the exact value
 * V = sum_p (A_hi + A_lo)_ip (B_hi + B_lo)_pj + (C_hi + C_lo)_ij is kept as a
 * nonoverlapping expansion of doubles (Shewchuk's GROW-EXPANSION with zero
 * elimination, fed every product as the exact pair TwoProd gives); then the
 * computed (R_hi, R_lo) is subtracted inside the same expansion, so the
 * difference R - V is exact before its final rounding.  Outputs: V and R - V
 * rounded to double (sum of the expansion from its small end).  Exact as long
 * as no TwoProd error term falls below the normal range (each such product
 * then loses at most 2^-1074).  Returns the threads used, or -1 when an
 * expansion would outgrow EXP_MAX terms (inputs spanning too many binades).
 */
#define EXP_MAX 600

static int grow_expansion(double *e, int n, double b) {
    double q = b;
    int h = 0;
    for (int i = 0; i < n; ++i) {
        dd_t s = two_sum(q, e[i]);
        q = s.hi;
        if (s.lo != 0.0) e[h++] = s.lo;
    }
    if (q != 0.0 || h == 0) e[h++] = q;
    return h;
}

static double expansion_value(const double *e, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += e[i];
    return s;
}

int oracle_exact_entries(int64_t count, const int64_t *I, const int64_t *J, int64_t k,
                         const double *Ahi, const double *Alo, int64_t lda,
                         const double *Bhi, const double *Blo, int64_t ldb,
                         const double *Chi, const double *Clo, int64_t ldc,
                         const double *Rhi, const double *Rlo,
                         double *exact, double *err, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int used = 1;
    int bad = 0;
#pragma omp parallel reduction(|:bad)
    {
#pragma omp single
        used = omp_get_num_threads();
        double e[EXP_MAX];
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < count; ++t) {
            const int64_t i = I[t], j = J[t];
            int n = 0;
            for (int64_t p = 0; p < k && !bad; ++p) {
                const double a[2] = {Ahi[i + p * lda], Alo[i + p * lda]};
                const double b[2] = {Bhi[p + j * ldb], Blo[p + j * ldb]};
                for (int x = 0; x < 2; ++x)
                    for (int y = 0; y < 2; ++y) {
                        dd_t pr = two_prod(a[x], b[y]);
                        if (n + 2 >= EXP_MAX) { bad = 1; break; }
                        n = grow_expansion(e, n, pr.lo);
                        n = grow_expansion(e, n, pr.hi);
                    }
            }
            if (n + 4 >= EXP_MAX) bad = 1;
            if (bad) continue;
            n = grow_expansion(e, n, Clo[i + j * ldc]);
            n = grow_expansion(e, n, Chi[i + j * ldc]);
            exact[t] = expansion_value(e, n);
            n = grow_expansion(e, n, -Rlo[t]);
            n = grow_expansion(e, n, -Rhi[t]);
            err[t] = -expansion_value(e, n);   /* R - V */
        }
    }
    return bad ? -1 : used;
}
