/* Host AddressSanitizer / UndefinedBehaviorSanitizer run of the C part of the
 * FP64x2 oracle (test infrastructure): every exported routine on small
 * problems, ragged shapes and transposes, with results checked where they
 * are exact (integer-valued operands give exact FP64x2 sums; the exact
 * reference gives zero error for the exact result).  Exit status 0 when
 * every check passes; a sanitizer report aborts with a nonzero status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_dd_gemm(int64_t m, int64_t n, int64_t k, int transa, int transb, const double *Ahi,
                   const double *Alo, int64_t lda, const double *Bhi, const double *Blo, int64_t ldb,
                   double *Chi, double *Clo, int64_t ldc, int nthreads);
int oracle_dd_gemm_entries(int64_t count, const int64_t *I, const int64_t *J, int64_t k, int transa,
                           int transb, const double *Ahi, const double *Alo, int64_t lda, const double *Bhi,
                           const double *Blo, int64_t ldb, const double *Chi, const double *Clo, int64_t ldc,
                           double *out_hi, double *out_lo, int nthreads);
int oracle_exact_entries(int64_t count, const int64_t *I, const int64_t *J, int64_t k, const double *Ahi,
                         const double *Alo, int64_t lda, const double *Bhi, const double *Blo, int64_t ldb,
                         const double *Chi, const double *Clo, int64_t ldc, const double *Rhi,
                         const double *Rlo, double *exact, double *err, int nthreads);
void oracle_dd_add_vec(int64_t n, const double *xh, const double *xl, const double *yh, const double *yl,
                       double *zh, double *zl);

static int failures = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); ++failures; } } while (0)

static double *alloc(int64_t n) {
    double *p = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
    return p;
}

/* integers in [-8, 8] from a fixed linear congruential sequence */
static uint64_t state = 2303;
static double small_int(void) {
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)((int)((state >> 33) % 17) - 8);
}

static void one_shape(int64_t m, int64_t n, int64_t k, int transa, int transb) {
    const int64_t ar = transa ? k : m, ac = transa ? m : k, br = transb ? n : k, bc = transb ? k : n;
    const int64_t lda = ar + 2, ldb = br + 1, ldc = m + 3;   /* padded leading dimensions */
    double *Ah = alloc(lda * ac), *Al = alloc(lda * ac), *Bh = alloc(ldb * bc), *Bl = alloc(ldb * bc);
    double *Ch = alloc(ldc * n), *Cl = alloc(ldc * n), *Rh = alloc(ldc * n), *Rl = alloc(ldc * n);
    for (int64_t i = 0; i < lda * ac; ++i) { Ah[i] = small_int(); Al[i] = 0.0; }
    for (int64_t i = 0; i < ldb * bc; ++i) { Bh[i] = small_int(); Bl[i] = 0.0; }
    for (int64_t i = 0; i < ldc * n; ++i) { Ch[i] = small_int(); Cl[i] = 0.0; Rh[i] = Ch[i]; Rl[i] = 0.0; }
    oracle_dd_gemm(m, n, k, transa, transb, Ah, Al, lda, Bh, Bl, ldb, Rh, Rl, ldc, 2);
    int64_t cnt = m * n;
    int64_t *I = (int64_t *)malloc((size_t)(cnt > 0 ? cnt : 1) * sizeof(int64_t));
    int64_t *J = (int64_t *)malloc((size_t)(cnt > 0 ? cnt : 1) * sizeof(int64_t));
    double *Eh = alloc(cnt), *El = alloc(cnt);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double s = Ch[i + j * ldc];
            for (int64_t p = 0; p < k; ++p) {
                const double a = transa ? Ah[p + i * lda] : Ah[i + p * lda];
                const double b = transb ? Bh[j + p * ldb] : Bh[p + j * ldb];
                s += a * b;   /* integers below 2^53: exact */
            }
            CHECK(Rh[i + j * ldc] == s && Rl[i + j * ldc] == 0.0);
            I[i + j * m] = i;
            J[i + j * m] = j;
        }
    oracle_dd_gemm_entries(cnt, I, J, k, transa, transb, Ah, Al, lda, Bh, Bl, ldb, Ch, Cl, ldc, Eh, El, 2);
    for (int64_t t = 0; t < cnt; ++t) CHECK(Eh[t] == Rh[I[t] + J[t] * ldc] && El[t] == Rl[I[t] + J[t] * ldc]);
    if (!transa && !transb) {
        double *Gh = alloc(cnt), *Gl = alloc(cnt), *X = alloc(cnt), *D = alloc(cnt);
        for (int64_t t = 0; t < cnt; ++t) { Gh[t] = Eh[t]; Gl[t] = El[t]; }
        int used = oracle_exact_entries(cnt, I, J, k, Ah, Al, lda, Bh, Bl, ldb, Ch, Cl, ldc, Gh, Gl, X, D, 2);
        CHECK(used >= 1);
        for (int64_t t = 0; t < cnt; ++t) CHECK(D[t] == 0.0 && X[t] == Eh[t]);
        free(Gh); free(Gl); free(X); free(D);
    }
    free(I); free(J); free(Eh); free(El);
    free(Ah); free(Al); free(Bh); free(Bl); free(Ch); free(Cl); free(Rh); free(Rl);
}

int main(void) {
    const int64_t shapes[][3] = {{1, 1, 1}, {3, 2, 5}, {7, 5, 9}, {17, 3, 33}, {4, 9, 0}};
    for (int s = 0; s < 5; ++s)
        for (int ta = 0; ta < 2; ++ta)
            for (int tb = 0; tb < 2; ++tb) one_shape(shapes[s][0], shapes[s][1], shapes[s][2], ta, tb);
    /* the vector addition: x + (-x) = 0, x + 0 = x, in place */
    double xh[3] = {1.0, 0.5, -3.0}, xl[3] = {0x1p-60, 0.0, 0x1p-55};
    double yh[3] = {-1.0, 0.0, 3.0}, yl[3] = {-0x1p-60, 0.0, -0x1p-55};
    double zh[3], zl[3];
    oracle_dd_add_vec(3, xh, xl, yh, yl, zh, zl);
    CHECK(zh[0] == 0.0 && zl[0] == 0.0 && zh[1] == 0.5 && zl[1] == 0.0 && zh[2] == 0.0 && zl[2] == 0.0);
    oracle_dd_add_vec(3, xh, xl, xh, xl, xh, xl);
    CHECK(xh[0] == 2.0 && xl[0] == 0x1p-59 && xh[2] == -6.0 && xl[2] == 0x1p-54);
    if (failures) fprintf(stderr, "%d checks failed\n", failures);
    else printf("oracle checks passed\n");
    return failures ? 1 : 0;
}
