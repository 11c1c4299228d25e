/* Host AddressSanitizer / UndefinedBehaviorSanitizer run of the C ABI's
 * argument checks: every entry point called with invalid arguments must
 * return the documented negative position (or DD_OK for quick returns)
 * without touching a device, and calls that pass the checks must fail
 * cleanly when no GPU is present.  Exit status 0 when every check passes. */
#include <stdint.h>
#include <stdio.h>

#include "../../include/ddgemm.h"

static int failures = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); ++failures; } } while (0)
#define P(x) ((double *)(uintptr_t)(x))

int main(void) {
    const double *A = P(1 << 20), *Al = P(1 << 21), *B = P(1 << 22), *Bl = P(1 << 23);
    double *C = P(1 << 24), *Cl = P(1 << 25);
    /* dd_gemm */
    CHECK(dd_gemm(-1, 2, 3, A, Al, 1, B, Bl, 3, C, Cl, 1, 0) == -1);
    CHECK(dd_gemm(4, 4, 4, A, Al, 3, B, Bl, 4, C, Cl, 4, 0) == -6);
    CHECK(dd_gemm(4, 4, 4, A, Al, 4, B, Bl, 3, C, Cl, 4, 0) == -9);
    CHECK(dd_gemm(4, 4, 4, A, Al, 4, B, Bl, 4, C, Cl, 3, 0) == -12);
    CHECK(dd_gemm(4, 4, 4, 0, Al, 4, B, Bl, 4, C, Cl, 4, 0) == -4);
    CHECK(dd_gemm(4, 4, 4, A, Al, 4, B, Bl, 4, P(1 << 20), Cl, 4, 0) == -10);   /* C over A */
    CHECK(dd_gemm(0, 4, 4, A, Al, 1, B, Bl, 4, C, Cl, 1, 0) == DD_OK);          /* quick return */
    /* dd_gemm_ex options */
    dd_gemm_opts o = {0};
    o.kc = 6;
    CHECK(dd_gemm_ex(DD_OP_N, DD_OP_N, 4, 4, 4, A, Al, 4, B, Bl, 4, C, Cl, 4, NULL, 0, &o, 0) == -17);
    o.kc = 0; o.algo = 9;
    CHECK(dd_gemm_ex(DD_OP_N, DD_OP_N, 4, 4, 4, A, Al, 4, B, Bl, 4, C, Cl, 4, NULL, 0, &o, 0) == -17);
    o.algo = 0; o.tile = 7;
    CHECK(dd_gemm_ex(DD_OP_N, DD_OP_N, 4, 4, 4, A, Al, 4, B, Bl, 4, C, Cl, 4, NULL, 0, &o, 0) == -17);
    o.tile = 0;
    CHECK(dd_gemm_ex((dd_op)2, DD_OP_N, 4, 4, 4, A, Al, 4, B, Bl, 4, C, Cl, 4, NULL, 0, &o, 0) == -1);
    CHECK(dd_gemm_ex(DD_OP_N, DD_OP_N, 4, 4, 4, A, Al, 4, B, Bl, 4, C, Cl, 4, NULL, 64, &o, 0) == -15);
    CHECK(dd_gemm_noalloc(DD_OP_N, DD_OP_N, 4, 4, 4, A, Al, 4, B, Bl, 4, C, Cl, 3, &o, 0) == -14);
    /* workspace sizes */
    CHECK(dd_gemm_workspace_size(DD_OP_N, DD_OP_N, 100, 70, 300, NULL) > 0);
    CHECK(dd_gemm_workspace_size((dd_op)3, DD_OP_N, 100, 70, 300, NULL) == 0);
    CHECK(td_gemm_workspace_size(DD_OP_N, DD_OP_N, 100, 70, 300, 6) == 0);
    /* FP64x3, vector calls, splits, batched plans, tuner */
    CHECK(td_gemm_ex(DD_OP_N, DD_OP_N, 4, 4, 4, A, Al, Al, 3, B, Bl, Bl, 4, C, Cl, Cl, 4, NULL, 0, 0, 0) == -9);
    CHECK(dd_dot(-1, A, Al, 1, B, Bl, 1, C, 0) == -1);
    CHECK(dd_scal(4, 0, A, Al, 1, C, Cl, 1, 0) == -2);
    CHECK(dd_add(4, A, Al, 1, B, Bl, 0, C, Cl, 1, 0) == -7);
    CHECK(dd_add(4, A, Al, 1, B, Bl, 1, P((1 << 20) + 8), Cl, 1, 0) == -8);
    CHECK(dd_cascade_split(2, DD_OP_N, 4, 4, A, Al, 4, 0, NULL, NULL, 0) == -1);
    CHECK(dd_slices_split(0, DD_OP_N, 4, 4, A, Al, 4, 5, 0, 0, NULL, NULL, 0) == -8);
    int64_t m[2] = {4, 5}, n[2] = {4, -1}, k[2] = {4, 4}, ld[2] = {4, 5};
    dd_batched_plan plan = NULL;
    CHECK(dd_batched_plan_create(2, m, n, k, ld, ld, ld, NULL, &plan) == -2 && plan == NULL);
    CHECK(dd_batched_plan_create(-1, m, n, k, ld, ld, ld, NULL, &plan) == -1);
    CHECK(dd_batched_plan_schedule(NULL, 1, 1, 0, 0) == -1);
    CHECK(dd_batched_plan_destroy(NULL) == DD_OK);
    int32_t shapes[2];
    CHECK(dd_tune(2, m, n, k, NULL, 0, shapes, 0) == -6);
    CHECK(dd_tune(2, m, n, k, NULL, 1, shapes, 0) == -2);
    /* valid calls without a GPU fail cleanly */
    const dd_status st = dd_gemm(4, 4, 4, A, Al, 4, B, Bl, 4, C, Cl, 4, 0);
    CHECK(st == DD_ERR_HIP || st == DD_ERR_UNSUPPORTED);
    CHECK(dd_status_string(-3) != NULL && dd_version() >= 100);
    if (failures) fprintf(stderr, "%d checks failed\n", failures);
    else printf("abi checks passed\n");
    return failures ? 1 : 0;
}
