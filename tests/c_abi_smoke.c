/* A plain C99 caller of the C ABI: compiled with gcc against include/eik.h and
 * include/eik_probe.h, linked with libeik.so and libeik_probe.so, and run without a GPU (only
 * the host-side entry points are called: sizes, argument checks, names; the fake device
 * pointers are refused before any use). */
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include "eik.h"
#include "eik_probe.h"

static int fails = 0;
#define CHECK(c) do { if (!(c)) { printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } } while (0)

int main(void) {
    int64_t dims[3] = {65, 65, 65};
    size_t grid = 0, ws = 0;
    CHECK(eik_problem_bytes(dims, 8, EIK_F32, EIK_MODE_FP64, &grid) == EIK_OK);
    CHECK(grid > (size_t)65 * 65 * 65 * (8 + 4));
    CHECK(eik_query_workspace(dims, 8, EIK_F32, EIK_MODE_FP64, &ws) == EIK_OK && ws > grid);
    CHECK(eik_problem_bytes(dims, 6, EIK_F32, EIK_MODE_FP64, &grid) == EIK_EINVAL);
    int64_t bad[3] = {1, 65, 65};
    CHECK(eik_problem_bytes(bad, 8, EIK_F32, EIK_MODE_FP64, &grid) == EIK_EINVAL);
    /* invalid arguments are refused before any device work */
    eik_sources src;
    memset(&src, 0, sizeof src);
    CHECK(eik_solve(dims, 0.1, NULL, EIK_F32, &src, NULL, 8, 0.0, NULL) == EIK_EINVAL);
    eik_problem pb;
    memset(&pb, 0, sizeof pb);
    CHECK(eik_solve_batch(0, &pb, EIK_F32, 8, NULL, NULL) == EIK_EINVAL);
    CHECK(eik_server_create(NULL, 1, 1, 1, 8, EIK_F32, NULL, NULL) == EIK_EINVAL);
    /* cells of 16: 65 nodes -> 5 cells per axis; two sweep streams are refused there */
    size_t g16 = 0;
    CHECK(eik_problem_bytes(dims, 16, EIK_F32, EIK_MODE_FP64, &g16) == EIK_OK);
    CHECK(g16 >= (size_t)125 * 4096 * (8 + 4) + (size_t)125 * 1536 * 8);
    CHECK(eik_problem_bytes(dims, 32, EIK_F32, EIK_MODE_FP64, &g16) == EIK_EINVAL);
    eik_options dual;
    memset(&dual, 0, sizeof dual);
    dual.inner = EIK_INNER_DUAL;
    int64_t idx[3] = {0, 0, 0};
    double q0 = 0.0;
    eik_sources one;
    memset(&one, 0, sizeof one);
    one.n = 1;
    one.idx3 = idx;
    one.q = &q0;
    CHECK(eik_solve_ex(dims, 0.1, (const void*)16, EIK_F32, &one, (double*)16, 16, 0.0, NULL,
                       &dual) == EIK_EINVAL);
    eik_server* srv = NULL;
    CHECK(eik_server_create(&srv, 1 << 20, 100, 2, 16, EIK_F32, NULL, &dual) == EIK_EINVAL);
    CHECK(srv == NULL);
    float ms = 0.0f;
    CHECK(eikp_copy(NULL, NULL, 16, 1, NULL, &ms) == -1);
    CHECK(strcmp(eik_strerror(EIK_OK), "EIK_OK") == 0);
    CHECK(strncmp(eik_version(), "eik-mi355x", 10) == 0);
    CHECK(sizeof(eik_problem) == 96);
    CHECK(sizeof(eik_options) == 88 && offsetof(eik_options, schedule) == 72 &&
          offsetof(eik_options, jitter) == 80);
    printf("%s: %d failures\n", eik_version(), fails);
    return fails != 0;
}
