/* A plain C99 program that drives GPU solves through the C ABI alone: no Python and no torch in
 * the process, device memory from the HIP runtime's C API.  Compiled with gcc against
 * include/eik.h, linked with libeik.so and libamdhip64.so.
 *
 * Workload: constant speed on a 65^3 grid, h = 2^-6 (so that sums of h along a grid line are
 * exact), one exit at the centre with value q.  What eq. (2) fixes without a reference solve:
 *   - on the six axis rays through the exit the solution is q + d h exactly (one-term updates
 *     from the previous node; the off-axis neighbours are larger);
 *   - at offsets (1,1,0) and (1,1,1) the two- and three-term roots: q + h + h / sqrt(2) and
 *     q + h + h / sqrt(2) + h / sqrt(3);
 *   - everywhere else the residual of eq. (2) itself vanishes (to rounding).
 * Each entry point is checked against these: eik_solve (FP32 speeds), eik_solve_ex in
 * EIK_MODE_MIXED with timing, eik_solve_batch of two grids, and a server that admits three
 * problems two at a time. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "eik.h"

#define N 65
#define NN ((size_t)N * N * N)
#define IDX(i, j, k) ((size_t)(i) + (size_t)N * ((size_t)(j) + (size_t)N * (size_t)(k)))

static int fails = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);            \
            fflush(stdout);                                               \
            ++fails;                                                      \
        }                                                                 \
    } while (0)
#define HIPOK(x) CHECK((x) == hipSuccess)

static const double H = 1.0 / 64.0;

static double at(const double* u, int i, int j, int k) {
    if (i < 0 || j < 0 || k < 0 || i >= N || j >= N || k >= N) return INFINITY;
    return u[IDX(i, j, k)];
}

/* Largest |sum_axes max(u - a, 0)^2 - h^2| / h^2 over non-exit nodes (speed 1), and the count
 * of nodes that are not finite. */
static double residual(const double* u, int ce, int* nonfinite) {
    double worst = 0.0;
    *nonfinite = 0;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                double v = u[IDX(i, j, k)];
                if (!isfinite(v)) { ++*nonfinite; continue; }
                if (i == ce && j == ce && k == ce) continue;
                double a[3] = {fmin(at(u, i - 1, j, k), at(u, i + 1, j, k)),
                               fmin(at(u, i, j - 1, k), at(u, i, j + 1, k)),
                               fmin(at(u, i, j, k - 1), at(u, i, j, k + 1))};
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    if (v > a[d]) s += (v - a[d]) * (v - a[d]);
                double r = fabs(s - H * H) / (H * H);
                if (r > worst) worst = r;
            }
    return worst;
}

/* The closed-form values and the residual; returns the number of failed checks. */
static int check_solution(const double* u, double q, const char* what) {
    int before = fails;
    const int c = N / 2;
    for (int d = 0; d <= c; ++d) {
        double want = q + d * H;
        CHECK(u[IDX(c + d, c, c)] == want && u[IDX(c - d, c, c)] == want);
        CHECK(u[IDX(c, c + d, c)] == want && u[IDX(c, c - d, c)] == want);
        CHECK(u[IDX(c, c, c + d)] == want && u[IDX(c, c, c - d)] == want);
    }
    double two = q + H + H / sqrt(2.0);
    double three = two + H / sqrt(3.0);
    CHECK(fabs(u[IDX(c + 1, c + 1, c)] - two) <= 1e-14 * two);
    CHECK(fabs(u[IDX(c - 1, c, c + 1)] - two) <= 1e-14 * two);
    CHECK(fabs(u[IDX(c + 1, c - 1, c + 1)] - three) <= 1e-14 * three);
    int nonfinite = 0;
    double rho = residual(u, c, &nonfinite);
    CHECK(nonfinite == 0);
    CHECK(rho <= 1e-10);
    printf("%s: residual %.2e, corner %.17g, %d failed checks\n", what, rho, u[IDX(0, 0, 0)],
           fails - before);
    fflush(stdout);
    return fails - before;
}

static int fetch_check(const double* d_u, double* h_u, double q, const char* what) {
    HIPOK(hipMemcpy(h_u, d_u, NN * sizeof(double), hipMemcpyDeviceToHost));
    return check_solution(h_u, q, what);
}

int main(void) {
    const int64_t dims[3] = {N, N, N};
    const int64_t src_idx[3] = {N / 2, N / 2, N / 2};
    const double qs[3] = {0.0, 0.25, 1.5};

    float* h_f32 = (float*)malloc(NN * sizeof(float));
    double* h_f64 = (double*)malloc(NN * sizeof(double));
    double* h_u = (double*)malloc(NN * sizeof(double));
    if (!h_f32 || !h_f64 || !h_u) return 2;
    for (size_t n = 0; n < NN; ++n) { h_f32[n] = 1.0f; h_f64[n] = 1.0; }

    void *d_f32 = NULL, *d_f64 = NULL;
    double* d_u[3] = {NULL, NULL, NULL};
    HIPOK(hipMalloc(&d_f32, NN * sizeof(float)));
    HIPOK(hipMalloc(&d_f64, NN * sizeof(double)));
    for (int p = 0; p < 3; ++p) HIPOK(hipMalloc((void**)&d_u[p], NN * sizeof(double)));
    if (fails) { printf("device allocation failed\n"); return 1; }
    HIPOK(hipMemcpy(d_f32, h_f32, NN * sizeof(float), hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(d_f64, h_f64, NN * sizeof(double), hipMemcpyHostToDevice));
    hipStream_t stream = NULL;
    HIPOK(hipStreamCreate(&stream));

    eik_sources src[3];
    for (int p = 0; p < 3; ++p) {
        memset(&src[p], 0, sizeof src[p]);
        src[p].n = 1;
        src[p].idx3 = src_idx;
        src[p].q = &qs[p];
        src[p].on_device = 0;
    }

    /* eik_solve: FP32 speeds, default options. */
    eik_stats st;
    memset(&st, 0, sizeof st);
    int rc = eik_solve(dims, H, d_f32, EIK_F32, &src[0], d_u[0], 8, 0.0, stream);
    if (rc != EIK_OK) printf("eik_solve returned %s\n", eik_strerror(rc));
    CHECK(rc == EIK_OK);
    CHECK(eik_stream_status(stream, &st) == EIK_OK);
    CHECK(st.cells == 9 * 9 * 9 && st.visits >= st.cells && st.rounds > 0);
    printf("eik_solve: rounds %lld, visits %lld, updates %lld\n", (long long)st.rounds,
           (long long)st.visits, (long long)st.updates);
    fetch_check(d_u[0], h_u, qs[0], "eik_solve");

    /* eik_solve_ex: FP64 speeds, FP32 bulk + FP64 polish, timed. */
    eik_options opt;
    memset(&opt, 0, sizeof opt);
    opt.mode = EIK_MODE_MIXED;
    opt.timing = 1;
    CHECK(eik_solve_ex(dims, H, d_f64, EIK_F64, &src[1], d_u[1], 8, 0.0, stream, &opt) == EIK_OK);
    CHECK(eik_stream_status(stream, NULL) == EIK_OK);
    double solve_ms = 0.0, total_ms = 0.0;
    CHECK(eik_kernel_times(stream, 1, &solve_ms, &total_ms) == 1);
    CHECK(solve_ms > 0.0 && total_ms >= solve_ms);
    printf("eik_solve_ex (mixed): kernel %.3f ms, call %.3f ms\n", solve_ms, total_ms);
    fetch_check(d_u[1], h_u, qs[1], "eik_solve_ex mixed");

    /* eik_solve_batch: two grids in one launch. */
    eik_problem pb[3];
    for (int p = 0; p < 3; ++p) {
        memset(&pb[p], 0, sizeof pb[p]);
        memcpy(pb[p].dims, dims, sizeof dims);
        pb[p].h = H;
        pb[p].F = d_f32;
        pb[p].sources = src[p];
        pb[p].u_out = d_u[p];
        pb[p].tol = 0.0;
        pb[p].u_approx = NULL;
    }
    for (int p = 0; p < 3; ++p) HIPOK(hipMemset(d_u[p], 0, NN * sizeof(double)));
    CHECK(eik_solve_batch(2, pb, EIK_F32, 8, stream, NULL) == EIK_OK);
    int bst[2] = {-99, -99};
    CHECK(eik_batch_status(stream, 2, bst) == 2 && bst[0] == EIK_OK && bst[1] == EIK_OK);
    fetch_check(d_u[0], h_u, qs[0], "eik_solve_batch grid 0");
    fetch_check(d_u[1], h_u, qs[1], "eik_solve_batch grid 1");

    /* A server with room for two problems at a time: the third waits for a retirement. */
    for (int p = 0; p < 3; ++p) HIPOK(hipMemset(d_u[p], 0, NN * sizeof(double)));
    size_t grid_bytes = 0;
    CHECK(eik_problem_bytes(dims, 8, EIK_F32, EIK_MODE_FP64, &grid_bytes) == EIK_OK);
    eik_server* srv = NULL;
    CHECK(eik_server_create(&srv, 2 * grid_bytes + (1 << 20), 2 * 729, 2, 8, EIK_F32, stream,
                            NULL) == EIK_OK);
    if (srv) {
        int64_t tk = -1;
        CHECK(eik_server_submit(srv, &pb[0], &tk) == EIK_OK && tk == 0);
        CHECK(eik_server_submit(srv, &pb[1], &tk) == EIK_OK && tk == 1);
        CHECK(eik_server_submit(srv, &pb[2], &tk) == EIK_EBUSY);
        int done = 0, submitted = 2, steps = 0;
        int status_of[3] = {-99, -99, -99};
        while (done < 3 && steps < 10000) {
            int fin = 0;
            int rc = eik_server_step(srv, 16, &fin);
            CHECK(rc == EIK_OK);
            if (rc != EIK_OK) break;
            ++steps;
            int64_t tickets[3];
            int status[3], got = 0;
            CHECK(eik_server_poll(srv, 3, tickets, status, &got) == EIK_OK);
            for (int t = 0; t < got; ++t) {
                if (tickets[t] >= 0 && tickets[t] < 3) status_of[tickets[t]] = status[t];
                ++done;
            }
            if (submitted == 2 && got > 0) {
                CHECK(eik_server_submit(srv, &pb[2], &tk) == EIK_OK && tk == 2);
                submitted = 3;
            }
        }
        CHECK(done == 3);
        for (int p = 0; p < 3; ++p) CHECK(status_of[p] == EIK_OK);
        int probs = -1;
        CHECK(eik_server_load(srv, &probs, NULL, NULL) == EIK_OK && probs == 0);
        printf("server: %d steps of 16 rounds\n", steps);
        CHECK(eik_server_destroy(srv) == EIK_OK);
        for (int p = 0; p < 3; ++p) {
            char what[32];
            snprintf(what, sizeof what, "server ticket %d", p);
            fetch_check(d_u[p], h_u, qs[p], what);
        }
    }

    eik_release();
    HIPOK(hipStreamDestroy(stream));
    for (int p = 0; p < 3; ++p) HIPOK(hipFree(d_u[p]));
    HIPOK(hipFree(d_f32));
    HIPOK(hipFree(d_f64));
    free(h_f32);
    free(h_f64);
    free(h_u);
    printf("%s: %d failures\n", eik_version(), fails);
    return fails != 0;
}
