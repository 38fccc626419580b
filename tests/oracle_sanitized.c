/* Drives the oracle's C code, built with AddressSanitizer and UndefinedBehaviorSanitizer, over
 * seeded random grids (2-14 nodes per axis, speeds in [0.2, 2.2], 1-4 exits with q in [0, 0.1]):
 * every FMM result must equal brute-force Jacobi iteration to 1e-12 relative and satisfy eq. (2)
 * to a residual of 1e-13 at every node.  Any memory error, undefined behaviour or leak ends the
 * run through the sanitizers. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_fmm(int64_t nx, int64_t ny, int64_t nz, double h, const double* F, int64_t nsrc,
               const int64_t* idx3, const double* q, double* u);
int64_t oracle_jacobi(int64_t nx, int64_t ny, int64_t nz, double h, const double* F,
                      int64_t nsrc, const int64_t* idx3, const double* q, int64_t max_sweeps,
                      double* v);
double oracle_residual(int64_t nx, int64_t ny, int64_t nz, double h, const double* F,
                       int64_t nsrc, const int64_t* idx3, const double* U, double bad_tol,
                       int64_t* n_bad);

static uint32_t state = 12345u;
static uint32_t next(uint32_t m) {
    state = state * 1103515245u + 12345u;
    return (state >> 8) % m;
}

int main(void) {
    int bad = 0;
    for (int t = 0; t < 40; ++t) {
        const int64_t nx = 2 + next(13), ny = 2 + next(11), nz = 2 + next(9);
        const int64_t M = nx * ny * nz, ns = 1 + next(4);
        double* F = malloc((size_t)M * sizeof(double));
        double* u = malloc((size_t)M * sizeof(double));
        double* v = malloc((size_t)M * sizeof(double));
        int64_t* idx = malloc((size_t)(3 * ns) * sizeof(int64_t));
        double* q = malloc((size_t)ns * sizeof(double));
        if (!F || !u || !v || !idx || !q) return 2;
        for (int64_t i = 0; i < M; ++i) F[i] = 0.2 + next(1000) / 500.0;
        for (int64_t k = 0; k < ns; ++k) {
            idx[3 * k] = next((uint32_t)nx);
            idx[3 * k + 1] = next((uint32_t)ny);
            idx[3 * k + 2] = next((uint32_t)nz);
            q[k] = next(100) / 1000.0;
        }
        const double h = 0.1;
        int ok = oracle_fmm(nx, ny, nz, h, F, ns, idx, q, u) == 0 &&
                 oracle_jacobi(nx, ny, nz, h, F, ns, idx, q, 100000, v) >= 0;
        double worst = 0.0;
        for (int64_t i = 0; i < M; ++i) {
            const double d = fabs(u[i] - v[i]) / (u[i] > 0.0 ? u[i] : 1.0);
            if (d > worst) worst = d;
        }
        int64_t nbad = 0;
        const double rho = oracle_residual(nx, ny, nz, h, F, ns, idx, u, 1e-13, &nbad);
        if (!ok || worst > 1e-12 || nbad != 0 || !(rho <= 1e-13)) {
            ++bad;
            printf("case %d (%lld x %lld x %lld): jacobi diff %.2e, residual %.2e, bad %lld\n", t,
                   (long long)nx, (long long)ny, (long long)nz, worst, rho, (long long)nbad);
        }
        free(F);
        free(u);
        free(v);
        free(idx);
        free(q);
    }
    printf("oracle under sanitizers: %d bad cases\n", bad);
    return bad != 0;
}
