/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, serial FP64 reference for the first-order upwind discretisation of the
 * Eikonal equation |grad u| F = 1 (Chacon & Vladimirsky, "A parallel Heap-Cell Method for
 * Eikonal equations", Section 1.1, eq. (2) "eq:Eik_discr").  Only tests/, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no code, header,
 * table or helper with the GPU solver; the GPU solver never calls it.
 *
 * Contents
 *   oracle_fmm          Fast Marching Method (Section 2, FMM paragraph): Dijkstra-like
 *                       acceptance order with a binary min-heap of "considered" nodes.
 *   oracle_jacobi       Brute-force Jacobi iteration V <- min(V, Gamma(V)) from V = +inf
 *                       to an exact floating-point fixed point (Section 1.1: the system can be
 *                       solved iteratively with temporary labels V until they stop changing).
 *   oracle_residual     Per-node residual of eq. (2) written out directly (sum of squared
 *                       one-sided upwind differences minus 1/F^2), max over non-source nodes.
 *
 * Conventions (shared with the GPU solver only through the written interface, not code)
 *   grid     nx*ny*nz nodes, node (i,j,k) at (i h, j h, k h); arrays are row-major with i
 *            fastest: lin = i + nx*(j + ny*k).  Values beyond the grid are +inf (Section 1.1).
 *   sources  the exit nodes Q' (Section 3 notation): fixed at U = q, never recomputed
 *            (Algorithm 2 only updates nodes outside Q').  A node listed twice keeps min q.
 *   F        speed, finite and > 0 at every node; s = h / F is the local travel time.
 *
 * Local solve Gamma.  The paper states that eq. (2) is solved for U_ijk given the neighbour
 * values but prints no formula.  With m_k the smaller of the two axis-k neighbours, eq. (2)
 * at a node reads  sum_k max(U - m_k, 0)^2 = s^2  (multiply eq. (2) by h^2).  Its unique root
 * is found by sorting a <= b <= c and trying one, two, then three terms; the discriminants are
 * written in difference form so that no large-magnitude cancellation occurs.  The expanded
 * form (a+b+c)^2 - 3(a^2+b^2+c^2-s^2) is algebraically equal but loses about log10((U/h)^2)
 * digits.
 *
 * Built with -O2 -ffp-contract=off and without -ffast-math so every operation is a plain
 * IEEE double operation in program order.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* ---------------------------------------------------------------------------------------- */
/* Local solve of eq. (2) at one node.  m0, m1, m2: the upwind (smaller) neighbour value along
 * each axis, +inf when neither neighbour is finite.  s = h / F > 0.  Returns the smallest U
 * with sum_k max(U - m_k, 0)^2 = s^2, or +inf if all m_k are +inf.
 * variant: 0 = the correct solve; 1..3 = deliberately wrong solves used only by the tests
 * that show the pins detect plausible mistakes (1: three-term branch dropped; 2: wrong sign
 * of the square root in the two-term branch; 3: expanded-form three-term discriminant). */
static double orc_gamma(double m0, double m1, double m2, double s, int variant) {
    double a = m0, b = m1, c = m2, t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    if (isinf(a)) return INFINITY;
    double u = a + s;
    if (u <= b) return u;
    /* Two terms: 2u^2 - 2(a+b)u + a^2 + b^2 - s^2 = 0. */
    double d2 = 2.0 * s * s - (a - b) * (a - b);
    if (d2 < 0.0) d2 = 0.0; /* cannot happen when b - a < s; kept for rounding safety */
    if (variant == 2)
        u = (a + b - sqrt(d2)) / 2.0;
    else
        u = (a + b + sqrt(d2)) / 2.0;
    if (u <= c || variant == 1) return u;
    /* Three terms: 3u^2 - 2(a+b+c)u + a^2 + b^2 + c^2 - s^2 = 0. */
    double d3;
    if (variant == 3)
        d3 = (a + b + c) * (a + b + c) - 3.0 * (a * a + b * b + c * c - s * s);
    else
        d3 = 3.0 * s * s - (a - b) * (a - b) - (a - c) * (a - c) - (b - c) * (b - c);
    if (d3 < 0.0) d3 = 0.0;
    return (a + b + c + sqrt(d3)) / 3.0;
}

/* Exported for the closed-form tests of the local solve. */
double oracle_gamma(double m0, double m1, double m2, double s) {
    return orc_gamma(m0, m1, m2, s, 0);
}

static int check_grid(int64_t nx, int64_t ny, int64_t nz, double h) {
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    if (!(h > 0.0) || isinf(h)) return 0;
    return 1;
}

/* Marks the exit nodes and their values.  Returns 0 on success. */
static int place_sources(int64_t nx, int64_t ny, int64_t nz, int64_t nsrc, const int64_t* idx3,
                         const double* q, double* u, uint8_t* fixed) {
    for (int64_t n = 0; n < nsrc; ++n) {
        int64_t i = idx3[3 * n], j = idx3[3 * n + 1], k = idx3[3 * n + 2];
        if (i < 0 || i >= nx || j < 0 || j >= ny || k < 0 || k >= nz) return ORC_EINVAL;
        if (!(q[n] >= 0.0) || isinf(q[n])) return ORC_EINVAL;
        int64_t x = i + nx * (j + ny * k);
        if (!fixed[x] || q[n] < u[x]) u[x] = q[n];
        fixed[x] = 1;
    }
    return ORC_OK;
}

/* ------------------------------------ binary min-heap ------------------------------------ */
/* Keys are (U, linear index) compared lexicographically, so the pop order is deterministic. */
typedef struct {
    int64_t* node; /* heap slot -> node */
    int64_t* pos;  /* node -> heap slot, -1 if absent */
    int64_t size;
    const double* u;
} orc_heap;

static int heap_less(const orc_heap* H, int64_t x, int64_t y) {
    double ux = H->u[x], uy = H->u[y];
    if (ux < uy) return 1;
    if (ux > uy) return 0;
    return x < y;
}

static void heap_place(orc_heap* H, int64_t slot, int64_t x) {
    H->node[slot] = x;
    H->pos[x] = slot;
}

static void heap_sift_up(orc_heap* H, int64_t slot) {
    int64_t x = H->node[slot];
    while (slot > 0) {
        int64_t parent = (slot - 1) / 2;
        int64_t p = H->node[parent];
        if (!heap_less(H, x, p)) break;
        heap_place(H, slot, p);
        slot = parent;
    }
    heap_place(H, slot, x);
}

static void heap_sift_down(orc_heap* H, int64_t slot) {
    int64_t x = H->node[slot];
    for (;;) {
        int64_t l = 2 * slot + 1, r = l + 1, best = slot;
        int64_t bx = x;
        if (l < H->size && heap_less(H, H->node[l], bx)) { best = l; bx = H->node[l]; }
        if (r < H->size && heap_less(H, H->node[r], bx)) { best = r; bx = H->node[r]; }
        if (best == slot) break;
        heap_place(H, slot, bx);
        slot = best;
    }
    heap_place(H, slot, x);
}

static void heap_push_or_decrease(orc_heap* H, int64_t x) {
    if (H->pos[x] < 0) {
        heap_place(H, H->size, x);
        H->size++;
        heap_sift_up(H, H->size - 1);
    } else {
        heap_sift_up(H, H->pos[x]);
    }
}

static int64_t heap_pop(orc_heap* H) {
    int64_t top = H->node[0];
    H->pos[top] = -1;
    H->size--;
    if (H->size > 0) {
        heap_place(H, 0, H->node[H->size]);
        heap_sift_down(H, 0);
    }
    return top;
}

/* ------------------------------------------ FMM ------------------------------------------ */
enum { FAR = 0, TRIAL = 1, KNOWN = 2 };

/* Upwind neighbour along one axis taking only accepted (KNOWN) nodes into account. */
static double known_min(const double* u, const uint8_t* st, int64_t x, int64_t stride,
                        int has_lo, int has_hi) {
    double m = INFINITY;
    if (has_lo && st[x - stride] == KNOWN && u[x - stride] < m) m = u[x - stride];
    if (has_hi && st[x + stride] == KNOWN && u[x + stride] < m) m = u[x + stride];
    return m;
}

static int fmm_impl(int64_t nx, int64_t ny, int64_t nz, double h, const double* F,
                    int64_t nsrc, const int64_t* idx3, const double* q, double* u,
                    int variant, int64_t progress) {
    if (!check_grid(nx, ny, nz, h) || nsrc < 0) return ORC_EINVAL;
    const int64_t M = nx * ny * nz, sy = nx, sz = nx * ny;
    for (int64_t x = 0; x < M; ++x)
        if (!(F[x] > 0.0) || isinf(F[x])) return ORC_EINVAL;
    uint8_t* st = (uint8_t*)calloc((size_t)M, 1);
    uint8_t* fixed = (uint8_t*)calloc((size_t)M, 1);
    orc_heap H;
    H.node = (int64_t*)malloc((size_t)M * sizeof(int64_t));
    H.pos = (int64_t*)malloc((size_t)M * sizeof(int64_t));
    H.size = 0;
    H.u = u;
    if (!st || !fixed || !H.node || !H.pos) {
        free(st); free(fixed); free(H.node); free(H.pos);
        return ORC_ENOMEM;
    }
    for (int64_t x = 0; x < M; ++x) { u[x] = INFINITY; H.pos[x] = -1; }
    int rc = place_sources(nx, ny, nz, nsrc, idx3, q, u, fixed);
    if (rc == ORC_OK) {
        for (int64_t x = 0; x < M; ++x)
            if (fixed[x]) { st[x] = TRIAL; heap_push_or_decrease(&H, x); }
        int64_t accepted = 0;
        while (H.size > 0) {
            int64_t x = heap_pop(&H);
            st[x] = KNOWN;
            if (progress > 0 && ++accepted % progress == 0) {
                fprintf(stderr, "oracle FMM: %lld of %lld nodes accepted\n",
                        (long long)accepted, (long long)M);
                fflush(stderr);
            }
            int64_t i = x % nx, j = (x / nx) % ny, k = x / sz;
            int64_t nb[6];
            int nn = 0;
            if (i > 0) nb[nn++] = x - 1;
            if (i + 1 < nx) nb[nn++] = x + 1;
            if (j > 0) nb[nn++] = x - sy;
            if (j + 1 < ny) nb[nn++] = x + sy;
            if (k > 0) nb[nn++] = x - sz;
            if (k + 1 < nz) nb[nn++] = x + sz;
            for (int t = 0; t < nn; ++t) {
                int64_t y = nb[t];
                if (st[y] == KNOWN || fixed[y]) continue;
                int64_t yi = y % nx, yj = (y / nx) % ny, yk = y / sz;
                double mx = known_min(u, st, y, 1, yi > 0, yi + 1 < nx);
                double my = known_min(u, st, y, sy, yj > 0, yj + 1 < ny);
                double mz = known_min(u, st, y, sz, yk > 0, yk + 1 < nz);
                double v = orc_gamma(mx, my, mz, h / F[y], variant);
                if (v < u[y]) {
                    u[y] = v;
                    st[y] = TRIAL;
                    heap_push_or_decrease(&H, y);
                }
            }
        }
    }
    free(st); free(fixed); free(H.node); free(H.pos);
    return rc;
}

/* Serial FP64 FMM.  F, idx3, q and u are host arrays; u receives nx*ny*nz values.
 * Returns 0, ORC_EINVAL for invalid input (u then unspecified), ORC_ENOMEM. */
int oracle_fmm(int64_t nx, int64_t ny, int64_t nz, double h, const double* F, int64_t nsrc,
               const int64_t* idx3, const double* q, double* u) {
    return fmm_impl(nx, ny, nz, h, F, nsrc, idx3, q, u, 0, 0);
}

/* oracle_fmm that prints a line to stderr after every `progress` accepted nodes (for grids
 * whose solve takes minutes); the arithmetic is that of oracle_fmm. */
int oracle_fmm_progress(int64_t nx, int64_t ny, int64_t nz, double h, const double* F,
                        int64_t nsrc, const int64_t* idx3, const double* q, double* u,
                        int64_t progress) {
    return fmm_impl(nx, ny, nz, h, F, nsrc, idx3, q, u, 0, progress);
}

/* Same as oracle_fmm but with a deliberately wrong local solve (variant 1..3, see
 * orc_gamma).  Used only to show that the tests' pins catch such mistakes. */
int oracle_fmm_planted(int64_t nx, int64_t ny, int64_t nz, double h, const double* F,
                       int64_t nsrc, const int64_t* idx3, const double* q, double* u,
                       int variant) {
    if (variant < 1 || variant > 3) return ORC_EINVAL;
    return fmm_impl(nx, ny, nz, h, F, nsrc, idx3, q, u, variant, 0);
}

/* ---------------------------------------- Jacobi ----------------------------------------- */
/* Upwind neighbour along one axis using all current values (beyond the grid: +inf). */
static double any_min(const double* v, int64_t x, int64_t stride, int has_lo, int has_hi) {
    double m = INFINITY;
    if (has_lo && v[x - stride] < m) m = v[x - stride];
    if (has_hi && v[x + stride] < m) m = v[x + stride];
    return m;
}

/* Brute-force Jacobi: every sweep computes W_x = min(V_x, Gamma_x(V)) for every non-source
 * node from the previous iterate V, then V <- W; stops at the first sweep that changes no
 * value (an exact floating-point fixed point).  Returns the number of sweeps performed
 * (including the final unchanged one), ORC_EINVAL, ORC_ENOMEM, or -3 if max_sweeps ran out. */
int64_t oracle_jacobi(int64_t nx, int64_t ny, int64_t nz, double h, const double* F,
                      int64_t nsrc, const int64_t* idx3, const double* q, int64_t max_sweeps,
                      double* v) {
    if (!check_grid(nx, ny, nz, h) || nsrc < 0) return ORC_EINVAL;
    const int64_t M = nx * ny * nz, sy = nx, sz = nx * ny;
    for (int64_t x = 0; x < M; ++x)
        if (!(F[x] > 0.0) || isinf(F[x])) return ORC_EINVAL;
    uint8_t* fixed = (uint8_t*)calloc((size_t)M, 1);
    double* w = (double*)malloc((size_t)M * sizeof(double));
    if (!fixed || !w) { free(fixed); free(w); return ORC_ENOMEM; }
    for (int64_t x = 0; x < M; ++x) v[x] = INFINITY;
    int64_t rc = place_sources(nx, ny, nz, nsrc, idx3, q, v, fixed);
    int64_t sweeps = 0;
    if (rc == ORC_OK) {
        rc = -3;
        while (sweeps < max_sweeps) {
            ++sweeps;
            int changed = 0;
            for (int64_t k = 0; k < nz; ++k)
                for (int64_t j = 0; j < ny; ++j)
                    for (int64_t i = 0; i < nx; ++i) {
                        int64_t x = i + nx * (j + ny * k);
                        w[x] = v[x];
                        if (fixed[x]) continue;
                        double g = orc_gamma(any_min(v, x, 1, i > 0, i + 1 < nx),
                                             any_min(v, x, sy, j > 0, j + 1 < ny),
                                             any_min(v, x, sz, k > 0, k + 1 < nz),
                                             h / F[x], 0);
                        if (g < v[x]) { w[x] = g; changed = 1; }
                    }
            memcpy(v, w, (size_t)M * sizeof(double));
            if (!changed) { rc = sweeps; break; }
        }
    }
    free(fixed); free(w);
    return rc;
}

/* --------------------------------------- residual ---------------------------------------- */
/* Residual of eq. (2) at every node outside Q', written directly from the equation:
 *   R_x = sum_k max(U_x - m_k, 0)^2 - s_x^2,   s_x = h / F_x,
 * with m_k the smaller axis-k neighbour (+inf beyond the grid).  Scaled to be free of units
 * as rho_x = |R_x| / (s_x * max(U_x, s_x)); a rounding-level solution has rho ~ 1e-15.
 * Returns max rho over non-source nodes with finite U.  Nodes with U = +inf count as violating
 * (rho = +inf) unless all six neighbours are +inf too (an unreachable component).
 * *n_bad receives the number of nodes with rho > bad_tol.  Source nodes are skipped here;
 * their values are checked separately against q. */
double oracle_residual(int64_t nx, int64_t ny, int64_t nz, double h, const double* F,
                       int64_t nsrc, const int64_t* idx3, const double* U, double bad_tol,
                       int64_t* n_bad) {
    if (!check_grid(nx, ny, nz, h) || nsrc < 0) return NAN;
    const int64_t M = nx * ny * nz, sy = nx, sz = nx * ny;
    uint8_t* fixed = (uint8_t*)calloc((size_t)M, 1);
    if (!fixed) return NAN;
    for (int64_t n = 0; n < nsrc; ++n) {
        int64_t i = idx3[3 * n], j = idx3[3 * n + 1], k = idx3[3 * n + 2];
        if (i < 0 || i >= nx || j < 0 || j >= ny || k < 0 || k >= nz) { free(fixed); return NAN; }
        fixed[i + nx * (j + ny * k)] = 1;
    }
    double worst = 0.0;
    int64_t bad = 0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t x = i + nx * (j + ny * k);
                if (fixed[x]) continue;
                double m[3];
                m[0] = any_min(U, x, 1, i > 0, i + 1 < nx);
                m[1] = any_min(U, x, sy, j > 0, j + 1 < ny);
                m[2] = any_min(U, x, sz, k > 0, k + 1 < nz);
                double ux = U[x], rho;
                if (isinf(ux)) {
                    rho = (isinf(m[0]) && isinf(m[1]) && isinf(m[2])) ? 0.0 : INFINITY;
                } else {
                    double s = h / F[x], sum = 0.0;
                    for (int t = 0; t < 3; ++t) {
                        double d = ux - m[t];
                        if (d > 0.0) sum += d * d;
                    }
                    double scale = s * (ux > s ? ux : s);
                    rho = fabs(sum - s * s) / scale;
                }
                if (!(rho <= bad_tol)) ++bad;
                if (!(rho <= worst)) worst = rho;
            }
    free(fixed);
    if (n_bad) *n_bad = bad;
    return worst;
}
