// eik_kernels.hip -- gfx950 kernels of the cell-scheduled Eikonal solver.
//
// Method: Chacon & Vladimirsky, "A parallel Heap-Cell Method for Eikonal equations".
//   * local solve of eq. (2) (Section 1.1) at one node from its three upwind axis values;
//   * modified locking-sweeping update inside a cell (Algorithm 2): active flags, strict
//     decrease, activation of larger neighbours, tagging of "currently downwind" cells;
//   * cell values of eq. (3) with the reset to +inf on removal (Section 4) and the initial
//     cell values of the exit cells;
//   * preferred sweep directions set by the tagging neighbour (Section 4, "Processing cells");
//   * the parallel main loop of Algorithm 3, re-designed for one GPU: every wave64 is a
//     worker that pops cells; cells are popped in rounds from a device worklist, and each
//     round takes the cells whose value lies in the lowest band [min, min + delta) -- a
//     bucketed priority queue in place of the per-thread heaps and locks of Algorithms 3-5
//     (the parallel main loop, "Set Cell Value", "Add Cell").
// Algorithms are numbered in the paper's order: 1 the HCM main loop, 2 the modified LSM update at
// a gridpoint (Section 4), 3 the pHCM pseudocode, 4 Set Cell Value, 5 Add Cell (Section 5).
//
// GPU design notes (what differs from the paper's shared-memory CPU design):
//   * The grid is stored cell-blocked (each r^3 cell contiguous) and every cell also keeps a
//     copy of its six border layers ("faces"), so the one-node halo of a cell is read as six
//     contiguous r^2 runs and the cell as one r^3 run.
//   * A visit stages the cell, its halo and s = h/F in LDS and runs the in-cell sweeps there;
//     a sweep in direction d visits the planes x'+y'+z' = p of the reflected cell coordinates
//     in increasing p (the Cuthill-McKee plane order of Section 3 used inside one cell): nodes
//     of one plane do not depend on each other, so one wave updates a whole plane per step
//     and the result equals a lexicographic Gauss-Seidel sweep in direction d.
//   * Active flags never cross a cell boundary.  Instead the tagging cell sets a dirty bit for
//     the face it changed; the tagged cell activates the layer next to every dirty face.
//   * Rounds are separated by a grid barrier inside one persistent cooperative launch.  The
//     cell state (value, flags, membership) is double-buffered by round parity: a visit in round
//     t only consumes state produced in round t-1, whose data the barrier made visible across
//     the eight XCD-local L2 caches; state produced in round t is consumed in round t+1.
//     Halo values read during a round may be older than a concurrent neighbour's writes; values
//     only decrease, so they are upper bounds, and the neighbour's tag re-queues the cell.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <cstdlib>

#include "eik_internal.h"

namespace eik {

// ------------------------------------------------------------------------------------------
// Constant tables.

// Nodes of a cell of side R grouped by diagonal plane p = x + y + z (canonical direction +++),
// stored as the node's index x + R y + R^2 z in the cell; 0xFFFF marks an unused (step, lane)
// slot.  R is a power of two, so the reflection R - 1 - x of a coordinate is x ^ (R - 1) and a
// sweep direction reflects the whole index with one XOR.  A sweep takes the
// planes in order, 64 nodes per wave step: one step per plane up to r = 8 (at most 48 nodes), and
// a plane of more than 64 nodes (r = 16: up to 192) over consecutive steps.  Nodes of one plane
// are not neighbours of each other, so splitting a plane over steps keeps the plane order.
constexpr int plane_nodes(int R, int p) {
    int n = 0;
    for (int z = 0; z < R; ++z)
        for (int y = 0; y < R; ++y)
            if (p - y - z >= 0 && p - y - z < R) ++n;
    return n;
}
constexpr int plane_steps(int R) {
    int s = 0;
    for (int p = 0; p < 3 * R - 2; ++p) s += (plane_nodes(R, p) + 63) / 64;
    return s;
}

template <int R>
struct PlaneTable {
    static constexpr int NP = 3 * R - 2;
    static constexpr int NSTEP = plane_steps(R);
    uint16_t slot[NSTEP * 64];
    constexpr PlaneTable() : slot() {
        for (int i = 0; i < NSTEP * 64; ++i) slot[i] = 0xFFFF;
        int step = 0;
        for (int p = 0; p < NP; ++p) {
            int n = 0;
            for (int z = 0; z < R; ++z)
                for (int y = 0; y < R; ++y) {
                    int x = p - y - z;
                    if (x < 0 || x >= R) continue;
                    slot[(step + n / 64) * 64 + n % 64] = (uint16_t)(x + R * (y + R * z));
                    ++n;
                }
            step += (n + 63) / 64;
        }
    }
};
static_assert(PlaneTable<4>::NSTEP == 10 && PlaneTable<8>::NSTEP == 22 &&
                  PlaneTable<16>::NSTEP == 88, "one step per plane up to r = 8");

__constant__ PlaneTable<4> kPlanes4 = PlaneTable<4>();
__constant__ PlaneTable<8> kPlanes8 = PlaneTable<8>();
__constant__ PlaneTable<16> kPlanes16 = PlaneTable<16>();

// Two sweep streams on one cell, offset by half a sweep: at step t, lanes [0, n_t) take the
// nodes of plane t of stream 0 and the next lanes take plane (t + H) mod NP of stream 1
// (bit 15 set), H = NP / 2.  The two planes hold at most 49 nodes at r = 8 (13 at r = 4).
template <int R>
struct DualTable {
    static constexpr int NP = 3 * R - 2;
    static constexpr int H = NP / 2;
    uint16_t slot[NP * 64];
    constexpr DualTable() : slot() {
        for (int i = 0; i < NP * 64; ++i) slot[i] = 0xFFFF;
        for (int t = 0; t < NP; ++t) {
            int n = 0;
            for (int stream = 0; stream < 2; ++stream) {
                const int p = stream ? (t + H) % NP : t;
                for (int z = 0; z < R; ++z)
                    for (int y = 0; y < R; ++y) {
                        int x = p - y - z;
                        if (x < 0 || x >= R) continue;
                        slot[t * 64 + n] = (uint16_t)((x + R * (y + R * z)) | (stream << 15));
                        ++n;
                    }
            }
        }
    }
};

__constant__ DualTable<4> kDual4 = DualTable<4>();
__constant__ DualTable<8> kDual8 = DualTable<8>();

template <int R>
__device__ __forceinline__ const uint16_t* dual_slots();
template <>
__device__ __forceinline__ const uint16_t* dual_slots<4>() { return kDual4.slot; }
template <>
__device__ __forceinline__ const uint16_t* dual_slots<8>() { return kDual8.slot; }

template <int R>
__device__ __forceinline__ const uint16_t* plane_slots();
template <>
__device__ __forceinline__ const uint16_t* plane_slots<4>() { return kPlanes4.slot; }
template <>
__device__ __forceinline__ const uint16_t* plane_slots<8>() { return kPlanes8.slot; }
template <>
__device__ __forceinline__ const uint16_t* plane_slots<16>() { return kPlanes16.slot; }

// Gray-code order of the 8 sweep directions; bit a of a direction set = descending along axis a.
__constant__ int kGray[8] = {0, 1, 3, 2, 6, 7, 5, 4};

// Directions preferred by a cell whose face g received new inflow: sweep away from that face.
__device__ __forceinline__ uint32_t pref_mask_for_face(int g) {
    // g: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z
    const uint32_t m[6] = {0x55u, 0xAAu, 0x33u, 0xCCu, 0x0Fu, 0xF0u};
    return m[g];
}

// ------------------------------------------------------------------------------------------
// Small helpers.

// Whether any lane of the wave has p: the ballot's scalar mask compared on the scalar unit
// (HIP's __any goes through a per-lane 0/1 select and a compare).
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0ull; }

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ uint64_t dbits(double d) { return (uint64_t)__double_as_longlong(d); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ uint32_t ld_acquire_u32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_relaxed_u64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Accesses to cell values and face copies.  Under the round barrier (ASYNC = false) they are
// plain loads and stores: the barrier's release/acquire publishes a round's writes to the eight
// XCD-local L2 caches.  Without rounds (ASYNC = true) every such access is an agent-scope
// relaxed atomic, which the hardware keeps coherent across the XCDs without writing back or
// invalidating an L2 (a release or acquire fence costs tens of microseconds there when every
// wave issues one per visit); mem_wait() then orders them against the cell-state atomics.
template <bool ASYNC, typename T>
__device__ __forceinline__ T ld_val(const T* p) {
    if constexpr (ASYNC) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
template <bool ASYNC, typename T>
__device__ __forceinline__ void st_val(T* p, T v) {
    if constexpr (ASYNC) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}
// Write-back of a visit's values (cell nodes and face copies).  With rounds, the stores are
// non-temporal: they leave the XCD's L2 early, so a neighbour visited later in the same round on
// another XCD (which reads face copies at device scope, see stage_cell) more often finds them
// fresh, and the round's release fence has fewer dirty lines to write back (measured: 3.8 ->
// 3.7 visits per cell on the 513^3 maze, 3.4% faster together with the face loads).  The
// min-store build (EIK_DEBUG_MIN_STORES, libeik_minstore.so) writes through an atomic minimum
// of the bit patterns instead: values are >= +0, so their bit order is their order, and an
// active flag carried in the sign bit is ORed in afterwards.  A minimum cannot lose a decrease
// to another writer of the same word, so a result that differs from the plain build's shows
// that two visits wrote one cell at once.
template <bool ASYNC, typename T>
__device__ __forceinline__ void st_writeback(T* p, T v) {
#ifdef EIK_DEBUG_MIN_STORES
    if constexpr (sizeof(T) == 8) {
        unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        atomicMin(q, b & ~(1ull << 63));
        if (b >> 63) atomicOr(q, 1ull << 63);
    } else {
        unsigned int* q = reinterpret_cast<unsigned int*>(p);
        const unsigned int b = __float_as_uint(v);
        atomicMin(q, b & 0x7FFFFFFFu);
        if (b >> 31) atomicOr(q, 0x80000000u);
    }
#else
    if constexpr (ASYNC) st_val<ASYNC>(p, v);
    else __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T*)p);
#endif
}

// Waits until every earlier vector memory access of the wave has completed (stores are then
// visible device-wide, atomics have returned), and keeps the compiler from moving memory
// accesses across it.
__device__ __forceinline__ void mem_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// ------------------------------------------------------------------------------------------
// Square root of a discriminant of the local solve: hardware reciprocal square root refined by
// one Goldschmidt step (which squares its relative error to ~2^-50) and one Newton correction
// (without the rescaling for subnormal or huge arguments that the discriminants here never
// need).  Within about one ulp for d > 0.  The callers use the root only in the case whose
// discriminant exceeds s^2 > 0 (two terms: 2 s^2 - (b - a)^2 with b - a < s; three terms:
// 3 s^2 minus three squared gaps, two of them together below s^2 and the third below s^2), so
// there is no guard for d <= 0: the value then (NaN or inf) is discarded by the caller's select.
__device__ __forceinline__ double disc_sqrt(double d) {
    const double r = __builtin_amdgcn_rsq(d);
    double g = d * r, hh = 0.5 * r;
    const double e = fma(-hh, g, 0.5);
    g = fma(g, e, g);
    hh = fma(hh, e, hh);
    const double res = fma(-g, g, d);
    return fma(res, hh, g);
}

// IEEE minimum / maximum of two doubles as single instructions.  (The library fmin/fmax first
// quiet signalling NaNs with an extra instruction per operand; these values never hold one.)
__device__ __forceinline__ double vmin(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double vmax(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
// min(|a|, |b|): the smaller of two neighbour values whose sign bit may carry an active flag.
__device__ __forceinline__ double vmin_abs(double a, double b) {
    double r;
    asm("v_min_f64 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ float vmin(float a, float b) {
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float vmax(float a, float b) {
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float vmin_abs(float a, float b) {
    float r;
    asm("v_min_f32 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Local solve of eq. (2): the smallest U with sum_k max(U - m_k, 0)^2 = s^2 given the upwind
// axis values m_k (+inf when absent).  With a <= b <= c sorted, g(U) = sum_k max(U - m_k, 0)^2
// is increasing, so the root uses exactly the values below it: one term (a + s) if that does
// not exceed b, else two terms if g restricted to {a, b} reaches s^2 at c, i.e.
// (c - a)^2 + (c - b)^2 >= s^2, else three.  The term count is decided first, so one square
// root serves all cases.  Discriminants are in difference form (no cancellation of O(U^2)
// quantities): k s^2 - sum over pairs of the used values of (m_i - m_j)^2.  With b or c = +inf
// the comparisons select the terms that stay finite.
__device__ __forceinline__ double local_solve(double m0, double m1, double m2, double s) {
    const double t1 = vmin(m0, m1), t2 = vmax(m0, m1);
    const double t3 = vmin(t2, m2), c = vmax(t2, m2);
    const double a = vmin(t1, t3), b = vmax(t1, t3);
    const double ss = s * s;
    const double u1 = a + s;
    const double dab = b - a, dca = c - a, dcb = c - b;
    const double qc = fma(dca, dca, dcb * dcb);  // the terms c adds to the three-term sum
    const bool two = qc >= ss;
    const double d2 = fma(-dab, dab, 2.0 * ss);
    const double d3 = (d2 + ss) - qc;
    const double sum = two ? a + b : (a + b) + c;
    const double u = (sum + disc_sqrt(two ? d2 : d3)) * (two ? 0.5 : (1.0 / 3.0));
    return u1 <= b ? u1 : u;
}

// The local solve in the single-precision mode: FP32 values, sort, term selection and two-term
// root; the three-term root -- the step whose rounding dominates the FP32 error, because its sum
// a + b + c and discriminant are formed at the scale of U -- in FP64 from the FP32 inputs,
// rounded once to FP32.  Hardware FP32 square root (within one ulp).
__device__ __forceinline__ float fsqrt_pos(float d) { return d > 0.f ? __builtin_amdgcn_sqrtf(d) : 0.f; }
__device__ __forceinline__ float local_solve(float m0, float m1, float m2, float s) {
    const float t1 = vmin(m0, m1), t2 = vmax(m0, m1);
    const float t3 = vmin(t2, m2), c = vmax(t2, m2);
    const float a = vmin(t1, t3), b = vmax(t1, t3);
    const float ss = s * s;
    const float u1 = a + s;
    const float dab = b - a, dca = c - a, dcb = c - b;
    const bool two = fmaf(dca, dca, dcb * dcb) >= ss;
    const float u2 = (a + b + fsqrt_pos(fmaf(-dab, dab, 2.f * ss))) * 0.5f;
    const double ad = a, bd = b, cd = c, sd = s;
    const double e1 = bd - ad, e2 = cd - ad, e3 = cd - bd;
    const double d3 = fma(-e2, e2, fma(-e3, e3, fma(-e1, e1, 3.0 * sd * sd)));
    const float u3 = (float)(((ad + bd) + cd + disc_sqrt(d3)) * (1.0 / 3.0));
    return u1 <= b ? u1 : (two ? u2 : u3);
}

// ------------------------------------------------------------------------------------------
// Geometry.

struct CellXYZ {
    int x, y, z;
};

// Cell coordinates of local cell lc of a slot.
__device__ __forceinline__ CellXYZ cell_coords(const Slot& S, int lc) {
    CellXYZ r;
    r.x = lc % S.ncx;
    r.y = (lc / S.ncx) % S.ncy;
    r.z = lc / (S.ncx * S.ncy);
    return r;
}

// Local neighbour cell across face f (0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z); -1 beyond the grid.
__device__ __forceinline__ int cell_neighbour(const Slot& S, int lc, CellXYZ cc, int f) {
    switch (f) {
        case 0: return cc.x > 0 ? lc - 1 : -1;
        case 1: return cc.x + 1 < S.ncx ? lc + 1 : -1;
        case 2: return cc.y > 0 ? lc - S.ncx : -1;
        case 3: return cc.y + 1 < S.ncy ? lc + S.ncx : -1;
        case 4: return cc.z > 0 ? lc - S.ncx * S.ncy : -1;
        default: return cc.z + 1 < S.ncz ? lc + S.ncx * S.ncy : -1;
    }
}

// Interior node of face f given in-plane coordinates (a, b): x-faces use (y, z), y-faces use
// (x, z), z-faces use (x, y).
template <int R>
__device__ __forceinline__ void face_node(int f, int a, int b, int& x, int& y, int& z) {
    const int side = (f & 1) ? R - 1 : 0;
    switch (f >> 1) {
        case 0: x = side; y = a; z = b; break;
        case 1: x = a; y = side; z = b; break;
        default: x = a; y = b; z = side; break;
    }
}

// ------------------------------------------------------------------------------------------
// Per-wave LDS of one cell visit.  The active flag of an interior node (Algorithm 2) is the
// sign bit of its stored value: values are >= +0, so -|U| marks "active" without extra storage
// and is read together with the value.  Every read of a value goes through fabs().

// In-cell solvers.
constexpr int INNER_SWEEP = 0;  // locking sweeps in diagonal-plane order (Algorithm 2)
constexpr int INNER_LIST = 1;   // relaxation over a compacted list of active nodes
constexpr int INNER_DUAL = 2;   // two sweep streams on one cell, half a sweep apart
constexpr int INNER_PAIR = 3;   // two cells swept by one wave, half a sweep apart

template <int R, int INNER, typename UT>
struct WaveLds {
    static constexpr int B = R + 2;
    static constexpr int BOX = B * B * B;
    static constexpr int NC = INNER == INNER_PAIR ? 2 : 1;  // cells held by the wave
    UT U[NC * BOX];       // cell values with a one-node halo (edges/corners unused), per cell
    UT S[NC * R * R * R]; // s = h/F; -1 marks an exit node, 0 a padding node
    int32_t q[64];        // cells newly queued for the next round, not yet published
    uint16_t lst[INNER == INNER_LIST ? 2 : 0][R * R * R];  // lists of the list relaxation
    uint8_t A[INNER == INNER_DUAL ? ((BOX + 7) & ~7) : 0];  // active flags of the dual sweep
};

template <int R>
__device__ __forceinline__ int box_index(int x, int y, int z) {
    constexpr int B = R + 2;
    return (x + 1) + B * ((y + 1) + B * (z + 1));
}

constexpr int log2_side(int R) { return R == 16 ? 4 : (R == 8 ? 3 : 2); }

// Box index of the cell node with index l = x + R y + R^2 z: (x + 1) + B (y + 1) + B^2 (z + 1)
// = l + (B - R) y + (B^2 - R^2) z + (1 + B + B^2).
// The products use the 24-bit multiplier (full rate; y, z < R), and the constant folds into the
// LDS offsets.
template <int R>
__device__ __forceinline__ int box_of_cell_index(uint32_t l) {
    constexpr int B = R + 2, LG = log2_side(R);
    const uint32_t y = (l >> LG) & (uint32_t)(R - 1), z = l >> (2 * LG);
    return (int)(__umul24(z, (uint32_t)(B * B - R * R)) + __umul24(y, (uint32_t)(B - R)) + l) +
           (1 + B + B * B);
}

// XOR mask that reflects a cell index for sweep direction d (bit a set: descending along a).
template <int R>
__device__ __forceinline__ uint32_t reflect_mask(int d) {
    constexpr int LG = log2_side(R);
    return ((d & 1) ? (uint32_t)(R - 1) : 0u) | ((d & 2) ? (uint32_t)(R - 1) << LG : 0u) |
           ((d & 4) ? (uint32_t)(R - 1) << (2 * LG) : 0u);
}

// Per-lane node coordinates of every sweep step (a diagonal plane, or 64 nodes of one), packed
// two steps per register, plus a bit mask of the steps in which the lane has a node.  Loaded
// once per kernel.
template <int R, int INNER>
struct PlaneRegs {
    static constexpr int NS =
        (INNER == INNER_DUAL || INNER == INNER_PAIR) ? 3 * R - 2 : PlaneTable<R>::NSTEP;
    uint32_t pk[(NS + 1) / 2];
    uint32_t valid[(NS + 31) / 32];
    int dummy;  // this lane's scratch slot: a box node on a halo edge, never read
    __device__ __forceinline__ bool has(int p) const { return (valid[p >> 5] >> (p & 31)) & 1u; }
};

template <int R, int INNER>
__device__ __forceinline__ void load_plane_regs(PlaneRegs<R, INNER>& pr, int lane) {
    static_assert((INNER != INNER_DUAL && INNER != INNER_PAIR) || R <= 8,
                  "two sweep streams fit one wave up to r = 8");
    const uint16_t* slots;
    if constexpr (INNER == INNER_DUAL || INNER == INNER_PAIR) slots = dual_slots<R>();
    else slots = plane_slots<R>();
    // Halo edges: lines where two coordinates are -1 or R (12 R nodes); lane -> one of them.
    {
        const int e = lane % (12 * R), edge = e / R, t = e % R;
        const int u = (edge & 1) ? R : -1, v = (edge & 2) ? R : -1;
        const int kind = edge >> 2;
        const int x = kind == 0 ? u : (kind == 1 ? u : t);
        const int y = kind == 0 ? v : (kind == 1 ? t : u);
        const int z = kind == 0 ? t : v;
        pr.dummy = box_index<R>(x, y, z);
    }
#pragma unroll
    for (int w = 0; w < (PlaneRegs<R, INNER>::NS + 31) / 32; ++w) pr.valid[w] = 0;
#pragma unroll
    for (int p = 0; p < PlaneRegs<R, INNER>::NS; ++p) {
        const uint32_t raw = slots[p * 64 + lane];
        const bool ok = raw != 0xFFFFu;
        if (ok) pr.valid[p >> 5] |= 1u << (p & 31);
        const uint32_t e = ok ? raw : 0u;
        if (p & 1) pr.pk[p >> 1] |= e << 16;
        else pr.pk[p >> 1] = e;
    }
}

__device__ __forceinline__ bool is_active(double v) { return __double_as_longlong(v) < 0; }
__device__ __forceinline__ bool is_active(float v) { return __float_as_int(v) < 0; }

// Marks the LDS node p active given its (non-negative) value v: only the word that holds the
// sign bit is written.  Lanes that mark the same node in one step write the same word.
__device__ __forceinline__ void mark_active(double* p, double) {
    __hip_atomic_fetch_or(reinterpret_cast<uint32_t*>(p) + 1, 0x80000000u, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void mark_active(float* p, float) {
    __hip_atomic_fetch_or(reinterpret_cast<uint32_t*>(p), 0x80000000u, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ------------------------------------------------------------------------------------------
// Tagging a neighbour cell for the next round (Algorithm 3 "for each c_k in DN", with Set Cell
// Value = atomic min of the cell value and Add Cell = append to the next round's list unless
// already queued).

// With the earlier cell values (eq. (4), Section 6 "Other cell values") the value is first combined with the cell's kept value (which no
// visit resets), and the kept value lowered to the result.
__device__ __forceinline__ double kept_value(const SolveParams& P, int c, double value) {
    if (!P.cell_value) return value;
    const uint64_t old = atomicMin((unsigned long long*)&P.key_keep[c],
                                   (unsigned long long)dbits(value));
    return fmin(bitsd(old), value);
}

// Slot minima of the cell values queued for round `round`.
__device__ __forceinline__ uint64_t* slot_minkeys(const SolveParams& P, int64_t round) {
    return P.slot_minkey + (size_t)(round & 3) * (size_t)P.nslots;
}

// Single-thread form, used while seeding: queue cell nb for round `round`.
__device__ __forceinline__ void tag_cell(const SolveParams& P, int64_t round, int nb,
                                         uint32_t bits, double value) {
    RoundCtl* ctl_next = &P.ctl[round & 3];
    const int nxt = (int)(round & 1);
    value = kept_value(P, nb, value);
    const uint64_t kb = dbits(value);
    atomicMin((unsigned long long*)&P.key[nxt][nb], (unsigned long long)kb);
    const uint32_t old = atomicOr(&P.flags[nxt][nb], bits | FL_QUEUED);
    if (!(old & FL_QUEUED)) {
        const uint32_t i = atomicAdd(&ctl_next->count, 1u);
        P.list[nxt][i] = nb;
    }
    atomicMin((unsigned long long*)&ctl_next->minkey, (unsigned long long)kb);
    if (P.slot_band)
        atomicMin((unsigned long long*)&slot_minkeys(P, round)[P.cell_slot[nb]],
                  (unsigned long long)kb);
}

// Wave-level publishing of newly queued cells: they collect in the wave's LDS buffer and are
// appended to the next round's list with one atomic per flush.
struct WaveQueue {
    int n;          // entries in the LDS buffer (wave-uniform)
    double minkey;  // per-lane smallest value tagged this round (used with a priority band)
};

// Slot minima of the round whose control block is ctl_next.
__device__ __forceinline__ uint64_t* slot_minkeys_of(const SolveParams& P,
                                                     const RoundCtl* ctl_next) {
    return P.slot_minkey + (size_t)(ctl_next - P.ctl) * (size_t)P.nslots;
}

template <int R, int INNER, typename UT>
__device__ __forceinline__ void queue_flush(const SolveParams& P, int nxt, RoundCtl* ctl_next,
                                            WaveLds<R, INNER, UT>& L, int lane, WaveQueue& wq) {
    if (wq.n == 0) return;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&ctl_next->count, (uint32_t)wq.n);
    base = __shfl(base, 0, 64);
    if (lane < wq.n) P.list[nxt][base + lane] = L.q[lane];
    wq.n = 0;
    wave_sync();
}

// End-of-round form for a whole workgroup (every wave calls it): the W waves' buffers are
// appended with one atomic, so that a round's end does not meet every wave's flush on the one
// count word.
template <int R, int INNER, typename UT, int W>
__device__ __forceinline__ void queue_flush_group(const SolveParams& P, int nxt,
                                                  RoundCtl* ctl_next, WaveLds<R, INNER, UT>& L,
                                                  int lane, int wave, WaveQueue& wq) {
    __shared__ uint32_t s_qn[W];
    __shared__ uint32_t s_qbase;
    if (lane == 0) s_qn[wave] = (uint32_t)wq.n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t total = 0;
        for (int w = 0; w < W; ++w) total += s_qn[w];
        s_qbase = total ? atomicAdd(&ctl_next->count, total) : 0u;
    }
    __syncthreads();
    uint32_t off = s_qbase;
    for (int w = 0; w < wave; ++w) off += s_qn[w];
    if (lane < wq.n) P.list[nxt][off + lane] = L.q[lane];
    wq.n = 0;
    wave_sync();
}

// Every lane with do_tag set tags one cell (any lanes, in parallel): cell value <- min(value),
// flags |= bits | QUEUED, and the cell joins the next round's list unless already queued.
// band_slot: the slot of every tagged cell when they share one (a visit's neighbours), or -1.
template <int R, int INNER, typename UT>
__device__ __forceinline__ void tag_lanes(const SolveParams& P, int nxt, RoundCtl* ctl_next,
                                          WaveLds<R, INNER, UT>& L, int lane, WaveQueue& wq, bool do_tag,
                                          int target, uint32_t bits, double value, int band_slot) {
    bool newq = false;
    if (do_tag) {
        // Cell values are only read by a priority band; without one they are not kept.
        if (P.delta > 0.0) {
            value = kept_value(P, target, value);
            atomicMin((unsigned long long*)&P.key[nxt][target], (unsigned long long)dbits(value));
        }
        const uint32_t old = atomicOr(&P.flags[nxt][target], bits | FL_QUEUED);
        newq = !(old & FL_QUEUED);
        wq.minkey = fmin(wq.minkey, value);
        if (P.slot_band && P.delta > 0.0 && band_slot < 0)
            atomicMin((unsigned long long*)&slot_minkeys_of(P, ctl_next)[P.cell_slot[target]],
                      (unsigned long long)dbits(value));
    }
    if (P.slot_band && P.delta > 0.0 && band_slot >= 0) {
        // One atomic for the visit: the smallest value it queued in its slot.
        const double m = wave_min(do_tag ? value : __builtin_inf());
        if (lane == 0 && m < __builtin_inf())
            atomicMin((unsigned long long*)&slot_minkeys_of(P, ctl_next)[band_slot],
                      (unsigned long long)dbits(m));
    }
    const uint64_t mask = __ballot(newq);
    const int k = __popcll(mask);
    if (k == 0) return;
    if (wq.n + k > 64) queue_flush<R, INNER, UT>(P, nxt, ctl_next, L, lane, wq);
    if (newq) {
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        L.q[wq.n + rank] = target;
    }
    wq.n += k;
    wave_sync();
}

// ------------------------------------------------------------------------------------------
// Scheduling without rounds.  A cell's flag word (flags[0]) carries, besides the tag bits,
// QUEUED (the cell is in the ring or will be pushed by its owner) and RUNNING (a worker is
// visiting it).  A tag ORs its bits and QUEUED in; whoever turns QUEUED on for a cell that is
// not RUNNING pushes it.  A pop exchanges the word for RUNNING (taking the tag bits); at the end
// of the visit the owner clears RUNNING and, if a tag arrived meanwhile (QUEUED set), pushes the
// cell again.  `pending` counts cells queued or being visited: a push adds before the pushed
// cell can be popped, a visit subtracts only after its own pushes, so it reaches 0 exactly when
// no work is left (the pHCM's active cell count, decremented after propagation).

// Whether the host asked this solve to stop (eik_cancel): the cancel word lives in host memory
// mapped into the device's address space, so it is read at system scope.
__device__ __forceinline__ bool cancel_requested(const SolveParams& P) {
    return P.cancel &&
           __hip_atomic_load(P.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) >= P.cancel_seq;
}

// A pseudo-random delay of 0 to 31 short sleeps (up to about 50 us) before a visit when jitter is
// on: the visits of a round and of a ring then interleave in ever different orders, as uneven
// processor speeds do on a CPU.
__device__ __forceinline__ void jitter_delay(const SolveParams& P, uint64_t salt) {
    if (!P.jitter) return;
    uint64_t z = P.jitter + salt * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int n = (int)__builtin_amdgcn_readfirstlane((uint32_t)(z & 31u));
    for (int i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(63);
}

__device__ __forceinline__ void async_cancel(const SolveParams& P) {
    atomicCAS(P.status, 0, EIK_ECANCELLED_DEV);
    __hip_atomic_store(P.async_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// FIFO ring (no band): lanes with `push` set append their cell (one counter update per wave).
__device__ __forceinline__ void fifo_push(const SolveParams& P, int lane, bool push, int c) {
    const uint64_t mask = __ballot(push);
    const int k = __popcll(mask);
    if (k == 0) return;
    unsigned long long base = 0;
    if (lane == 0) {
        atomicAdd(P.async_pending, (unsigned long long)k);
        mem_wait();  // counted before any of them can be popped and visited
        base = atomicAdd(P.async_tail, (unsigned long long)k);
    }
    base = __shfl(base, 0, 64);
    if (push) {
        const uint64_t pos = base + (uint64_t)__popcll(mask & ((1ull << lane) - 1ull));
        int32_t* slotp = &P.list[0][pos % (uint64_t)(2 * P.ncells + kRingExtra)];
        // The position is empty unless its previous occupant is still being read by the
        // worker that took it (see kRingExtra).
        uint64_t polls = 0;
        while (__hip_atomic_load(slotp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != -1) {
            __builtin_amdgcn_s_sleep(1);
            if (++polls > P.watchdog_polls) {
                async_cancel(P);
                break;
            }
        }
        __hip_atomic_store(slotp, (int32_t)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Bucketed rings (a band of width delta): control words and the bucket of a cell value.
__device__ __forceinline__ unsigned long long* bq_head(const SolveParams& P, int b) {
    return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(P.bq_ctl) + b * 128);
}
__device__ __forceinline__ unsigned long long* bq_tail(const SolveParams& P, int b) {
    return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(P.bq_ctl) + b * 128 + 64);
}
__device__ __forceinline__ unsigned long long* bq_low(const SolveParams& P) {
    return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(P.bq_ctl) +
                                                 kBuckets * 128);
}
// Absolute bucket floor(value / delta), moved into the window [low, low + kBuckets): a value
// below the lowest bucket joins it (the front moved past it), one beyond the window joins the
// last bucket.
__device__ __forceinline__ uint64_t bucket_of(const SolveParams& P, double value, uint64_t low) {
    const double a = value / P.delta;
    uint64_t A = a < 1.0e18 ? (uint64_t)a : ~0ull;
    if (A < low) A = low;
    if (A > low + (kBuckets - 1)) A = low + (kBuckets - 1);
    return A;
}

// A bucket ring position p holds a 64-bit word: the lap p / bq_cap + 1 in its high half and a
// cell id (or kAbandoned) in its low half; a word of an older lap means "free".  Tickets are
// taken with fetch-and-add on both ends, so no pop retries on a contended head: a wave that
// took a ticket past the last push waits briefly, then marks the position abandoned, and the
// push that reaches it takes another position.
constexpr uint32_t kAbandoned = 0xFFFFFFFFu;

__device__ __forceinline__ unsigned long long* bq_slot(const SolveParams& P, int b, uint64_t pos) {
    return reinterpret_cast<unsigned long long*>(P.bq_ring) + (size_t)b * (size_t)P.bq_cap +
           pos % (uint64_t)P.bq_cap;
}

__device__ __forceinline__ void bq_push(const SolveParams& P, int lane, bool push, int c,
                                        double value) {
    const uint64_t mask = __ballot(push);
    const int k = __popcll(mask);
    if (k == 0) return;
    if (lane == 0) {
        atomicAdd(P.async_pending, (unsigned long long)k);
        mem_wait();  // counted before any of them can be popped and visited
    }
    if (push) {
        const uint64_t low =
            __hip_atomic_load(bq_low(P), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int b = (int)(bucket_of(P, value, low) % (uint64_t)kBuckets);
        uint64_t tries = 0;
        for (bool done = false; !done;) {
            const uint64_t pos = atomicAdd(bq_tail(P, b), 1ull);
            const uint64_t lap = pos / (uint64_t)P.bq_cap + 1;
            unsigned long long* sp = bq_slot(P, b, pos);
            unsigned long long v = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while ((v >> 32) < lap) {  // free in this lap: claim it for the cell
                const unsigned long long prev =
                    atomicCAS(sp, v, (unsigned long long)((lap << 32) | (uint32_t)c));
                if (prev == v) {
                    done = true;
                    break;
                }
                v = prev;
            }
            // Otherwise the wave holding this ticket gave up on it: take another position.
            if (!done && ++tries > P.watchdog_polls) {
                async_cancel(P);
                break;
            }
        }
    }
}

// Pop of one ticket of bucket b by lane 0: the cell, or -1 if the position stayed empty for a
// short while (and is now marked abandoned).
__device__ __forceinline__ int bq_take(const SolveParams& P, int b) {
    const uint64_t t = atomicAdd(bq_head(P, b), 1ull);
    const uint64_t lap = t / (uint64_t)P.bq_cap + 1;
    unsigned long long* sp = bq_slot(P, b, t);
    int waits = 0;
    unsigned long long v = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if ((v >> 32) == lap) return (int)(uint32_t)v;  // the push of position t
        if (++waits > 8) {
            const unsigned long long prev =
                atomicCAS(sp, v, (unsigned long long)((lap << 32) | kAbandoned));
            if (prev == v) return -1;
            v = prev;  // the push arrived meanwhile
            continue;
        }
        __builtin_amdgcn_s_sleep(4);
        v = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ void queue_push(const SolveParams& P, int lane, bool push, int c,
                                           double value) {
    if (P.delta > 0.0) bq_push(P, lane, push, c, value);
    else fifo_push(P, lane, push, c);
}

// Every lane with do_tag set tags one cell (see above); with a band the cell value is lowered
// to `value` first (eq. (3), or eq. (4) combined with the kept value) and a pushed cell goes to
// the bucket of its value.
__device__ __forceinline__ void tag_lanes_async(const SolveParams& P, int lane, bool do_tag,
                                                int target, uint32_t bits, double value) {
    bool push = false;
    double key = value;
    if (do_tag) {
        if (P.delta > 0.0) {
            key = kept_value(P, target, value);
            const uint64_t old = atomicMin((unsigned long long*)&P.key[0][target],
                                           (unsigned long long)dbits(key));
            key = fmin(bitsd(old), key);
        }
        const uint32_t old = atomicOr(&P.flags[0][target], bits | FL_QUEUED);
        push = !(old & (FL_QUEUED | FL_RUNNING));
    }
    queue_push(P, lane, push, target, key);
}

// Pop of one cell by lane 0 of a wave: the next ticket of the FIFO ring, or a ticket of the
// lowest non-empty bucket.  Returns the cell, or -1 once no cell is queued or being visited
// (or the watchdog cancelled the launch).
__device__ __forceinline__ int pop_cell(const SolveParams& P, int lane) {
    int c = -1;
    if (P.delta > 0.0) {
        uint64_t polls = 0;
        for (;;) {
            // Lane j looks at bucket low + j; one memory round trip for the whole window.
            const uint64_t low =
                __hip_atomic_load(bq_low(P), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int b = (int)((low + (uint64_t)lane) % (uint64_t)kBuckets);
            const uint64_t hd = __hip_atomic_load(bq_head(P, b), __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t tl = __hip_atomic_load(bq_tail(P, b), __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t nonempty = __ballot(hd < tl);
            if (nonempty) {
                const int j = __builtin_ctzll(nonempty);
                int got = -1;
                if (lane == 0) {
                    // The lowest bucket is empty: the window starts at the first non-empty one.
                    if (j > 0)
                        atomicCAS(bq_low(P), (unsigned long long)low,
                                  (unsigned long long)(low + (uint64_t)j));
                    got = bq_take(P, (int)((low + (uint64_t)j) % (uint64_t)kBuckets));
                }
                got = __shfl(got, 0, 64);
                if (got >= 0) return got;
                if (__hip_atomic_load(P.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    return -1;
                if (++polls > P.watchdog_polls) {
                    if (lane == 0) async_cancel(P);
                    return -1;
                }
                continue;  // overtaken by other waves: look again
            }
            if (__hip_atomic_load(P.async_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                return -1;
            if (++polls > P.watchdog_polls) {
                if (lane == 0) async_cancel(P);
                return -1;
            }
            __builtin_amdgcn_s_sleep(16);
        }
    }
    if (lane == 0) {
        const uint64_t cap = (uint64_t)(2 * P.ncells + kRingExtra);
        const uint64_t t = atomicAdd(P.async_head, 1ull);
        int32_t* sp = &P.list[0][t % cap];
        uint64_t polls = 0;
        for (;;) {
            const int v = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v >= 0) {
                c = v;
                break;
            }
            if ((polls & 3) == 0 &&
                __hip_atomic_load(P.async_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                break;
            if (++polls > P.watchdog_polls) {
                async_cancel(P);
                break;
            }
            __builtin_amdgcn_s_sleep(16);
        }
        if (c >= 0) __hip_atomic_store(sp, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return __shfl(c, 0, 64);
}

// ------------------------------------------------------------------------------------------
// One visit of cell c by one wave: stage in, locking sweeps until no change, write back,
// tag currently-downwind neighbours.

struct VisitCounters {
    unsigned long long sweeps, updates, requeued;
    unsigned long long cyc_stage, cyc_sweep, cyc_write;
};

__device__ __forceinline__ unsigned long long cycles() { return __builtin_readcyclecounter(); }

// Box offset of the halo node across face f from the border node.
template <int R>
__device__ __forceinline__ int face_step(int f) {
    constexpr int B = R + 2;
    const int axis = f >> 1, dir = (f & 1) ? 1 : -1;
    return dir * (axis == 0 ? 1 : (axis == 1 ? B : B * B));
}

// Stage-in of one cell into the wave's LDS: cell values, s = h/F and the halo (the
// neighbours' opposite face copies, +inf beyond the grid).  The face copies are read at device
// scope (past a line the XCD's L2 may hold from earlier in the round), so that faces written
// during the round by neighbours on other XCDs are seen when they have reached memory; any
// value read is an upper bound of the solution either way.
template <int R, typename FT, typename UT, bool ASYNC>
__device__ __forceinline__ void stage_cell(const Slot& S, int lc, CellXYZ cc, UT* __restrict__ U,
                                           UT* __restrict__ Sv, int lane) {
    constexpr int R2 = R * R, R3 = R * R * R;
    constexpr int FPL = (R2 + 63) / 64;
    const UT INF = (UT)__builtin_inf();
    const UT* __restrict__ ug = reinterpret_cast<const UT*>(S.u) + (size_t)lc * R3;
    const UT* __restrict__ faces = reinterpret_cast<const UT*>(S.faces);
    const FT* __restrict__ fg = reinterpret_cast<const FT*>(S.f) + (size_t)lc * R3;
    // Stage in: cell values, s = h/F and the halo (the neighbours' opposite face copies, +inf
    // beyond the grid).  Every load is issued before any is used, so the visit waits for one
    // memory round trip instead of one per load (up to r = 8; at r = 16, one per 16 nodes a
    // lane, so that the values in flight fit the registers).
    static_assert(R3 % 64 == 0, "whole 64-lane passes over the cell");
    constexpr int PER = R3 / 64;
    constexpr int CH = PER < 16 ? PER : 16;
    UT hv[6][FPL];
#pragma unroll
    for (int k0 = 0; k0 < PER; k0 += CH) {
        UT uv[CH];
        FT fv[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            uv[k] = ld_val<ASYNC>(&ug[lane + 64 * (k0 + k)]);
            fv[k] = fg[lane + 64 * (k0 + k)];
        }
        if (k0 == 0) {
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                const int nb = cell_neighbour(S, lc, cc, f);
                // Beyond the grid the cell's own face is read (an address inside the array) and
                // ignored.
                const size_t src = ((size_t)(nb >= 0 ? nb : lc) * 6 + (f ^ 1)) * R2 + lane;
#pragma unroll
                for (int j = 0; j < FPL; ++j) {
                    hv[f][j] = lane + 64 * j < R2 ? ld_val<true>(&faces[src + 64 * j]) : INF;
                    if (nb < 0) hv[f][j] = INF;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int l = lane + 64 * (k0 + k);
            const int x = l % R, y = (l / R) % R, z = l / R2;
            U[box_index<R>(x, y, z)] = uv[k];
            // s = h / F formed in FP64 and rounded once to the value type.
            Sv[l] = fv[k] > FT(0) ? (UT)(S.h / (double)fv[k])
                                   : (fv[k] < FT(0) ? UT(-1) : UT(0));
        }
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
#pragma unroll
        for (int j = 0; j < FPL; ++j) {
            const int e = lane + 64 * j;
            if (e < R2) {
                int x, y, z;
                face_node<R>(f, e % R, e / R, x, y, z);
                U[box_index<R>(x, y, z) + face_step<R>(f)] = hv[f][j];
            }
        }
    }
    wave_sync();
}

// Write-back of one visited cell whose box (with halo) is U: the cell's values (with their
// active flags if keep_active), every face copy with a decreased border node, and the tag of each
// neighbour across a face with new inflow (eq. (3) value: the smallest newly decreased border
// value below the neighbour's value; eq. (4): the largest one plus the time to the middle of the
// neighbour).  Lane tag_base + f takes the tag of face f.
template <int R, typename FT, typename UT, bool ASYNC>
__device__ __forceinline__ void publish_cell(const SolveParams& P, const Slot& S, int lc,
                                             CellXYZ cc, const UT* __restrict__ U,
                                             const UT (&before)[6][(R * R + 63) / 64],
                                             bool visit_changed, bool keep_active, int lane,
                                             int tag_base, bool& my_tag, int& my_target,
                                             uint32_t& my_bits, double& my_value) {
    constexpr int R2 = R * R, R3 = R * R * R;
    constexpr int FPL = (R2 + 63) / 64;
    const UT INF = (UT)__builtin_inf();
    if (!visit_changed) return;
    UT* __restrict__ uw = reinterpret_cast<UT*>(S.u) + (size_t)lc * R3;
    UT* __restrict__ fw = reinterpret_cast<UT*>(S.faces);
    for (int l = lane; l < R3; l += 64) {
        const int x = l % R, y = (l / R) % R, z = l / R2;
        const UT v = U[box_index<R>(x, y, z)];
        st_writeback<ASYNC>(&uw[l], keep_active ? v : fabs(v));
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int nb = cell_neighbour(S, lc, cc, f);
        bool ch = false, inflow = false;
        UT v[FPL], in_min = INF, in_max = -INF;
#pragma unroll
        for (int j = 0; j < FPL; ++j) {
            const int e = lane + 64 * j;
            v[j] = INF;
            if (e < R2) {
                int x, y, z;
                face_node<R>(f, e % R, e / R, x, y, z);
                const int b = box_index<R>(x, y, z);
                v[j] = fabs(U[b]);
                const bool chj = v[j] < before[f][j];
                const bool inj = chj && v[j] < fabs(U[b + face_step<R>(f)]);
                ch |= chj;
                inflow |= inj;
                in_min = inj ? vmin(in_min, v[j]) : in_min;
                in_max = inj ? vmax(in_max, v[j]) : in_max;
            }
        }
        if (__any(ch)) {
#pragma unroll
            for (int j = 0; j < FPL; ++j)
                if (lane + 64 * j < R2)
                    st_writeback<ASYNC>(&fw[((size_t)lc * 6 + f) * R2 + lane + 64 * j], v[j]);
        }
        if (nb >= 0 && __any(inflow)) {
            double kv = (double)wave_min(in_min);
            if (P.cell_value) {
                kv = (double)wave_max(in_max);
                if (lane == tag_base + f) {
                    const CellXYZ nc = cell_coords(S, nb);
                    const int ex = min(R, S.nx - nc.x * R), ey = min(R, S.ny - nc.y * R),
                              ez = min(R, S.nz - nc.z * R);
                    const int mx = min(R / 2, ex - 1), my = min(R / 2, ey - 1),
                              mz = min(R / 2, ez - 1);
                    const double fv = (double)reinterpret_cast<const FT*>(S.f)[
                        (size_t)nb * R3 + mx + R * (my + R * mz)];
                    if (fv > 0.0) kv += 0.5 * (R * S.h + S.h) / fv;
                }
            }
            if (lane == tag_base + f) {
                const int g = f ^ 1;
                my_tag = true;
                my_target = S.cell_base + nb;
                my_bits = (1u << g) | (pref_mask_for_face(g) << FL_DIR_SHIFT);
                my_value = kv;
            }
        }
    }
}

template <int R, typename FT, int INNER, typename UT, bool ASYNC = false>
__device__ __forceinline__ void visit_cell(const SolveParams& P, int c, int slot, uint32_t fl,
                                           double popped_key, WaveLds<R, INNER, UT>& L,
                                           const PlaneRegs<R, INNER>& pr, int lane,
                                           RoundCtl* ctl_next, int nxt, VisitCounters& cnt,
                                           WaveQueue& wq) {
    constexpr int R2 = R * R, R3 = R * R * R, B = R + 2, NP = 3 * R - 2;
    constexpr int NS = PlaneRegs<R, INNER>::NS;
    // face nodes per lane: one up to r = 8, four at r = 16
    constexpr int FPL = (R2 + 63) / 64;
    constexpr int BOFF = 1 + B + B * B;
    const UT INF = (UT)__builtin_inf();
    const unsigned long long t0 = cycles();
    // The cell's grid (slot, looked up by the pop) and its local index there; c itself is a
    // global cell id.
    c = __builtin_amdgcn_readfirstlane(c);
    slot = __builtin_amdgcn_readfirstlane(slot);
    const Slot S = P.slots[slot];
    const int lc = c - S.cell_base;
    const CellXYZ cc = cell_coords(S, lc);
    stage_cell<R, FT, UT, ASYNC>(S, lc, cc, L.U, L.S, lane);
    // Border values before the visit (every visit publishes its border, so these equal the
    // published face copies; a border node below them has decreased), then the initial active
    // set: every node on a first visit, otherwise the layer next to each face that received new
    // inflow (plus, after a capped visit, the active flags it stored).
    UT before[6][FPL];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
#pragma unroll
        for (int j = 0; j < FPL; ++j) {
            const int e = lane + 64 * j;
            before[f][j] = INF;
            if (e < R2) {
                int x, y, z;
                face_node<R>(f, e % R, e / R, x, y, z);
                before[f][j] = fabs(L.U[box_index<R>(x, y, z)]);
            }
        }
    }
    wave_sync();
    // Marks node b active: the sign bit of its value, or its flag byte for the dual sweep.
    auto activate = [&](int b) {
        if constexpr (INNER == INNER_DUAL) L.A[b] = 1;
        else L.U[b] = -fabs(L.U[b]);
    };
    if constexpr (INNER == INNER_DUAL) {
        for (int b = lane; b < WaveLds<R, INNER, UT>::BOX; b += 64) L.A[b] = 0;
        wave_sync();
    }
    if (fl & FL_ALL) {
        for (int l = lane; l < R3; l += 64) {
            const int x = l % R, y = (l / R) % R, z = l / R2;
            if (L.S[l] > UT(0)) activate(box_index<R>(x, y, z));
        }
    } else {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
#pragma unroll
            for (int j = 0; j < FPL; ++j) {
                const int e = lane + 64 * j;
                if ((fl & (1u << f)) && e < R2) {
                    int x, y, z;
                    face_node<R>(f, e % R, e / R, x, y, z);
                    if (L.S[x + R * (y + R * z)] > UT(0)) activate(box_index<R>(x, y, z));
                }
            }
        }
    }
    wave_sync();

    const unsigned long long t1 = cycles();
    bool visit_changed = false, requeue = false;
    // How a capped visit resumes: with its stored active flags, or (dual sweeps) with every node
    // active.
    uint32_t requeue_bits = INNER == INNER_DUAL ? FL_ALL : 0u;
    unsigned int upd = 0;
    int nsweeps = 0;
    const bool track_dec = S.tol > 0.0;
    if constexpr (INNER == INNER_SWEEP) {
        // Sweeps: preferred directions first (Gray order), then the default Gray cycle.  A sweep in
        // direction d visits the planes of the reflected coordinates x ^ mx etc. in increasing order.
        // A visit resumed after the sweep cap continues the Gray cycle where the capped one
        // stopped.
        const uint32_t pref = (fl >> FL_DIR_SHIFT) & 0xFFu;
        int pi = 0, ci = (fl & FL_GRAY_SET) ? (int)((fl >> FL_GRAY_SHIFT) & 7u) : 0;
        int last_gi = 0;
        for (;;) {
            int d = -1;
            while (pi < 8) {
                const int gi = pi++;
                if (pref & (1u << kGray[gi])) { d = kGray[gi]; last_gi = gi; break; }
            }
            if (d < 0) {
                last_gi = ci & 7;
                d = kGray[last_gi];
                ++ci;
            }
            const uint32_t mref = reflect_mask<R>(d);
            bool changed = false;
            UT maxdec = UT(0);
    #pragma unroll
            for (int p = 0; p < NS; ++p) {
                uint32_t e = (pr.pk[p >> 1] >> ((p & 1) * 16)) & 0xFFFFu;
                // Keep the decode inside the sweep loop: hoisting the NS decoded addresses out
                // of it costs more registers than the few ALU operations it saves.
                asm volatile("" : "+v"(e));
                const uint32_t lr = e ^ mref;
                const int l = (int)lr;
                const int b = box_of_cell_index<R>(lr);
                UT raw = L.U[b];
                UT s = L.S[l];
                UT xm = L.U[b - 1], xp = L.U[b + 1];
                UT ym = L.U[b - B], yp = L.U[b + B];
                UT zm = L.U[b - B * B], zp = L.U[b + B * B];
                // Issue every LDS read of the step before the activity test: one LDS round trip.
                asm volatile("" : "+v"(raw), "+v"(s), "+v"(xm), "+v"(xp), "+v"(ym), "+v"(yp),
                             "+v"(zm), "+v"(zp));
                const bool act = pr.has(p) && is_active(raw);
                if (wave_any(act)) {
                    // An active lane stores its value back (|raw| clears the flag); a decrease
                    // activates every neighbour that is inactive (sign clear) and larger than
                    // the new value, which the raw value tells in one comparison.  Neighbour
                    // values enter the local solve through |.| (the abs modifier of the min).
                    // Two lanes never store different values to one node in one step (a plane's
                    // nodes are not neighbours of each other; activations of a shared neighbour
                    // agree).  The stores are predicated, at fixed offsets from the lane's node.
                    const UT old = fabs(raw);
                    const UT g = local_solve(vmin_abs(xm, xp), vmin_abs(ym, yp),
                                             vmin_abs(zm, zp), s);
                    const bool live = act && s > UT(0);
                    const bool dec = live && g < old;
                    upd += (unsigned)__popcll(__ballot(live));  // wave total, scalar unit
                    UT* const ub = &L.U[b];
                    if (act) ub[0] = dec ? g : old;
                    changed |= dec;
                    // A step in which no lane decreased activates nothing (one wave vote).
                    if (wave_any(dec)) {
                        if (track_dec && dec) maxdec = vmax(maxdec, old - g);
                        if (dec && xm > g) mark_active(ub - 1, xm);
                        if (dec && xp > g) mark_active(ub + 1, xp);
                        if (dec && ym > g) mark_active(ub - B, ym);
                        if (dec && yp > g) mark_active(ub + B, yp);
                        if (dec && zm > g) mark_active(ub - B * B, zm);
                        if (dec && zp > g) mark_active(ub + B * B, zp);
                    }
                }
                wave_sync();
            }
            ++nsweeps;
            const bool any_changed = __any(changed);
            visit_changed |= any_changed;
            if (!any_changed) break;
            // Done when no node is left active (all were evaluated in this sweep except those
            // activated in planes it had already passed): saves the confirming sweep.
            bool left = false;
            for (int l = lane; l < R3; l += 64) {
                const int x = l % R, y = (l / R) % R, z = l / R2;
                left |= is_active(L.U[box_index<R>(x, y, z)]);
            }
            if (!__any(left)) break;
            if (track_dec && (double)wave_max(maxdec) <= S.tol) break;
            if (nsweeps >= P.max_sweeps) {
                requeue = true;
                requeue_bits = FL_GRAY_SET | ((uint32_t)((last_gi + 1) & 7) << FL_GRAY_SHIFT);
                break;
            }
        }
    } else if constexpr (INNER == INNER_DUAL) {
        // Two sweep streams on the cell at once, half a sweep apart: at step t stream 0
        // updates plane t of its direction and stream 1 plane t + H of its own.  For two
        // directions that differ in one or two axes the two planes never share a node (their
        // plane indices differ by an odd number below H, or by an even number, never by H),
        // so each node has one writer per step; reads of nodes the other stream writes in the
        // same step see the older value (an upper bound), which the activation flags repair.
        // Per step: values first, then the own flags cleared, then neighbour flags set, so an
        // activation is never lost.  Directions come from the same sequence as the sweeps
        // (preferred ones first, then the Gray cycle); a stream never takes the direction
        // opposite to the other stream's (the one pair whose planes can meet).
        constexpr int H = NP / 2;
        const uint32_t pref = (fl >> FL_DIR_SHIFT) & 0xFFu;
        int pi = 0, ci = 0;
        auto next_dir = [&]() {
            while (pi < 8) {
                const int cand = kGray[pi++];
                if (pref & (1u << cand)) return cand;
            }
            return kGray[(ci++) & 7];
        };
        int d0 = next_dir();
        int d1 = next_dir();
        if (__popc((uint32_t)(d0 ^ d1)) == 3) d1 = d0;
        bool done = false;
        UT maxdec = UT(0), dec_prev = UT(0);
        bool changed = false;
        const int dm = pr.dummy;
        while (!done) {
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                if (t == 0 && nsweeps > 0) {
                    d0 = next_dir();
                    if (__popc((uint32_t)(d0 ^ d1)) == 3) d0 = d1;
                }
                if (t == H && nsweeps > 1) {
                    d1 = next_dir();
                    if (__popc((uint32_t)(d0 ^ d1)) == 3) d1 = d0;
                }
                const uint32_t mref0 = reflect_mask<R>(d0), mref1 = reflect_mask<R>(d1);
                uint32_t e = (pr.pk[t >> 1] >> ((t & 1) * 16)) & 0xFFFFu;
                asm volatile("" : "+v"(e));
                const uint32_t lr = (e & 0x7FFFu) ^ ((e & 0x8000u) ? mref1 : mref0);
                const int l = (int)lr;
                const int b = box_of_cell_index<R>(lr);
                UT old = L.U[b];
                UT s = L.S[l];
                UT xm = L.U[b - 1], xp = L.U[b + 1];
                UT ym = L.U[b - B], yp = L.U[b + B];
                UT zm = L.U[b - B * B], zp = L.U[b + B * B];
                uint32_t af = L.A[b];
                asm volatile("" : "+v"(old), "+v"(s), "+v"(xm), "+v"(xp), "+v"(ym), "+v"(yp),
                             "+v"(zm), "+v"(zp), "+v"(af));
                const bool act = pr.has(t) && af != 0u;
                if (__any(act)) {
                    const UT g = local_solve(vmin(xm, xp), vmin(ym, yp), vmin(zm, zp), s);
                    const bool live = act && s > UT(0);
                    const bool dec = live && g < old;
                    upd += (unsigned)__popcll(__ballot(live));  // wave total, scalar unit
                    changed |= dec;
                    if (track_dec && dec) maxdec = vmax(maxdec, old - g);
                    L.U[dec ? b : dm] = g;
                    L.A[act ? b : dm] = 0;
                    L.A[(dec && xm > g) ? b - 1 : dm] = 1;
                    L.A[(dec && xp > g) ? b + 1 : dm] = 1;
                    L.A[(dec && ym > g) ? b - B : dm] = 1;
                    L.A[(dec && yp > g) ? b + B : dm] = 1;
                    L.A[(dec && zm > g) ? b - B * B : dm] = 1;
                    L.A[(dec && zp > g) ? b + B * B : dm] = 1;
                }
                wave_sync();
                if (t == H - 1 || t == NP - 1) {
                    // One sweep's worth of steps (H steps of two streams) has passed.
                    ++nsweeps;
                    const bool any_changed = __any(changed);
                    visit_changed |= any_changed;
                    bool left = false;
                    for (int q = lane; q < R3; q += 64) {
                        const int qx = q % R, qy = (q / R) % R, qz = q / R2;
                        left |= L.A[box_index<R>(qx, qy, qz)] != 0;
                    }
                    // The tol test needs a complete sweep: the last NP steps hold one for the
                    // stream whose sweep began NP steps ago.
                    const UT dec_half = track_dec ? wave_max(maxdec) : UT(0);
                    const bool small =
                        track_dec && nsweeps >= 2 && (double)vmax(dec_half, dec_prev) <= S.tol;
                    dec_prev = dec_half;
                    if (!__any(left) || small) {
                        done = true;
                        break;
                    }
                    // The cap applies at the end of a cycle, after which stream 0 has swept
                    // every node once: a capped visit still evaluates every active node.
                    if (t == NP - 1 && nsweeps >= P.max_sweeps) {
                        requeue = true;
                        done = true;
                        break;
                    }
                    changed = false;
                    maxdec = UT(0);
                }
            }
        }
    } else {
        // Relaxation over a list of active nodes (the cell sub-problem of Section 4 solved by a
        // label-correcting iteration instead of sweeps, which Section 5 allows): every pass
        // evaluates the listed nodes in dense 64-lane chunks, and a node that decreases queues
        // its larger in-cell neighbours for the next pass (Algorithm 2 activation).  The sign bit
        // of a value means "listed and not yet evaluated"; setting it with an LDS atomic
        // dedupes the lists.  Chunks see earlier chunks' results (values only decrease), so the
        // iteration reaches the same fixed point as the sweeps.
        int n_cur = 0, cur = 0;
        for (int base = 0; base < R3; base += 64) {
            const int l = base + lane;
            bool on = false;
            if (l < R3) {
                const int x = l % R, y = (l / R) % R, z = l / R2;
                on = is_active(L.U[box_index<R>(x, y, z)]);
            }
            const uint64_t m = __ballot(on);
            if (on) L.lst[0][n_cur + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)l;
            n_cur += __popcll(m);
        }
        wave_sync();
        const uint64_t below = (1ull << lane) - 1ull;
        while (n_cur > 0) {
            int n_next = 0;
            bool changed = false;
            UT maxdec = UT(0);
            for (int base = 0; base < n_cur; base += 64) {
                const bool valid = base + lane < n_cur;
                const int l = valid ? (int)L.lst[cur][base + lane] : 0;
                const int x = l % R, y = (l / R) % R, z = l / R2;
                const int b = x + B * (y + B * z) + BOFF;
                UT raw = L.U[b];
                UT s = L.S[l];
                UT xm = L.U[b - 1], xp = L.U[b + 1];
                UT ym = L.U[b - B], yp = L.U[b + B];
                UT zm = L.U[b - B * B], zp = L.U[b + B * B];
                asm volatile("" : "+v"(raw), "+v"(s), "+v"(xm), "+v"(xp), "+v"(ym), "+v"(yp),
                             "+v"(zm), "+v"(zp));
                const UT old = fabs(raw);
                xm = fabs(xm); xp = fabs(xp); ym = fabs(ym);
                yp = fabs(yp); zm = fabs(zm); zp = fabs(zp);
                const UT g = local_solve(fmin(xm, xp), fmin(ym, yp), fmin(zm, zp), s);
                const bool live = valid && s > UT(0);
                const bool dec = live && g < old;
                upd += (unsigned)__popcll(__ballot(live));  // wave total, scalar unit
                L.U[valid ? b : 0] = dec ? g : old;  // positive: no longer listed
                if (dec) {
                    maxdec = vmax(maxdec, old - g);
                    changed = true;
                }
                // Queue the larger in-cell neighbours (halo nodes belong to other cells).
                const bool want[6] = {dec && x > 0 && xm > g, dec && x < R - 1 && xp > g,
                                      dec && y > 0 && ym > g, dec && y < R - 1 && yp > g,
                                      dec && z > 0 && zm > g, dec && z < R - 1 && zp > g};
                const int off[6] = {-1, 1, -B, B, -B * B, B * B};
                const int loff[6] = {-1, 1, -R, R, -R2, R2};
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    bool app = false;
                    if (want[k]) {
                        // the word that holds the sign bit
                        unsigned int* hi = reinterpret_cast<unsigned int*>(&L.U[b + off[k]]) +
                                           (sizeof(UT) == 8 ? 1 : 0);
                        app = !(atomicOr(hi, 0x80000000u) & 0x80000000u);
                    }
                    const uint64_t m = __ballot(app);
                    if (app) L.lst[cur ^ 1][n_next + __popcll(m & below)] = (uint16_t)(l + loff[k]);
                    n_next += __popcll(m);
                }
                wave_sync();
            }
            ++nsweeps;
            const bool any_changed = __any(changed);
            visit_changed |= any_changed;
            cur ^= 1;
            n_cur = n_next;
            if (track_dec && (double)wave_max(maxdec) <= S.tol) break;
            if (n_cur > 0 && nsweeps >= P.max_sweeps) { requeue = true; break; }
        }
    }
    cnt.sweeps += (unsigned long long)nsweeps;
    cnt.updates += upd;
    const unsigned long long t2 = cycles();

    // Write back the cell and the faces that changed; tag downwind neighbours (eq. (3) value:
    // the smallest newly decreased border value below the neighbour's value across the face).
    // Lane f (f < 6) tags the neighbour across face f; lane 6 re-queues the cell itself.
    bool my_tag = false;
    int my_target = 0;
    uint32_t my_bits = 0;
    double my_value = __builtin_inf();
    // A visit publishes every border node that decreased (below its value at stage-in, which is
    // the published face copy) and tags the neighbours across those faces.  A visit cut short by the
    // sweep cap (sweeps and list relaxation) also stores its values with their active flags
    // (sign bits), so the next visit resumes with the same active set.  Only the cell's own
    // visits read the stored flags; face copies and the output are taken through |.|.
    // (Publishing the partial result lets the neighbours start a round earlier; measured, that
    // beats holding it back until the cell completes.)
    const bool keep_active = requeue && INNER != INNER_DUAL;
    publish_cell<R, FT, UT, ASYNC>(P, S, lc, cc, L.U, before, visit_changed, keep_active, lane, 0,
                                   my_tag, my_target, my_bits, my_value);
    if (requeue) {
        if (lane == 6) {
            my_tag = true;
            my_target = c;
            my_bits = requeue_bits;
            my_value = popped_key;
        }
        cnt.requeued += 1;
    }
    if constexpr (ASYNC) {
        mem_wait();  // the visit's values and faces are visible before any neighbour is tagged
        tag_lanes_async(P, lane, my_tag, my_target, my_bits, my_value);
    } else {
        tag_lanes<R, INNER, UT>(P, nxt, ctl_next, L, lane, wq, my_tag, my_target, my_bits,
                                my_value, slot);
    }
    const unsigned long long t3 = cycles();
    cnt.cyc_stage += t1 - t0;
    cnt.cyc_sweep += t2 - t1;
    cnt.cyc_write += t3 - t2;
}

// ------------------------------------------------------------------------------------------
// One visit of two cells by one wave (INNER_PAIR): both are staged side by side in the wave's
// LDS and swept at once with the two-stream plane table -- at step t the lanes of stream 0 take
// plane t of cell 0's current sweep and the lanes of stream 1 plane (t + H) mod NP of cell 1's,
// at most 49 nodes at r = 8 -- so a wave instruction updates up to twice the nodes of a
// one-cell sweep.  Each cell has its own direction sequence, sweep count, stop test and cap, as
// in visit_cell; the cells are independent (their boxes are disjoint and a wave visits them
// within one round, like two workers would), so the locking sweeps of each are exactly those of
// a one-cell visit.  Cell 1 may be absent (c1 < 0).

template <int R, typename FT, typename UT>
__device__ __forceinline__ void visit_pair(const SolveParams& P, int c0, int slot0, uint32_t fl0,
                                           double key0, int c1, int slot1, uint32_t fl1,
                                           double key1, WaveLds<R, INNER_PAIR, UT>& L,
                                           const PlaneRegs<R, INNER_PAIR>& pr, int lane,
                                           RoundCtl* ctl_next, int nxt, VisitCounters& cnt,
                                           WaveQueue& wq, uint32_t (&sweeps_out)[2]) {
    constexpr int R2 = R * R, R3 = R * R * R, B = R + 2, NP = 3 * R - 2, H = NP / 2;
    constexpr int BOX = WaveLds<R, INNER_PAIR, UT>::BOX;
    static_assert(R2 <= 64, "one face node per lane");
    const UT INF = (UT)__builtin_inf();
    const unsigned long long t0 = cycles();
    const int cc_[2] = {__builtin_amdgcn_readfirstlane(c0), __builtin_amdgcn_readfirstlane(c1)};
    const int sl_[2] = {__builtin_amdgcn_readfirstlane(slot0),
                        __builtin_amdgcn_readfirstlane(slot1)};
    const uint32_t fl_[2] = {fl0, fl1};
    const bool has1 = cc_[1] >= 0;
    Slot S_[2];
    int lc_[2];
    CellXYZ xyz_[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int ck = k == 0 || has1 ? cc_[k] : cc_[0];
        S_[k] = P.slots[k == 0 || has1 ? sl_[k] : sl_[0]];
        lc_[k] = ck - S_[k].cell_base;
        xyz_[k] = cell_coords(S_[k], lc_[k]);
    }
    stage_cell<R, FT, UT, false>(S_[0], lc_[0], xyz_[0], L.U, L.S, lane);
    if (has1) {
        stage_cell<R, FT, UT, false>(S_[1], lc_[1], xyz_[1], L.U + BOX, L.S + R3, lane);
    } else {
        for (int l = lane; l < R3; l += 64) L.S[R3 + l] = UT(0);  // no live node in the box
    }
    wave_sync();
    // Border values before the visit, then the initial active sets (as in visit_cell).
    UT before[2][6][1];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            before[k][f][0] = INF;
            if (lane < R2) {
                int x, y, z;
                face_node<R>(f, lane % R, lane / R, x, y, z);
                before[k][f][0] = fabs(L.U[k * BOX + box_index<R>(x, y, z)]);
            }
        }
    wave_sync();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && !has1) continue;
        UT* Uk = L.U + k * BOX;
        const UT* Sk = L.S + k * R3;
        if (fl_[k] & FL_ALL) {
            for (int l = lane; l < R3; l += 64) {
                const int x = l % R, y = (l / R) % R, z = l / R2;
                if (Sk[l] > UT(0)) Uk[box_index<R>(x, y, z)] = -fabs(Uk[box_index<R>(x, y, z)]);
            }
        } else {
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                if ((fl_[k] & (1u << f)) && lane < R2) {
                    int x, y, z;
                    face_node<R>(f, lane % R, lane / R, x, y, z);
                    if (Sk[x + R * (y + R * z)] > UT(0)) {
                        const int b = box_index<R>(x, y, z);
                        Uk[b] = -fabs(Uk[b]);
                    }
                }
            }
        }
    }
    wave_sync();

    const unsigned long long t1 = cycles();
    const bool track_dec = S_[0].tol > 0.0 || (has1 && S_[1].tol > 0.0);
    // Per cell: preferred directions (taken first, in Gray order), Gray-cycle position (a capped
    // visit resumes there), running flag, sweeps, decreases, cap.
    uint32_t pref[2], nsw[2] = {0, 0};
    int pi[2] = {0, 0}, ci[2], last_gi[2] = {0, 0}, dir[2] = {0, 0};
    bool run[2] = {true, has1}, inflight[2] = {false, false}, vchg[2] = {false, false};
    bool requeue[2] = {false, false};
    uint32_t requeue_bits[2] = {0u, 0u};
    uint64_t chg[2] = {0ull, 0ull};
    UT maxdec[2] = {UT(0), UT(0)};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        pref[k] = (fl_[k] >> FL_DIR_SHIFT) & 0xFFu;
        ci[k] = (fl_[k] & FL_GRAY_SET) ? (int)((fl_[k] >> FL_GRAY_SHIFT) & 7u) : 0;
    }
    auto next_dir = [&](int k) {
        while (pi[k] < 8) {
            const int gi = pi[k]++;
            if (pref[k] & (1u << kGray[gi])) {
                last_gi[k] = gi;
                return kGray[gi];
            }
        }
        last_gi[k] = ci[k] & 7;
        ++ci[k];
        return kGray[last_gi[k]];
    };
    // End of a sweep of cell k: stop when it changed nothing, when no node is left active, when
    // its largest decrease is within tol, or at the sweep cap (re-queued, resuming the cycle).
    auto end_sweep = [&](int k) {
        inflight[k] = false;
        ++nsw[k];
        if (chg[k] == 0ull) {
            run[k] = false;
            return;
        }
        vchg[k] = true;
        const UT* Uk = L.U + k * BOX;
        bool left = false;
        for (int l = lane; l < R3; l += 64) {
            const int x = l % R, y = (l / R) % R, z = l / R2;
            left |= is_active(Uk[box_index<R>(x, y, z)]);
        }
        if (!__any(left)) {
            run[k] = false;
            return;
        }
        if (track_dec && (double)wave_max(maxdec[k]) <= S_[k].tol) {
            run[k] = false;
            return;
        }
        if ((int)nsw[k] >= P.max_sweeps) {
            run[k] = false;
            requeue[k] = true;
            requeue_bits[k] = FL_GRAY_SET | ((uint32_t)((last_gi[k] + 1) & 7) << FL_GRAY_SHIFT);
        }
    };
    unsigned int upd = 0;
    while (run[0] || run[1]) {
#pragma unroll
        for (int t = 0; t < NP; ++t) {
            if (t == 0 && run[0]) {
                dir[0] = next_dir(0);
                inflight[0] = true;
                chg[0] = 0ull;
                maxdec[0] = UT(0);
            }
            if (t == H && run[1]) {
                dir[1] = next_dir(1);
                inflight[1] = true;
                chg[1] = 0ull;
                maxdec[1] = UT(0);
            }
            const uint32_t mref0 = reflect_mask<R>(dir[0]), mref1 = reflect_mask<R>(dir[1]);
            uint32_t e = (pr.pk[t >> 1] >> ((t & 1) * 16)) & 0xFFFFu;
            asm volatile("" : "+v"(e));
            const bool st1 = (e & 0x8000u) != 0u;
            const uint32_t lr = (e & 0x7FFFu) ^ (st1 ? mref1 : mref0);
            const int b = box_of_cell_index<R>(lr) + (st1 ? BOX : 0);
            const int l = (int)lr + (st1 ? R3 : 0);
            UT raw = L.U[b];
            UT sv = L.S[l];
            UT xm = L.U[b - 1], xp = L.U[b + 1];
            UT ym = L.U[b - B], yp = L.U[b + B];
            UT zm = L.U[b - B * B], zp = L.U[b + B * B];
            asm volatile("" : "+v"(raw), "+v"(sv), "+v"(xm), "+v"(xp), "+v"(ym), "+v"(yp),
                         "+v"(zm), "+v"(zp));
            const bool on = st1 ? inflight[1] : inflight[0];
            const bool act = pr.has(t) && on && is_active(raw);
            if (__any(act)) {
                const UT old = fabs(raw);
                const UT g = local_solve(vmin_abs(xm, xp), vmin_abs(ym, yp), vmin_abs(zm, zp), sv);
                const bool live = act && sv > UT(0);
                const bool dec = live && g < old;
                upd += (unsigned)__popcll(__ballot(live));  // wave total, scalar unit
                UT* const ub = &L.U[b];
                if (act) ub[0] = dec ? g : old;
                const uint64_t decm = __ballot(dec), st1m = __ballot(st1);
                chg[0] |= decm & ~st1m;
                chg[1] |= decm & st1m;
                if (track_dec && dec) {
                    if (st1) maxdec[1] = vmax(maxdec[1], old - g);
                    else maxdec[0] = vmax(maxdec[0], old - g);
                }
                if (dec && xm > g) mark_active(ub - 1, xm);
                if (dec && xp > g) mark_active(ub + 1, xp);
                if (dec && ym > g) mark_active(ub - B, ym);
                if (dec && yp > g) mark_active(ub + B, yp);
                if (dec && zm > g) mark_active(ub - B * B, zm);
                if (dec && zp > g) mark_active(ub + B * B, zp);
            }
            wave_sync();
            if (t == NP - 1 && inflight[0]) end_sweep(0);
            if (t == H - 1 && inflight[1]) end_sweep(1);
            if (!run[0] && !run[1] && !inflight[0] && !inflight[1]) break;
        }
    }
    cnt.sweeps += (unsigned long long)(nsw[0] + nsw[1]);
    cnt.updates += upd;
    sweeps_out[0] = nsw[0];
    sweeps_out[1] = nsw[1];
    const unsigned long long t2 = cycles();

    // Write-back of each cell; lanes 0-5 tag across the faces of cell 0, lanes 8-13 across those
    // of cell 1; lanes 6 and 14 re-queue a capped cell.
    bool my_tag = false;
    int my_target = 0;
    uint32_t my_bits = 0;
    double my_value = __builtin_inf();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && !has1) continue;
        publish_cell<R, FT, UT, false>(P, S_[k], lc_[k], xyz_[k], L.U + k * BOX, before[k],
                                       vchg[k], requeue[k], lane, 8 * k, my_tag, my_target,
                                       my_bits, my_value);
        if (requeue[k]) {
            if (lane == 8 * k + 6) {
                my_tag = true;
                my_target = cc_[k];
                my_bits = requeue_bits[k];
                my_value = k == 0 ? key0 : key1;
            }
            cnt.requeued += 1;
        }
    }
    tag_lanes<R, INNER_PAIR, UT>(P, nxt, ctl_next, L, lane, wq, my_tag, my_target, my_bits,
                                 my_value, has1 && sl_[0] != sl_[1] ? -1 : sl_[0]);
    const unsigned long long t3 = cycles();
    cnt.cyc_stage += t1 - t0;
    cnt.cyc_sweep += t2 - t1;
    cnt.cyc_write += t3 - t2;
}

// ------------------------------------------------------------------------------------------
// Grid barrier for the persistent cooperative launch.  All workgroups are co-resident (the
// launch is cooperative), so every arrival is eventually followed by the last one.  A spin
// that outlives the watchdog (a bounded number of polls) sets the status to EIK_ECANCELLED and
// returns, so a broken invariant ends the kernel instead of hanging it.

__device__ bool grid_barrier(const SolveParams& P) {
    __syncthreads();
    __shared__ int s_abort;
    if (threadIdx.x == 0) {
        s_abort = 0;
        uint32_t* count = &P.bar[0];
        uint32_t* gen = &P.bar[kBarGen];
        const uint32_t g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t arrived = atomicAdd(count, 1u);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(gen, 1u);
        } else {
            uint64_t polls = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(8);
                if (++polls > P.watchdog_polls) {
                    atomicCAS(P.status, 0, EIK_ECANCELLED_DEV);
                    s_abort = 1;
                    break;
                }
            }
        }
        __threadfence();
    }
    __syncthreads();
    return s_abort == 0;
}

// ------------------------------------------------------------------------------------------
// The solver.  Each wave is an independent worker; each workgroup holds `W` workers.  One
// launch runs every round (persistent, grid barrier between rounds).

template <int R, typename FT, int W, int INNER, typename UT>
__global__ void __launch_bounds__(64 * W)
    __attribute__((amdgpu_waves_per_eu(R == 16 ? 1
                                       : INNER == INNER_PAIR ? 2 : (sizeof(UT) == 4 ? 4 : 3))))
k_solve(SolveParams P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WaveLds<R, INNER, UT>& L = reinterpret_cast<WaveLds<R, INNER, UT>*>(lds_raw)[wave];
    VisitCounters cnt{0, 0, 0, 0, 0, 0};
    unsigned long long cyc_pop = 0, cyc_wait = 0;
    PlaneRegs<R, INNER> pr;
    load_plane_regs<R, INNER>(pr, lane);
    unsigned long long visits = 0, deferred = 0;
    int rounds_done = 0;
    // Per-workgroup histograms of visits (sweeps; log2 of cycles) and counters, flushed at the
    // end.
    __shared__ unsigned int s_hist[64];
    __shared__ unsigned long long s_cnt[ST_COUNT];
    if (threadIdx.x < 64) s_hist[threadIdx.x] = 0u;
    if (threadIdx.x < ST_COUNT) s_cnt[threadIdx.x] = 0ull;
    __syncthreads();

    const int nwaves_total = (int)gridDim.x * W;
    for (int64_t t = P.round_begin;; ++t) {
        const int cur = (int)(t & 1), nxt = cur ^ 1;
        RoundCtl* ctl_cur = &P.ctl[t & 3];
        RoundCtl* ctl_next = &P.ctl[(t + 1) & 3];
        if (P.single_round) {
            // One round per launch (the host-driven loop): the launch runs round t unless an
            // earlier launch stopped the loop, the list is empty, the launch status is set or
            // the round cap is reached.  Every wave reads the same words, which no launch of
            // this round changes except to stop, so all agree.
            const uint32_t n0 = __hip_atomic_load(&ctl_cur->count, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t was_halted = __hip_atomic_load(P.halted, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
            if (blockIdx.x == 0 && threadIdx.x == 0 && !was_halted && cancel_requested(P))
                atomicCAS(P.status, 0, EIK_ECANCELLED_DEV);  // seen by this or the next launch
            const int st0 = __hip_atomic_load(P.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool stop = was_halted || n0 == 0 || st0 != 0 || t >= P.max_rounds;
            if (blockIdx.x == 0 && threadIdx.x == 0 && !was_halted) {
                *P.next_round = stop ? t : t + 1;
                if (n0 != 0 && st0 == 0 && t >= P.max_rounds) atomicCAS(P.status, 0, EIK_ENOCONV_DEV);
                if (stop) __hip_atomic_store(P.halted, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (stop) break;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            RoundCtl* r2 = &P.ctl[(t + 2) & 3];
            r2->count = 0;
            r2->minkey = dbits(__builtin_inf());
        }
        if (blockIdx.x == 0 && threadIdx.x < kPopSegs)
            P.seg_cursor[(((t + 2) & 3) * kPopSegs + threadIdx.x) * 32] = 0;
        // Per-slot bands: the row of round t + 2 is neither read nor written in round t.
        const bool slot_band = P.slot_band && P.delta > 0.0;
        if (slot_band) {
            uint64_t* r2 = slot_minkeys(P, t + 2);
            for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P.nslots;
                 i += gridDim.x * blockDim.x)
                r2[i] = dbits(__builtin_inf());
        }
        const uint32_t n = __hip_atomic_load(&ctl_cur->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double thr = P.delta > 0.0 ? bitsd(ld_relaxed_u64(&ctl_cur->minkey)) + P.delta
                                         : __builtin_inf();
        const uint64_t* smk_cur = slot_band ? slot_minkeys(P, t) : nullptr;
        // Pops.  The list is split into kPopSegs segments with a cursor each; a workgroup pops
        // from its own segment (workgroup index modulo kPopSegs: two segments per XCD, to which
        // workgroups are dealt in turn), and once that is exhausted from any other that is not
        // (found with one load per segment).  One cell per pop (two for a wave sweeping two cells
        // at once): with the pops spread over the segments' cursors, taking more cells at a time
        // saves little and leaves some waves with a second cell while others have none.
        constexpr uint32_t chunk_now = INNER == INNER_PAIR ? 2u : 1u;
        uint32_t* const segc = P.seg_cursor + (size_t)(t & 3) * kPopSegs * 32;
        const uint32_t seg_len = (n + kPopSegs - 1) / kPopSegs;
        int seg = (int)(blockIdx.x % kPopSegs);
        uint32_t seg_lo = 0, seg_hi = 0;
        auto seg_bounds = [&](int g) {
            seg_lo = min((uint32_t)g * seg_len, n);
            seg_hi = min(seg_lo + seg_len, n);
        };
        seg_bounds(seg);
        WaveQueue wq{0, __builtin_inf()};
        for (;;) {
            const unsigned long long tp0 = cycles();
            uint32_t base = 0;
            if (lane == 0) base = seg_lo + atomicAdd(&segc[seg * 32], chunk_now);
            base = __shfl(base, 0, 64);
            if (base >= seg_hi) {
                // Lane g reads segment g's cursor; the wave moves to the first open segment
                // after the current one (so that the waves that steal spread out), or stops.
                bool open = false;
                if (lane < kPopSegs) {
                    const uint32_t lo = min((uint32_t)lane * seg_len, n);
                    const uint32_t hi = min(lo + seg_len, n);
                    open = lo + __hip_atomic_load(&segc[lane * 32], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT) < hi;
                }
                const uint64_t om = __builtin_amdgcn_ballot_w64(open);
                if (om == 0u) { cyc_pop += cycles() - tp0; break; }
                const uint64_t rot = (om >> (seg + 1)) | (om << (kPopSegs - 1 - seg));
                seg = (seg + 1 + __builtin_ctzll(rot & ((1ull << kPopSegs) - 1ull))) % kPopSegs;
                seg_bounds(seg);
                cyc_pop += cycles() - tp0;
                continue;
            }
            const uint32_t cnt_here = seg_hi - base < chunk_now ? seg_hi - base : chunk_now;
            // Lanes j < cnt_here take cell j of the chunk: its flags and value are exchanged
            // for empty ones (the removal of Algorithm 3 with V^c <- +inf).
            int my_c = 0, my_slot = 0;
            uint32_t my_fl = 0;
            unsigned long long my_kb = 0;
            if ((uint32_t)lane < cnt_here) {
                uint32_t idx = base + lane;
                if (P.shuffle) {
                    const uint64_t mix = P.shuffle * 0x9E3779B97F4A7C15ull + (uint64_t)t * 0xBF58476D1CE4E5B9ull;
                    idx = (uint32_t)(((uint64_t)idx * 2654435761ull + (mix >> 17)) % n);
                }
                my_c = P.list[cur][idx];
                my_slot = P.cell_slot[my_c];  // issued beside the exchanges, read by the visit
                my_fl = atomicExch(&P.flags[cur][my_c], 0u);
                my_kb = P.delta > 0.0
                            ? atomicExch((unsigned long long*)&P.key[cur][my_c],
                                         (unsigned long long)dbits(__builtin_inf()))
                            : 0ull;
            }
            // Cells outside the lowest band (of the whole launch, or of their own slot) go
            // straight back to the next round's list.
            double my_thr = thr;
            if (slot_band && (uint32_t)lane < cnt_here)
                my_thr = bitsd(ld_relaxed_u64(&smk_cur[my_slot])) + P.delta;
            const bool defer = (uint32_t)lane < cnt_here && !(bitsd(my_kb) < my_thr);
            const uint64_t defer_mask = __ballot(defer);
            deferred += __popcll(defer_mask);
            tag_lanes<R, INNER, UT>(P, nxt, ctl_next, L, lane, wq, defer, my_c, my_fl & ~FL_QUEUED,
                         bitsd(my_kb), -1);
            cyc_pop += cycles() - tp0;
            if constexpr (INNER == INNER_PAIR) {
                // The cells of the chunk that were not deferred, two per visit.
                uint64_t todo = ~defer_mask & ((1ull << cnt_here) - 1ull);
                while (todo) {
                    const int ja = __builtin_ctzll(todo);
                    todo &= todo - 1ull;
                    const int jb = todo ? __builtin_ctzll(todo) : -1;
                    if (jb >= 0) todo &= todo - 1ull;
                    const int jj = jb >= 0 ? jb : ja;
                    const int ca = __shfl(my_c, ja, 64), cb = __shfl(my_c, jj, 64);
                    const int sa = __shfl(my_slot, ja, 64), sb = __shfl(my_slot, jj, 64);
                    const uint32_t fa = __shfl(my_fl, ja, 64), fb = __shfl(my_fl, jj, 64);
                    const double ka = bitsd(__shfl(my_kb, ja, 64));
                    const double kb2 = bitsd(__shfl(my_kb, jj, 64));
                    jitter_delay(P, ((uint64_t)t << 40) ^ ((uint64_t)blockIdx.x << 20) ^
                                        ((uint64_t)wave << 12) ^ visits);
                    const unsigned long long tv0 = cycles();
                    uint32_t nsw[2] = {0u, 0u};
                    visit_pair<R, FT, UT>(P, ca, sa, fa, ka, jb >= 0 ? cb : -1, sb, fb, kb2, L,
                                          pr, lane, ctl_next, nxt, cnt, wq, nsw);
                    visits += jb >= 0 ? 2 : 1;
                    if (lane == 0) {
                        const unsigned long long dt = cycles() - tv0;
                        const int lg = dt ? 63 - __builtin_clzll(dt) : 0;
                        for (int k = 0; k < (jb >= 0 ? 2 : 1); ++k) {
                            atomicAdd(&s_hist[nsw[k] < 31 ? nsw[k] : 31], 1u);
                            atomicAdd(&s_hist[32 + (lg < 31 ? lg : 31)], 1u);
                        }
                    }
                }
            } else
            for (uint32_t j = 0; j < cnt_here; ++j) {
                const int c = __shfl(my_c, (int)j, 64);
                const int cs = __shfl(my_slot, (int)j, 64);
                const uint32_t fl = __shfl(my_fl, (int)j, 64);
                const double key = bitsd(__shfl(my_kb, (int)j, 64));
                if ((defer_mask >> j) & 1ull) continue;
                jitter_delay(P, ((uint64_t)t << 40) ^ ((uint64_t)blockIdx.x << 20) ^
                                    ((uint64_t)wave << 12) ^ visits);
                ++visits;
                const unsigned long long sw0 = cnt.sweeps, tv0 = cycles();
                visit_cell<R, FT, INNER, UT>(P, c, cs, fl, key, L, pr, lane, ctl_next, nxt, cnt,
                                             wq);
                if (lane == 0) {
                    const unsigned long long dsw = cnt.sweeps - sw0, dt = cycles() - tv0;
                    atomicAdd(&s_hist[dsw < 31 ? dsw : 31], 1u);
                    const int lg = dt ? 63 - __builtin_clzll(dt) : 0;
                    atomicAdd(&s_hist[32 + (lg < 31 ? lg : 31)], 1u);
                }
            }
        }
        const unsigned long long tw0 = cycles();
        queue_flush_group<R, INNER, UT, W>(P, nxt, ctl_next, L, lane, wave, wq);
        if (P.delta > 0.0 && !slot_band) {
            const double mk = wave_min(wq.minkey);
            if (lane == 0 && mk < __builtin_inf())
                atomicMin((unsigned long long*)&ctl_next->minkey, (unsigned long long)dbits(mk));
        }
        ++rounds_done;
        if (P.single_round) {
            // The launch ends here; the next launch on the stream runs round t + 1.
            if (blockIdx.x == 0 && threadIdx.x == 0 && t < P.round_log_len) {
                P.round_log[2 * t] = (int64_t)n;
                P.round_log[2 * t + 1] = (int64_t)cycles();
            }
            break;
        }
        // The host's cancel request is read by one thread before the barrier, so every
        // workgroup sees the resulting status after it and all leave in the same round.
        if (blockIdx.x == 0 && threadIdx.x == 0 && cancel_requested(P))
            atomicCAS(P.status, 0, EIK_ECANCELLED_DEV);
        const bool ok = grid_barrier(P);
        cyc_wait += cycles() - tw0;
        if (blockIdx.x == 0 && threadIdx.x == 0 && t < P.round_log_len) {
            P.round_log[2 * t] = (int64_t)n;
            P.round_log[2 * t + 1] = (int64_t)cycles();
        }
        if (!ok) break;
        const uint32_t nnext = __hip_atomic_load(&ctl_next->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int st = __hip_atomic_load(P.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // Every workgroup reads the same words after the barrier, so all leave together.
        if (nnext == 0 || st != 0 || t + 1 >= P.round_end || t + 1 >= P.max_rounds) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                *P.next_round = t + 1;
                if (nnext != 0 && st == 0 && t + 1 >= P.max_rounds)
                    atomicCAS(P.status, 0, EIK_ENOCONV_DEV);
            }
            break;
        }
    }
    // Counters: summed over the workgroup's waves in LDS, then one device atomic per counter and
    // workgroup (a launch per round in the host-driven loop makes this flush per round).
    if (lane == 0) {
        atomicAdd(&s_cnt[ST_VISITS], visits);
        atomicAdd(&s_cnt[ST_SWEEPS], cnt.sweeps);
        atomicAdd(&s_cnt[ST_UPDATES], cnt.updates);
        atomicAdd(&s_cnt[ST_DEFERRED], deferred);
        atomicAdd(&s_cnt[ST_REQUEUED], cnt.requeued);
        atomicAdd(&s_cnt[ST_CYC_POP], cyc_pop);
        atomicAdd(&s_cnt[ST_CYC_STAGE], cnt.cyc_stage);
        atomicAdd(&s_cnt[ST_CYC_SWEEP], cnt.cyc_sweep);
        atomicAdd(&s_cnt[ST_CYC_WRITE], cnt.cyc_write);
        atomicAdd(&s_cnt[ST_CYC_WAIT], cyc_wait);
        if (P.count_workers) atomicAdd(&s_cnt[ST_WORKERS], 1ull);
        if (blockIdx.x == 0 && wave == 0) atomicAdd(&s_cnt[ST_ROUNDS], (unsigned long long)rounds_done);
    }
    // Every workgroup leaves the round loop in the same round, so all its waves get here.
    __syncthreads();
    if (threadIdx.x < ST_COUNT && s_cnt[threadIdx.x])
        atomicAdd(&P.stats[threadIdx.x], s_cnt[threadIdx.x]);
    if (threadIdx.x < 64 && s_hist[threadIdx.x])
        atomicAdd(&P.stats[ST_HIST_SWEEPS + threadIdx.x], (unsigned long long)s_hist[threadIdx.x]);
}

// ------------------------------------------------------------------------------------------
// The solver without rounds: each wave pops one cell at a time from a ring of queued cells,
// visits it, pushes the neighbours it tags, and pops again; there is no barrier between
// visits.  When no cell is queued or being visited, every wave leaves the pop loop and, after a
// grid barrier, the waves check every cell against eq. (2): a node whose local solve is below
// its value (by more than rounding) re-queues its cell with every node active, and the pop loop
// runs again.  The check makes the result independent of the order in which one visit's writes
// become visible to another: every value ever stored is an upper bound of the solution (the
// local solve is monotone and the exits hold q), so a stale read can only leave values too high,
// which the check finds; it ends when eq. (2) holds at every node, whose solution is unique.

// Whether some node of cell lc (stage already in L) has a local solve below its value.
template <int R, int INNER, typename UT>
__device__ __forceinline__ bool cell_above_fixed_point(WaveLds<R, INNER, UT>& L, int lane) {
    constexpr int R2 = R * R, R3 = R * R * R, B = R + 2;
    bool bad = false;
    for (int l = lane; l < R3; l += 64) {
        const UT s = L.S[l];
        if (!(s > UT(0))) continue;  // exit or padding
        const int x = l % R, y = (l / R) % R, z = l / R2;
        const int b = box_index<R>(x, y, z);
        const UT u = fabs(L.U[b]);
        const UT g = local_solve(vmin_abs(L.U[b - 1], L.U[b + 1]), vmin_abs(L.U[b - B], L.U[b + B]),
                                 vmin_abs(L.U[b - B * B], L.U[b + B * B]), s);
        bad |= g < u && (u == (UT)__builtin_inf() || u - g > u * (UT)0x1p-44);
    }
    return __any(bad);
}

template <int R, typename FT, int W, int INNER, typename UT>
__global__ void __launch_bounds__(64 * W)
    __attribute__((amdgpu_waves_per_eu(R == 16 ? 1 : (sizeof(UT) == 4 ? 4 : 3))))
k_solve_async(SolveParams P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WaveLds<R, INNER, UT>& L = reinterpret_cast<WaveLds<R, INNER, UT>*>(lds_raw)[wave];
    VisitCounters cnt{0, 0, 0, 0, 0, 0};
    unsigned long long cyc_pop = 0, cyc_wait = 0, visits = 0;
    PlaneRegs<R, INNER> pr;
    load_plane_regs<R, INNER>(pr, lane);
    __shared__ unsigned int s_hist[64];
    if (threadIdx.x < 64) s_hist[threadIdx.x] = 0u;
    const int nwaves_total = (int)gridDim.x * W;
    const int gwave = (int)blockIdx.x * W + wave;
    const bool band = P.delta > 0.0;
    // The exits' cells were queued for the first round by the seed: the first n0 entries of
    // list[0] (with QUEUED set in flags[0] and their cell values in key[0]).
    const uint32_t n0 = P.ctl[P.round_begin & 3].count;
    const size_t gtid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t gthreads = (size_t)gridDim.x * blockDim.x;
    if (!band) {
        // The FIFO ring is list[0..1] itself: the seeded cells are its first n0 entries.
        const uint64_t cap = (uint64_t)(2 * P.ncells + kRingExtra);
        for (uint64_t i = n0 + gtid; i < cap; i += gthreads) P.list[0][i] = -1;
        if (gtid == 0) {
            *P.async_head = 0;
            *P.async_tail = n0;
        }
    } else {
        const uint64_t total = (uint64_t)kBuckets * (uint64_t)P.bq_cap;
        unsigned long long* words = reinterpret_cast<unsigned long long*>(P.bq_ring);
        for (uint64_t i = gtid; i < total; i += gthreads) words[i] = 0ull;  // lap 0: free
        for (size_t i = gtid; i < (size_t)kBuckets; i += gthreads) {
            *bq_head(P, (int)i) = 0;
            *bq_tail(P, (int)i) = 0;
        }
        if (gtid == 0) *bq_low(P) = 0;
    }
    if (gtid == 0) {
        *P.async_pending = n0;
        *P.async_done = n0 == 0 ? 1u : 0u;
    }
    int passes = 0;
    bool ok = grid_barrier(P);
    if (ok && band) {
        // Seeded cells into the buckets of their values.
        for (size_t i = gtid; i < n0; i += gthreads) {
            const int c = P.list[0][i];
            const int b = (int)(bucket_of(P, bitsd(P.key[0][c]), 0) % (uint64_t)kBuckets);
            const uint64_t pos = atomicAdd(bq_tail(P, b), 1ull);
            *bq_slot(P, b, pos) = (unsigned long long)(((pos / (uint64_t)P.bq_cap + 1) << 32) |
                                                       (uint32_t)c);
        }
        ok = grid_barrier(P);
    }
    while (ok) {
        // Pop loop.
        for (;;) {
            const unsigned long long tp0 = cycles();
            const int c = pop_cell(P, lane);
            if (c < 0) {
                cyc_wait += cycles() - tp0;
                break;
            }
            uint32_t fl = 0;
            int slot = 0, st = 0;
            unsigned long long kb = 0;
            if (lane == 0) {
                fl = atomicExch(&P.flags[0][c], FL_RUNNING);
                if (band)  // the removal of the cell from the heap resets its value to +inf
                    kb = atomicExch((unsigned long long*)&P.key[0][c],
                                    (unsigned long long)dbits(__builtin_inf()));
                slot = P.cell_slot[c];
                // The host's cancel request (every 16 visits: a read of host memory), then the
                // launch status, in the same memory round trip as the exchange.
                if ((visits & 15) == 0 && cancel_requested(P)) async_cancel(P);
                st = __hip_atomic_load(P.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            fl = __shfl(fl, 0, 64) & ~FL_QUEUED;
            slot = __shfl(slot, 0, 64);
            kb = __shfl(kb, 0, 64);
            mem_wait();  // the exchange has returned before the visit reads the cell
            cyc_pop += cycles() - tp0;
            // A cancelled launch (by the host or a watchdog) stops popping although cells are
            // still queued; the cell just taken stays RUNNING, which the next solve's
            // initialisation clears.
            if (__shfl(st, 0, 64) != 0) break;
            jitter_delay(P, ((uint64_t)blockIdx.x << 20) ^ ((uint64_t)wave << 12) ^ visits);
            ++visits;
            const unsigned long long sw0 = cnt.sweeps, tv0 = cycles();
            WaveQueue wq{0, __builtin_inf()};
            visit_cell<R, FT, INNER, UT, true>(P, c, slot, fl, bitsd(kb), L, pr, lane, nullptr, 0,
                                               cnt, wq);
            // Release the cell; a tag that arrived during the visit left QUEUED set (and, with a
            // band, lowered its value).
            bool again = false;
            double again_key = 0.0;
            if (lane == 0) {
                again = (atomicAnd(&P.flags[0][c], ~FL_RUNNING) & FL_QUEUED) != 0;
                if (again && band) again_key = bitsd(ld_relaxed_u64(&P.key[0][c]));
            }
            again = __shfl((int)again, 0, 64) != 0;
            queue_push(P, lane, lane == 0 && again, c, again_key);
            if (lane == 0) {
                if (atomicAdd(P.async_pending, ~0ull) == 1ull)
                    __hip_atomic_store(P.async_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long dsw = cnt.sweeps - sw0, dt = cycles() - tv0;
                atomicAdd(&s_hist[dsw < 31 ? dsw : 31], 1u);
                const int lg = dt ? 63 - __builtin_clzll(dt) : 0;
                atomicAdd(&s_hist[32 + (lg < 31 ? lg : 31)], 1u);
            }
        }
        // No cell queued or being visited.  Abandon the tickets taken past the last push (so
        // that later pushes are popped), then check every cell.
        const unsigned long long tw0 = cycles();
        if (!(ok = grid_barrier(P))) break;
        if (__hip_atomic_load(P.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (!band) *P.async_head = *P.async_tail;
            *P.async_done = 0u;
        }
        if (!(ok = grid_barrier(P))) break;
        ++passes;
        for (int64_t c = gwave; c < P.ncells; c += nwaves_total) {
            const int cs = __builtin_amdgcn_readfirstlane(P.cell_slot[c]);
            const Slot S = P.slots[cs];
            const int lc = (int)c - S.cell_base;
            stage_cell<R, FT, UT, true>(S, lc, cell_coords(S, lc), L.U, L.S, lane);
            const bool redo = cell_above_fixed_point<R, INNER, UT>(L, lane);
            wave_sync();
            tag_lanes_async(P, lane, redo && lane == 0, (int)c, FL_ALL, 0.0);
        }
        if (!(ok = grid_barrier(P))) break;
        cyc_wait += cycles() - tw0;
        const unsigned long long left =
            __hip_atomic_load(P.async_pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (left == 0) break;
        if (passes >= 64) {  // a bound on check passes that a correct solve never nears
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(P.status, 0, EIK_ENOCONV_DEV);
            break;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *P.next_round = P.round_begin + 1;
    if (lane == 0) {
        atomicAdd(&P.stats[ST_VISITS], visits);
        atomicAdd(&P.stats[ST_SWEEPS], cnt.sweeps);
        atomicAdd(&P.stats[ST_UPDATES], cnt.updates);
        atomicAdd(&P.stats[ST_REQUEUED], cnt.requeued);
        atomicAdd(&P.stats[ST_CYC_POP], cyc_pop);
        atomicAdd(&P.stats[ST_CYC_STAGE], cnt.cyc_stage);
        atomicAdd(&P.stats[ST_CYC_SWEEP], cnt.cyc_sweep);
        atomicAdd(&P.stats[ST_CYC_WRITE], cnt.cyc_write);
        atomicAdd(&P.stats[ST_CYC_WAIT], cyc_wait);
        atomicAdd(&P.stats[ST_WORKERS], 1ull);
        if (blockIdx.x == 0 && wave == 0) atomicAdd(&P.stats[ST_ROUNDS], (unsigned long long)passes);
    }
    __syncthreads();
    if (threadIdx.x < 64 && s_hist[threadIdx.x])
        atomicAdd(&P.stats[ST_HIST_SWEEPS + threadIdx.x], (unsigned long long)s_hist[threadIdx.x]);
}

// ------------------------------------------------------------------------------------------
// Stage inputs (a1): row-major F -> cell-blocked F of one slot with padding marked 0, u <- +inf
// (NaN on padding), or, to polish a given approximation, u <- |u_approx| * lift.  Speeds that
// are not finite and positive, or whose s = h / F lies outside the range the local solve is
// exact in, set the slot's status to EIK_EINVAL.

// Range of s = h / F accepted per value type: the local solve squares s and differences of
// values of the size of s, so s^2 must stay a normal number with room to spare (FP64:
// 2^-500 .. 2^500; FP32: 2^-60 .. 2^60).
template <typename UT>
__device__ __forceinline__ bool s_in_range(double s) {
    constexpr double lo = sizeof(UT) == 4 ? 0x1p-60 : 0x1p-500;
    constexpr double hi = sizeof(UT) == 4 ? 0x1p60 : 0x1p500;
    return s >= lo && s <= hi;
}

template <int R, typename FT, typename UT>
__global__ void k_init_nodes(Slot S, const FT* __restrict__ F, const double* __restrict__ u_approx,
                             double lift, const int* only_if) {
    if (only_if && *only_if == 0) return;
    constexpr int R3 = R * R * R;
    const size_t total = (size_t)S.ncell * R3;
    const UT INF = (UT)__builtin_inf();
    FT* fb = reinterpret_cast<FT*>(S.f);
    UT* ub = reinterpret_cast<UT*>(S.u);
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const int lc = (int)(g / R3), l = (int)(g % R3);
        const int x = l % R, y = (l / R) % R, z = l / (R * R);
        const CellXYZ cc = cell_coords(S, lc);
        const int i = cc.x * R + x, j = cc.y * R + y, k = cc.z * R + z;
        FT fv = FT(0);
        if (i < S.nx && j < S.ny && k < S.nz) {
            fv = F[(size_t)i + (size_t)S.nx * ((size_t)j + (size_t)S.ny * k)];
            const double dv = (double)fv;
            if (!(dv > 0.0) || !(dv <= 1.7976931348623157e308) || !s_in_range<UT>(S.h / dv)) {
                atomicCAS(S.status, 0, EIK_EINVAL_DEV);
                fv = FT(1);
            }
        }
        fb[g] = fv;
        // Padding nodes hold NaN: the minimum ignores them (like +inf beyond the grid) and
        // every comparison with them is false, so they are never activated or used as inflow.
        UT v = INF;
        if (u_approx && fv != FT(0)) {
            const double a = fabs(u_approx[(size_t)i + (size_t)S.nx * ((size_t)j + (size_t)S.ny * k)]);
            if (a <= 1.7976931348623157e308) v = (UT)(a * lift);  // +inf and NaN stay +inf
        }
        ub[g] = fv == FT(0) ? (UT)__builtin_nan("") : v;
    }
}

// Face copies <- the border layers of the (initialised) values, +inf for padding nodes.
template <int R, typename UT>
__global__ void k_faces_from_u(Slot S, const int* only_if) {
    if (only_if && *only_if == 0) return;
    constexpr int R2 = R * R, R3 = R * R * R;
    const size_t nf = (size_t)S.ncell * 6 * R2;
    const UT* ub = reinterpret_cast<const UT*>(S.u);
    UT* fb = reinterpret_cast<UT*>(S.faces);
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < nf;
         g += (size_t)gridDim.x * blockDim.x) {
        const size_t lc = g / (6 * R2);
        const int f = (int)((g / R2) % 6), e = (int)(g % R2);
        int x, y, z;
        face_node<R>(f, e % R, e / R, x, y, z);
        const UT v = ub[lc * R3 + x + R * (y + R * z)];
        fb[g] = v == v ? v : (UT)__builtin_inf();
    }
}

// The slot's face copies <- +inf, its cells' state cleared and mapped to the slot.
template <int R, typename UT>
__global__ void k_init_cells(SolveParams P, Slot S, int slot, const int* only_if) {
    if (only_if && *only_if == 0) return;
    constexpr int R2 = R * R;
    const size_t nf = (size_t)S.ncell * 6 * R2;
    const double INF = __builtin_inf();
    UT* faces = reinterpret_cast<UT*>(S.faces);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t g0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    for (size_t g = g0; g < nf; g += stride) faces[g] = (UT)INF;
    for (size_t g = g0; g < (size_t)S.ncell; g += stride) {
        const size_t c = (size_t)S.cell_base + g;
        P.key[0][c] = dbits(INF);
        P.key[1][c] = dbits(INF);
        P.flags[0][c] = 0;
        P.flags[1][c] = 0;
        P.key_keep[c] = dbits(INF);
        const_cast<int*>(P.cell_slot)[c] = slot;
    }
    if (g0 == 0) *S.status = 0;
}

// Round control, barrier, launch status and counters (once per solve or server).
__global__ void k_init_global(SolveParams P) {
    const int g0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    const double INF = __builtin_inf();
    if (g0 < 4) {
        P.ctl[g0].count = 0;
        P.ctl[g0].minkey = dbits(INF);
    }
    if (g0 < 4 * kPopSegs) P.seg_cursor[g0 * 32] = 0;
    if (g0 < 2) P.bar[g0 * kBarGen] = 0;
    if (g0 == 0) {
        *P.status = 0;
        *P.next_round = 0;
    }
    for (int g = g0; g < ST_TOTAL; g += stride) P.stats[g] = 0;
    for (int g = g0; g < 4 * P.nslots; g += stride) P.slot_minkey[g] = dbits(INF);
}

// Seed (a2): exit nodes fixed at q (min over duplicates), marked as exits in the blocked speed
// array, copied into their cell's face layers; their cells and the cells of their six grid
// neighbours are queued for round `round` with every node active and cell value q (the initial
// cell values of Section 4).
// Atomic minimum of a value >= +0 (or +inf) through its bit pattern, which orders like the value.
__device__ __forceinline__ void atomic_min_val(double* p, double v) {
    atomicMin((unsigned long long*)p, (unsigned long long)dbits(v));
}
__device__ __forceinline__ void atomic_min_val(float* p, float v) {
    atomicMin((unsigned int*)p, __float_as_uint(v));
}

// Before seeding a grid that starts from an approximation: the exit nodes (and their face
// copies) <- +inf, so that the seed's minimum over duplicate exits sets them to q exactly even
// where the start held a smaller value.
template <int R, typename UT>
__global__ void k_seed_clear(Slot S, int64_t nsrc, const int64_t* __restrict__ idx3) {
    constexpr int R2 = R * R, R3 = R * R * R;
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nsrc) return;
    const int64_t i = idx3[3 * n], j = idx3[3 * n + 1], k = idx3[3 * n + 2];
    if (i < 0 || i >= S.nx || j < 0 || j >= S.ny || k < 0 || k >= S.nz) return;  // k_seed reports it
    const int x = (int)(i % R), y = (int)(j % R), z = (int)(k % R);
    const int lc = (int)(i / R) + S.ncx * ((int)(j / R) + S.ncy * (int)(k / R));
    const UT INF = (UT)__builtin_inf();
    reinterpret_cast<UT*>(S.u)[(size_t)lc * R3 + x + R * (y + R * z)] = INF;
    const int fx[6] = {x == 0, x == R - 1, y == 0, y == R - 1, z == 0, z == R - 1};
    for (int f = 0; f < 6; ++f) {
        if (!fx[f]) continue;
        const int a = (f >> 1) == 0 ? y : x;
        const int b = (f >> 1) == 2 ? y : z;
        reinterpret_cast<UT*>(S.faces)[((size_t)lc * 6 + f) * R2 + a + R * b] = INF;
    }
}

template <int R, typename FT, typename UT>
__global__ void k_seed(SolveParams P, Slot S, int64_t round, int64_t nsrc,
                       const int64_t* __restrict__ idx3, const double* __restrict__ q,
                       const int* only_if) {
    if (only_if && *only_if == 0) return;
    constexpr int R2 = R * R, R3 = R * R * R;
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nsrc) return;
    const int64_t i = idx3[3 * n], j = idx3[3 * n + 1], k = idx3[3 * n + 2];
    const double qv = q[n] + 0.0;  // -0.0 -> +0.0 so that bit order is value order
    const UT qu = (UT)qv;           // the exit value in the storage precision
    if (i < 0 || i >= S.nx || j < 0 || j >= S.ny || k < 0 || k >= S.nz || !(qv >= 0.0) ||
        !(qu <= (UT)1.7976931348623157e308)) {
        atomicCAS(S.status, 0, EIK_EINVAL_DEV);
        return;
    }
    const int cx = (int)(i / R), cy = (int)(j / R), cz = (int)(k / R);
    const int x = (int)(i % R), y = (int)(j % R), z = (int)(k % R);
    const int lc = cx + S.ncx * (cy + S.ncy * cz);
    const int l = x + R * (y + R * z);
    atomic_min_val(reinterpret_cast<UT*>(S.u) + (size_t)lc * R3 + l, qu);
    reinterpret_cast<FT*>(S.f)[(size_t)lc * R3 + l] = FT(-1);
    // Face copies of the exit node.
    const int fx[6] = {x == 0, x == R - 1, y == 0, y == R - 1, z == 0, z == R - 1};
    for (int f = 0; f < 6; ++f) {
        if (!fx[f]) continue;
        const int a = (f >> 1) == 0 ? y : x;
        const int b = (f >> 1) == 2 ? y : z;
        atomic_min_val(reinterpret_cast<UT*>(S.faces) + ((size_t)lc * 6 + f) * R2 + a + R * b, qu);
    }
    tag_cell(P, round, S.cell_base + lc, FL_ALL, (double)qu);
    const int64_t nbr[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k},
                               {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
    for (int t = 0; t < 6; ++t) {
        const int64_t a = nbr[t][0], b = nbr[t][1], e = nbr[t][2];
        if (a < 0 || a >= S.nx || b < 0 || b >= S.ny || e < 0 || e >= S.nz) continue;
        const int nc = (int)(a / R) + S.ncx * ((int)(b / R) + S.ncy * (int)(e / R));
        if (nc != lc) tag_cell(P, round, S.cell_base + nc, FL_ALL, (double)qu);
    }
}

// Output (a8): cell-blocked u of one slot -> row-major u_out.
template <int R, typename UT>
__global__ void k_output(Slot S, double* __restrict__ out, const int* only_if) {
    if (only_if && *only_if == 0) return;
    const UT* ub = reinterpret_cast<const UT*>(S.u);
    constexpr int R3 = R * R * R;
    const size_t total = (size_t)S.nx * S.ny * S.nz;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(g % S.nx);
        const int j = (int)((g / S.nx) % S.ny);
        const int k = (int)(g / ((size_t)S.nx * S.ny));
        const int lc = i / R + S.ncx * (j / R + S.ncy * (k / R));
        const int l = i % R + R * (j % R + R * (k % R));
        out[g] = fabs((double)ub[(size_t)lc * R3 + l]);
    }
}

// ------------------------------------------------------------------------------------------
// Mixed precision: the single-precision result lifted to an FP64 starting point for the
// double-precision polish.  Values only decrease under the method's updates, so the polish
// reaches the FP64 solution from any starting point at or above it; the FP32 values are
// multiplied by `factor` (a bound on their relative error, plus margin) to start above it.

template <int R>
__global__ void k_lift(Slot S32, Slot S64, double factor) {
    constexpr int R3 = R * R * R, R2 = R * R;
    const size_t nodes = (size_t)S64.ncell * R3, nf = (size_t)S64.ncell * 6 * R2;
    const float* u32 = reinterpret_cast<const float*>(S32.u);
    const float* f32 = reinterpret_cast<const float*>(S32.faces);
    double* u64 = reinterpret_cast<double*>(S64.u);
    double* f64 = reinterpret_cast<double*>(S64.faces);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t g0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    for (size_t g = g0; g < nodes; g += stride) u64[g] = fabs((double)u32[g]) * factor;
    for (size_t g = g0; g < nf; g += stride) f64[g] = (double)f32[g] * factor;
}

// Empty round lists and round counter 0 for a following launch (status and counters kept).
__global__ void k_reset_rounds(SolveParams P) {
    const int g0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    if (g0 < 4) {
        P.ctl[g0].count = 0;
        P.ctl[g0].minkey = dbits(__builtin_inf());
    }
    if (g0 < 4 * kPopSegs) P.seg_cursor[g0 * 32] = 0;
    if (g0 == 0) *P.next_round = 0;
    for (int g = g0; g < 4 * P.nslots; g += stride) P.slot_minkey[g] = dbits(__builtin_inf());
}

// Whether each slot has a cell in the list of the next launch's first round (the host's test
// for finished grids): 1 if so, else 0.  Every writer stores the same 1, so plain stores do.
__global__ void k_slot_counts_zero(int* counts, int nslots) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < nslots) counts[g] = 0;
}
__global__ void k_slot_counts(SolveParams P, int* counts) {
    const int64_t round = *P.next_round;
    const uint32_t n = P.ctl[round & 3].count;
    const int32_t* lst = P.list[round & 1];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        counts[P.cell_slot[lst[i]]] = 1;
}

// ------------------------------------------------------------------------------------------
// Host-side launchers.

template <int R, int W, int INNER, typename UT>
constexpr size_t solve_lds_bytes() { return sizeof(WaveLds<R, INNER, UT>) * W; }

template <int R, typename FT, int W, int INNER, typename UT, bool ASYNCK = false>
static hipError_t launch_solve_t(const SolveParams& P, hipStream_t s, int workers, int* used,
                                 int coop) {
    const size_t lds = solve_lds_bytes<R, W, INNER, UT>();
    auto kern = ASYNCK ? k_solve_async<R, FT, W, INNER, UT> : k_solve<R, FT, W, INNER, UT>;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int ncu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * W, lds);
    if (e != hipSuccess) return e;
    // The grid barrier needs every workgroup resident at once.  The occupancy query does not
    // round LDS up to the allocation granularity, so bound it again with a 2 KiB granule.
    int lds_cu = 0;
    e = hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    if (e != hipSuccess) return e;
    const size_t granule = 2048;
    const size_t lds_alloc = (lds + 1024 + granule - 1) / granule * granule;  // + static LDS
    const int per_cu_lds = (int)((size_t)lds_cu / lds_alloc);
    if (per_cu_lds < per_cu) per_cu = per_cu_lds;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int grid = per_cu * ncu;
    if (workers > 0) grid = workers < grid ? workers : grid;
    // The ring of the launch without rounds holds one outstanding ticket per wave beyond its
    // cells (kRingExtra).
    if (ASYNCK && (int64_t)grid * W * 2 > kRingExtra) return hipErrorInvalidConfiguration;
    *used = grid;
    if (std::getenv("EIK_DEBUG")) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess)
            std::fprintf(stderr,
                         "[eik] %s cu=%d lds/block=%zu lds/cu=%zu regs/cu=%d coop=%d | kernel R=%d "
                         "W=%d lds=%zu per_cu=%d grid=%d\n",
                         prop.gcnArchName, ncu, (size_t)prop.sharedMemPerBlock,
                         (size_t)prop.maxSharedMemoryPerMultiProcessor, prop.regsPerMultiprocessor,
                         prop.cooperativeLaunch, R, W, lds, per_cu, grid);
    }
    SolveParams Pc = P;
    if (!coop) {
        // One round, no grid barrier: the workgroups need not be resident together.
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * W), lds, s, Pc);
        return hipGetLastError();
    }
    void* args[] = {&Pc};
    e = hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(64 * W), args, lds, s);
    if (e != hipSuccess && std::getenv("EIK_DEBUG"))
        std::fprintf(stderr, "[eik] cooperative launch of %d x %d threads failed: %s\n", grid,
                     64 * W, hipGetErrorString(e));
    return e;
}

// Workers (waves) per workgroup: one workgroup fills a CU -- as many waves as the register
// budget allows (three per SIMD in FP64, four in FP32), bounded by the CU's 160 KiB of LDS
// (150 KiB of it up to r = 8; at r = 16 all but 1 KiB for the static arrays, which makes room
// for two FP64 or four FP32 cells per CU) -- so a round barrier has one arrival and one
// release/acquire pair per CU (each of those costs microseconds per round at hundreds of
// workgroups).
template <int R, int INNER, typename UT>
constexpr int waves_per_group() {
    // Two cells per wave need up to 256 registers: two waves per SIMD.
    constexpr int by_regs = INNER == INNER_PAIR ? 8 : (sizeof(UT) == 4 ? 16 : 12);
    constexpr unsigned budget = (R == 16 ? 159u : 150u) * 1024u;
    constexpr int by_lds = (int)(budget / sizeof(WaveLds<R, INNER, UT>));
    return by_regs < by_lds ? by_regs : by_lds;
}

template <int R, typename FT, typename UT, bool ASYNCK>
static hipError_t solve_rounds_ut(const SolveParams& P, hipStream_t s, int workers, int* used,
                                  int coop) {
    if (P.inner == INNER_SWEEP)
        return launch_solve_t<R, FT, waves_per_group<R, INNER_SWEEP, UT>(), INNER_SWEEP, UT,
                              ASYNCK>(P, s, workers, used, coop);
    if (P.inner == INNER_LIST)
        return launch_solve_t<R, FT, waves_per_group<R, INNER_LIST, UT>(), INNER_LIST, UT,
                              ASYNCK>(P, s, workers, used, coop);
    if constexpr (R <= 8) {
        if (P.inner == INNER_DUAL)
            return launch_solve_t<R, FT, waves_per_group<R, INNER_DUAL, UT>(), INNER_DUAL, UT,
                                  ASYNCK>(P, s, workers, used, coop);
        // Two cells per wave are taken from the rounds' lists, not from the ring.
        if (P.inner == INNER_PAIR && !ASYNCK)
            return launch_solve_t<R, FT, waves_per_group<R, INNER_PAIR, UT>(), INNER_PAIR, UT,
                                  false>(P, s, workers, used, coop);
    }
    return hipErrorInvalidValue;  // the host refuses two streams at r = 16 and pairs without rounds
}

template <int R, typename FT, bool ASYNCK = false>
static hipError_t solve_rounds_t(const SolveParams& P, hipStream_t s, int workers, int* used,
                                 int coop) {
    return P.fp32 ? solve_rounds_ut<R, FT, float, ASYNCK>(P, s, workers, used, coop)
                  : solve_rounds_ut<R, FT, double, ASYNCK>(P, s, workers, used, coop);
}

hipError_t launch_solve_async(const SolveParams& P, int cell, int f_dtype, hipStream_t s,
                              int workers, int* used) {
    if (cell == 16)
        return f_dtype == EIK_F32 ? solve_rounds_t<16, float, true>(P, s, workers, used, 1)
                                  : solve_rounds_t<16, double, true>(P, s, workers, used, 1);
    if (cell == 8)
        return f_dtype == EIK_F32 ? solve_rounds_t<8, float, true>(P, s, workers, used, 1)
                                  : solve_rounds_t<8, double, true>(P, s, workers, used, 1);
    if (cell == 4)
        return f_dtype == EIK_F32 ? solve_rounds_t<4, float, true>(P, s, workers, used, 1)
                                  : solve_rounds_t<4, double, true>(P, s, workers, used, 1);
    return hipErrorInvalidValue;
}

static int blocks_for(size_t n, int threads) {
    size_t b = (n + threads - 1) / threads;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : (int)b;
}

hipError_t launch_init_global(const SolveParams& P, hipStream_t s) {
    hipLaunchKernelGGL(k_init_global, dim3(blocks_for((size_t)4 * P.nslots + 64, 256)), dim3(256),
                       0, s, P);
    return hipGetLastError();
}

template <int R, typename UT>
static void init_slot_t(const SolveParams& P, const Slot& S, int slot, int f_dtype,
                        const void* F, const double* u_approx, double lift, int blocks,
                        int threads, hipStream_t s, const int* only_if) {
    hipLaunchKernelGGL((k_init_cells<R, UT>), dim3(blocks), dim3(threads), 0, s, P, S, slot,
                       only_if);
    if (f_dtype == EIK_F32)
        hipLaunchKernelGGL((k_init_nodes<R, float, UT>), dim3(blocks), dim3(threads), 0, s, S,
                           reinterpret_cast<const float*>(F), u_approx, lift, only_if);
    else
        hipLaunchKernelGGL((k_init_nodes<R, double, UT>), dim3(blocks), dim3(threads), 0, s, S,
                           reinterpret_cast<const double*>(F), u_approx, lift, only_if);
    if (u_approx)
        hipLaunchKernelGGL((k_faces_from_u<R, UT>), dim3(blocks), dim3(threads), 0, s, S,
                           only_if);
}

hipError_t launch_init_slot(const SolveParams& P, const Slot& S, int slot, int cell, int f_dtype,
                            const void* F, const double* u_approx, double lift, hipStream_t s,
                            const int* only_if) {
    const int threads = 256;
    const size_t nodes = (size_t)S.ncell * cell * cell * cell;
    const int blocks = blocks_for(nodes, threads);
    if (cell == 16 && S.fp32)
        init_slot_t<16, float>(P, S, slot, f_dtype, F, u_approx, lift, blocks, threads, s, only_if);
    else if (cell == 16)
        init_slot_t<16, double>(P, S, slot, f_dtype, F, u_approx, lift, blocks, threads, s, only_if);
    else if (cell == 8 && S.fp32)
        init_slot_t<8, float>(P, S, slot, f_dtype, F, u_approx, lift, blocks, threads, s, only_if);
    else if (cell == 8)
        init_slot_t<8, double>(P, S, slot, f_dtype, F, u_approx, lift, blocks, threads, s, only_if);
    else if (cell == 4 && S.fp32)
        init_slot_t<4, float>(P, S, slot, f_dtype, F, u_approx, lift, blocks, threads, s, only_if);
    else if (cell == 4)
        init_slot_t<4, double>(P, S, slot, f_dtype, F, u_approx, lift, blocks, threads, s, only_if);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int R, typename UT>
static void seed_t(const SolveParams& P, const Slot& S, int f_dtype, int64_t round, int64_t nsrc,
                   const int64_t* idx3, const double* q, hipStream_t s, const int* only_if,
                   bool clear_first) {
    const int sb = (int)((nsrc + 63) / 64);
    if (clear_first)
        hipLaunchKernelGGL((k_seed_clear<R, UT>), dim3(sb), dim3(64), 0, s, S, nsrc, idx3);
    if (f_dtype == EIK_F32)
        hipLaunchKernelGGL((k_seed<R, float, UT>), dim3(sb), dim3(64), 0, s, P, S, round, nsrc,
                           idx3, q, only_if);
    else
        hipLaunchKernelGGL((k_seed<R, double, UT>), dim3(sb), dim3(64), 0, s, P, S, round, nsrc,
                           idx3, q, only_if);
}

hipError_t launch_seed(const SolveParams& P, const Slot& S, int cell, int f_dtype, int64_t round,
                       int64_t nsrc, const int64_t* idx3, const double* q, hipStream_t s,
                       const int* only_if, bool clear_first) {
    if (nsrc <= 0) return hipSuccess;
#define EIK_SEED(R, UT) seed_t<R, UT>(P, S, f_dtype, round, nsrc, idx3, q, s, only_if, clear_first)
    if (cell == 16 && S.fp32) EIK_SEED(16, float);
    else if (cell == 16) EIK_SEED(16, double);
    else if (cell == 8 && S.fp32) EIK_SEED(8, float);
    else if (cell == 8) EIK_SEED(8, double);
    else if (cell == 4 && S.fp32) EIK_SEED(4, float);
    else if (cell == 4) EIK_SEED(4, double);
    else return hipErrorInvalidValue;
#undef EIK_SEED
    return hipGetLastError();
}

hipError_t launch_solve_rounds(const SolveParams& P, int cell, int f_dtype, hipStream_t s,
                               int workers, int* used, int coop) {
    if (cell == 16)
        return f_dtype == EIK_F32 ? solve_rounds_t<16, float>(P, s, workers, used, coop)
                                  : solve_rounds_t<16, double>(P, s, workers, used, coop);
    if (cell == 8)
        return f_dtype == EIK_F32 ? solve_rounds_t<8, float>(P, s, workers, used, coop)
                                  : solve_rounds_t<8, double>(P, s, workers, used, coop);
    if (cell == 4)
        return f_dtype == EIK_F32 ? solve_rounds_t<4, float>(P, s, workers, used, coop)
                                  : solve_rounds_t<4, double>(P, s, workers, used, coop);
    return hipErrorInvalidValue;
}

__global__ void k_put_slots(Slot a, Slot b, int n, Slot* dst) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        dst[0] = a;
        if (n > 1) dst[1] = b;
    }
}

struct HostExits {
    int64_t idx3[3 * kHostExitsMax];
    double q[kHostExitsMax];
};

__global__ void k_put_exits(HostExits x, int n, int64_t* idx3, double* q) {
    const int t = threadIdx.x;
    if (blockIdx.x != 0 || t >= n) return;
    idx3[3 * t] = x.idx3[3 * t];
    idx3[3 * t + 1] = x.idx3[3 * t + 1];
    idx3[3 * t + 2] = x.idx3[3 * t + 2];
    q[t] = x.q[t];
}

hipError_t launch_put_slots(const Slot& a, const Slot& b, int n, Slot* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_put_slots, dim3(1), dim3(64), 0, s, a, b, n, dst);
    return hipGetLastError();
}

hipError_t launch_put_exits(const int64_t* idx3, const double* q, int n, int64_t* idx3_dst,
                            double* q_dst, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > kHostExitsMax) return hipErrorInvalidValue;
    HostExits x;
    for (int t = 0; t < 3 * n; ++t) x.idx3[t] = idx3[t];
    for (int t = 0; t < n; ++t) x.q[t] = q[t];
    hipLaunchKernelGGL(k_put_exits, dim3(1), dim3(64), 0, s, x, n, idx3_dst, q_dst);
    return hipGetLastError();
}

__global__ void k_halt_reset(SolveParams P) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *P.halted = 0u;
}

// After the last one-round launch of a host-driven loop over rounds [begin, end): if no launch
// stopped the loop, round `end` is where the next launch starts, and with `end` at the round
// cap a non-empty list there means the cap was reached.
__global__ void k_hostloop_end(SolveParams P, int64_t end) {
    if (blockIdx.x != 0 || threadIdx.x != 0 || *P.halted) return;
    *P.next_round = end;
    if (end >= P.max_rounds && P.ctl[end & 3].count != 0) atomicCAS(P.status, 0, EIK_ENOCONV_DEV);
}

hipError_t launch_halt_reset(const SolveParams& P, hipStream_t s) {
    hipLaunchKernelGGL(k_halt_reset, dim3(1), dim3(64), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_hostloop_end(const SolveParams& P, int64_t end, hipStream_t s) {
    hipLaunchKernelGGL(k_hostloop_end, dim3(1), dim3(64), 0, s, P, end);
    return hipGetLastError();
}

hipError_t launch_output(const Slot& S, int cell, double* u_out, hipStream_t s,
                         const int* only_if) {
    const int threads = 256;
    const int ob = blocks_for((size_t)S.nx * S.ny * S.nz, threads);
    if (cell == 16 && S.fp32)
        hipLaunchKernelGGL((k_output<16, float>), dim3(ob), dim3(threads), 0, s, S, u_out, only_if);
    else if (cell == 16)
        hipLaunchKernelGGL((k_output<16, double>), dim3(ob), dim3(threads), 0, s, S, u_out, only_if);
    else if (cell == 8 && S.fp32)
        hipLaunchKernelGGL((k_output<8, float>), dim3(ob), dim3(threads), 0, s, S, u_out, only_if);
    else if (cell == 8)
        hipLaunchKernelGGL((k_output<8, double>), dim3(ob), dim3(threads), 0, s, S, u_out, only_if);
    else if (S.fp32)
        hipLaunchKernelGGL((k_output<4, float>), dim3(ob), dim3(threads), 0, s, S, u_out, only_if);
    else
        hipLaunchKernelGGL((k_output<4, double>), dim3(ob), dim3(threads), 0, s, S, u_out, only_if);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Restart of one slot from +inf with the inputs already staged (the conditional re-solve of a
// polish that failed its check): the blocked speeds still mark the exits (-1) and padding (0),
// and the exit nodes still hold q (they are never updated), so nothing of the caller's is read.

template <int R, typename FT, typename UT>
__global__ void k_restart_nodes(Slot S, const int* only_if) {
    if (only_if && *only_if == 0) return;
    constexpr int R3 = R * R * R;
    const size_t total = (size_t)S.ncell * R3;
    const FT* fb = reinterpret_cast<const FT*>(S.f);
    UT* ub = reinterpret_cast<UT*>(S.u);
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const FT fv = fb[g];
        if (fv > FT(0)) ub[g] = (UT)__builtin_inf();
        else if (fv == FT(0)) ub[g] = (UT)__builtin_nan("");
    }
}

// Queues, for round `round`, the cell of every exit node and the cells of its six grid
// neighbours with every node active and cell value q, as k_seed does from the exit list.
template <int R, typename FT, typename UT>
__global__ void k_reseed(SolveParams P, Slot S, int64_t round, const int* only_if) {
    if (only_if && *only_if == 0) return;
    constexpr int R3 = R * R * R;
    const size_t total = (size_t)S.ncell * R3;
    const FT* fb = reinterpret_cast<const FT*>(S.f);
    const UT* ub = reinterpret_cast<const UT*>(S.u);
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        if (!(fb[g] < FT(0))) continue;
        const int lc = (int)(g / R3), l = (int)(g % R3);
        const CellXYZ cc = cell_coords(S, lc);
        const int64_t i = cc.x * R + l % R, j = cc.y * R + (l / R) % R, k = cc.z * R + l / (R * R);
        const double qv = (double)ub[g];
        tag_cell(P, round, S.cell_base + lc, FL_ALL, qv);
        const int64_t nbr[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k},
                                   {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
        for (int t = 0; t < 6; ++t) {
            const int64_t a = nbr[t][0], b = nbr[t][1], e = nbr[t][2];
            if (a < 0 || a >= S.nx || b < 0 || b >= S.ny || e < 0 || e >= S.nz) continue;
            const int nc = (int)(a / R) + S.ncx * ((int)(b / R) + S.ncy * (int)(e / R));
            if (nc != lc) tag_cell(P, round, S.cell_base + nc, FL_ALL, qv);
        }
    }
}

template <int R, typename FT, typename UT>
static void restart_t(const SolveParams& P, const Slot& S, int slot, int64_t round, int blocks,
                      int threads, hipStream_t s, const int* only_if) {
    hipLaunchKernelGGL((k_init_cells<R, UT>), dim3(blocks), dim3(threads), 0, s, P, S, slot,
                       only_if);
    hipLaunchKernelGGL((k_restart_nodes<R, FT, UT>), dim3(blocks), dim3(threads), 0, s, S, only_if);
    hipLaunchKernelGGL((k_faces_from_u<R, UT>), dim3(blocks), dim3(threads), 0, s, S, only_if);
    hipLaunchKernelGGL((k_reseed<R, FT, UT>), dim3(blocks), dim3(threads), 0, s, P, S, round,
                       only_if);
}

hipError_t launch_restart_slot(const SolveParams& P, const Slot& S, int slot, int cell,
                               int f_dtype, int64_t round, hipStream_t s, const int* only_if) {
    const int threads = 256;
    const int blocks = blocks_for((size_t)S.ncell * cell * cell * cell, threads);
#define EIK_RESTART(R, UT)                                                                   \
    (f_dtype == EIK_F32 ? restart_t<R, float, UT>(P, S, slot, round, blocks, threads, s, only_if) \
                        : restart_t<R, double, UT>(P, S, slot, round, blocks, threads, s, only_if))
    if (cell == 16) { if (S.fp32) EIK_RESTART(16, float); else EIK_RESTART(16, double); }
    else if (cell == 8) { if (S.fp32) EIK_RESTART(8, float); else EIK_RESTART(8, double); }
    else if (cell == 4) { if (S.fp32) EIK_RESTART(4, float); else EIK_RESTART(4, double); }
    else return hipErrorInvalidValue;
#undef EIK_RESTART
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Check of a polished result (FP64, row-major u, tol 0): at the fixed point the method reaches,
// every node outside the exit set satisfies eq. (2) with its final neighbours, i.e. its local
// solve returns its own value up to rounding.  A polish that started below the solution
// somewhere cannot raise those values (updates only decrease), and the node where such a
// region meets correct upwind values has a local solve above its value.  A node whose local
// solve differs from its value by more than 1e-11 s + 2^-46 U (rounding of the same operator on
// the same values is a few units of 2^-53 U) flags the grid; an error that passes is at most
// the sum of such residuals along a characteristic, below 1e-10 relative.
__device__ __forceinline__ double nbr_min(const double* u, size_t g, size_t stride, bool lo,
                                          bool hi) {
    const double a = lo ? u[g - stride] : __builtin_inf();
    const double b = hi ? u[g + stride] : __builtin_inf();
    return vmin(a, b);
}

template <int R, typename FT>
__global__ void k_polish_check(Slot S, const double* __restrict__ u, int* redo,
                               unsigned long long* stats) {
    if (S.tol > 0.0) return;  // early-terminated sweeps stop above the fixed point by design
    constexpr int R3 = R * R * R;
    const FT* fb = reinterpret_cast<const FT*>(S.f);
    const size_t nx = S.nx, ny = S.ny, nz = S.nz, total = nx * ny * nz;
    bool bad = false;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(g % nx), j = (int)((g / nx) % ny), k = (int)(g / (nx * ny));
        const int lc = i / R + S.ncx * (j / R + S.ncy * (k / R));
        const double fv = (double)fb[(size_t)lc * R3 + i % R + R * (j % R + R * (k % R))];
        if (!(fv > 0.0)) continue;  // exit node (fixed at q)
        const double U = u[g];
        const double s = S.h / fv;
        const double G = local_solve(nbr_min(u, g, 1, i > 0, i + 1 < S.nx),
                                     nbr_min(u, g, nx, j > 0, j + 1 < S.ny),
                                     nbr_min(u, g, nx * ny, k > 0, k + 1 < S.nz), s);
        if (U == __builtin_inf() && G == __builtin_inf()) continue;  // unreachable
        const double thr = 1e-11 * s + 0x1p-46 * U;
        bad |= !(fabs(G - U) <= thr);  // NaN and a finite G at an unreached node fail too
    }
    if (__any(bad) && (threadIdx.x & 63) == 0 && atomicExch(redo, 1) == 0)
        atomicAdd(&stats[ST_REDONE], 1ull);
}

__global__ void k_clear_int(int* p, int n) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) p[g] = 0;
}

hipError_t launch_polish_check(const Slot& S, int cell, int f_dtype, const double* u_out,
                               int* redo, unsigned long long* stats, hipStream_t s) {
    const int threads = 256;
    const int ob = blocks_for((size_t)S.nx * S.ny * S.nz, threads);
#define EIK_CHECK_LAUNCH(R, FT) \
    hipLaunchKernelGGL((k_polish_check<R, FT>), dim3(ob), dim3(threads), 0, s, S, u_out, redo, stats)
    if (cell == 16) {
        if (f_dtype == EIK_F32) EIK_CHECK_LAUNCH(16, float); else EIK_CHECK_LAUNCH(16, double);
    } else if (cell == 8) {
        if (f_dtype == EIK_F32) EIK_CHECK_LAUNCH(8, float); else EIK_CHECK_LAUNCH(8, double);
    } else {
        if (f_dtype == EIK_F32) EIK_CHECK_LAUNCH(4, float); else EIK_CHECK_LAUNCH(4, double);
    }
#undef EIK_CHECK_LAUNCH
    return hipGetLastError();
}

hipError_t launch_clear_ints(int* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_int, dim3(blocks_for((size_t)n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_lift(const Slot& S32, const Slot& S64, int cell, double factor, hipStream_t s) {
    const int threads = 256;
    const int blocks = blocks_for((size_t)S64.ncell * cell * cell * cell, threads);
    if (cell == 16)
        hipLaunchKernelGGL((k_lift<16>), dim3(blocks), dim3(threads), 0, s, S32, S64, factor);
    else if (cell == 8)
        hipLaunchKernelGGL((k_lift<8>), dim3(blocks), dim3(threads), 0, s, S32, S64, factor);
    else
        hipLaunchKernelGGL((k_lift<4>), dim3(blocks), dim3(threads), 0, s, S32, S64, factor);
    return hipGetLastError();
}


hipError_t launch_reset_rounds(const SolveParams& P, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_rounds, dim3(blocks_for((size_t)4 * P.nslots + 64, 256)),
                       dim3(256), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_slot_counts(const SolveParams& P, int* counts, int nslots, hipStream_t s) {
    hipLaunchKernelGGL(k_slot_counts_zero, dim3(blocks_for((size_t)nslots, 256)), dim3(256), 0,
                       s, counts, nslots);
    hipLaunchKernelGGL(k_slot_counts, dim3(64), dim3(256), 0, s, P, counts);
    return hipGetLastError();
}

}  // namespace eik
