// eik_internal.h -- types shared by the kernels and the host API of libeik (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/eik.h"

namespace eik {

// Cell flag word (one per cell and round parity).
constexpr uint32_t FL_FACES = 0x3Fu;      // bit f: face f received new inflow (0 -x ... 5 +z)
constexpr uint32_t FL_ALL = 1u << 6;      // every node active (first visit / re-queue)
constexpr uint32_t FL_QUEUED = 1u << 7;   // already in that round's list
constexpr int FL_DIR_SHIFT = 8;           // bits 8..15: preferred sweep directions
constexpr int FL_GRAY_SHIFT = 16;         // bits 16..18: Gray-cycle position to resume at
constexpr uint32_t FL_GRAY_SET = 1u << 19;  // bits 16..18 are valid (a capped visit resumes)
constexpr uint32_t FL_RUNNING = 1u << 20;   // without rounds: a worker owns the cell now

// Device status values are the public codes.
constexpr int EIK_EINVAL_DEV = EIK_EINVAL;
constexpr int EIK_ENOCONV_DEV = EIK_ENOCONV;
constexpr int EIK_ECANCELLED_DEV = EIK_ECANCELLED;


// Counter slots.
enum {
    ST_ROUNDS = 0, ST_VISITS, ST_SWEEPS, ST_UPDATES, ST_DEFERRED, ST_REQUEUED,
    // shader-clock cycles summed over workers, by phase
    ST_CYC_POP, ST_CYC_STAGE, ST_CYC_SWEEP, ST_CYC_WRITE, ST_CYC_WAIT, ST_WORKERS,
    ST_REDONE,  // polished grids that failed the eq. (2) check and were solved again
    ST_COUNT = 16,
    // histograms over visits: sweeps (bucket min(n, 31)) and duration (bucket floor(log2 cycles))
    ST_HIST_SWEEPS = 16, ST_HIST_CYCLES = 48, ST_TOTAL = 80
};

// Per-round control block: list length and smallest cell value in the list, each on its own
// cache line so that appends and minimum updates do not contend (the pop cursors are
// seg_cursor).
struct RoundCtl {
    uint32_t pad0[32];
    uint32_t count;
    uint32_t pad1[15];
    uint64_t minkey;
    uint64_t pad2[7];
};
static_assert(sizeof(RoundCtl) == 256, "RoundCtl is 256 bytes");

// Small control area of the workspace (byte offsets).
constexpr size_t kSmallCtl = 0;        // 4 x RoundCtl
constexpr size_t kSmallBar = 1024;     // barrier: arrivals at [0], generation at [64] (uint32)
constexpr size_t kSmallStatus = 2048;  // int
constexpr size_t kSmallNextRound = 2112;  // int64: first round of the next launch
constexpr size_t kSmallHalted = 2176;  // uint32: a one-round launch found nothing left to do
constexpr size_t kSmallStats = 2304;   // ST_TOTAL x uint64
// Scheduling without rounds: ring head and tail (uint64 tickets), queued-or-running cell count
// (uint64) and the done word (uint32), each on its own 256-byte line.
constexpr size_t kSmallAsyncHead = 3072;
constexpr size_t kSmallAsyncTail = 3328;
constexpr size_t kSmallAsyncPending = 3584;
constexpr size_t kSmallAsyncDone = 3840;
// Pop cursors of the rounds' list segments: [4 rounds][kPopSegs], 128 bytes apart.
constexpr size_t kSmallSegCursor = 4096;
constexpr size_t kSmallBytes = 12288;
// A round's list is popped through this many segments (two per XCD), each with its own cursor,
// so that the pops of the 256 workgroups do not all meet on one atomic word.
constexpr int kPopSegs = 16;
constexpr int kBarGen = 64;            // index of the generation word in the barrier array

// One grid of a (possibly batched) solve.  Its cells occupy the global cell ids
// [cell_base, cell_base + ncell); its arrays are its own.
struct Slot {
    int nx, ny, nz;        // grid nodes per axis
    int ncx, ncy, ncz;     // cells per axis
    int cell_base;         // global id of the slot's cell 0
    int ncell;             // ncx * ncy * ncz
    double h, tol;
    void* u;               // [ncell][r^3] cell-blocked values (FP64, or FP32 if fp32)
    void* f;               // [ncell][r^3] cell-blocked speeds (F dtype); 0 padding, <0 exit
    void* faces;           // [ncell][6][r^2] border layers (value type of u)
    int* status;           // this grid's status word (device)
    int fp32;              // values stored and computed in single precision
    int pad;
};

struct SolveParams {
    int max_sweeps;
    int inner;             // in-cell solver: 0 sweeps, 1 active-list relaxation, 2 dual sweeps
    int fp32;              // value type of every slot of the launch: 1 FP32, 0 FP64
    int cell_value;        // 0: eq. (3) cell values; 1: the earlier eq. (4), kept across visits
    int slot_band;         // 1: with a band, each slot's band starts at that slot's own minimum
    int nslots;            // entries of the slot table (row length of slot_minkey)
    int single_round;      // 1: one round per launch, no grid barrier (host-driven loop)
    int count_workers;     // 1: this launch adds its waves to the worker counter
    int64_t round_begin;   // first round of this launch
    int64_t round_end;     // the launch stops after round round_end - 1 (end of an epoch)
    int64_t max_rounds;    // absolute cap on rounds -> EIK_ENOCONV
    double delta;
    uint64_t shuffle;
    uint64_t watchdog_polls;  // polls of the barrier word before a wait is abandoned
    const Slot* slots;     // slot table (device)
    const int* cell_slot;  // [global cells] slot of each cell
    uint64_t* key[2];      // cell values (FP64 bit patterns, all >= +0), global cell ids
    uint64_t* key_keep;    // [global cells] eq. (4) cell values, never reset by a visit
    uint32_t* flags[2];
    int32_t* list[2];
    RoundCtl* ctl;         // [4] control blocks, slot = round & 3
    uint32_t* seg_cursor;  // round t, segment g: seg_cursor[((t & 3) * kPopSegs + g) * 32]
    uint64_t* slot_minkey; // [4][nslots] smallest cell value queued per slot, row = round & 3
    uint32_t* bar;         // grid barrier: bar[0] arrivals, bar[kBarGen] generation
    int* status;           // device status word of the launch (watchdog, round cap)
    unsigned long long* stats;  // [ST_TOTAL]
    int64_t* next_round;   // written when the launch ends: the first round of the next launch
    uint32_t* halted;      // host-driven loop: set by the first launch that finds its round's
                           // list empty, the launch status set or the round cap reached
    int64_t* round_log;    // optional [2 * round_log_len]
    int64_t round_log_len;
    // Scheduling without rounds (k_solve_async): the ring of queued cells is list[0..1] taken as
    // one array of 2 * ncells + kRingExtra entries (-1 = empty).
    int64_t ncells;        // global cells of the launch
    unsigned long long* async_head;     // next ticket to pop
    unsigned long long* async_tail;     // next position to push
    unsigned long long* async_pending;  // cells queued or being visited
    uint32_t* async_done;               // set when async_pending reaches 0
    // Race-detection aids: a host-mapped cancel word (a solve stops once it holds a sequence
    // number >= cancel_seq) and a seed of pseudo-random delays before each visit (0 = none).
    const uint32_t* cancel;
    uint32_t cancel_seq;
    uint64_t jitter;
    unsigned long long* bq_ctl;         // bucket heads, tails and the lowest bucket (or null)
    int32_t* bq_ring;                   // kBuckets rings of bq_cap 64-bit words (lap, cell)
    int64_t bq_cap;
};

// Positions of the ring of queued cells (scheduling without rounds) beyond twice the cells: a
// ring position is in use from the push or the ticket that claims it, whichever comes first,
// until the item is read; at most one item per cell is queued and at most one ticket per wave
// is outstanding, so 2 * cells + this (above the waves of any launch) positions never wrap
// onto a position in use.
constexpr int64_t kRingExtra = 16384;
// Scheduling without rounds with a priority band (delta > 0): cells are kept in kBuckets rings
// by cell value, bucket floor(value / delta) (relative to a moving lowest bucket), each ring
// with room for every cell plus kRingExtra; a wave pops from the lowest non-empty bucket.
constexpr int kBuckets = 64;
// Control words of the buckets (byte offsets in their region): head and tail of bucket b at
// b * 128 and b * 128 + 64, the lowest bucket (absolute number) at kBuckets * 128.
constexpr size_t kBucketCtlBytes = (size_t)kBuckets * 128 + 256;

// Host-side exits that a kernel argument can carry (the allocation-free solve).
constexpr int kHostExitsMax = 32;

// Launchers (eik_kernels.hip).  All enqueue on `s` and return the first launch error.
// Slot table entries dst[0..n) <- a, b written by a kernel from its arguments (n = 1 or 2).
hipError_t launch_put_slots(const Slot& a, const Slot& b, int n, Slot* dst, hipStream_t s);
// n <= kHostExitsMax host-side exits (idx3: n x 3, q: n) copied to device arrays through a
// kernel's arguments.
hipError_t launch_put_exits(const int64_t* idx3, const double* q, int n, int64_t* idx3_dst,
                            double* q_dst, hipStream_t s);
hipError_t launch_init_global(const SolveParams& P, hipStream_t s);
// Cells of slot S cleared, speeds staged, values <- +inf or, if u_approx (row-major, device) is
// given, <- |u_approx| * lift with face copies to match.
// only_if (device, may be null): the init, seed and output kernels do nothing unless *only_if
// is nonzero (the conditional re-solve after a failed polish check).
hipError_t launch_init_slot(const SolveParams& P, const Slot& S, int slot, int cell, int f_dtype,
                            const void* F, const double* u_approx, double lift, hipStream_t s,
                            const int* only_if = nullptr);
// clear_first: the grid starts from an approximation, whose values at the exits are replaced
// (not lowered) by q.
hipError_t launch_seed(const SolveParams& P, const Slot& S, int cell, int f_dtype, int64_t round,
                       int64_t nsrc, const int64_t* idx3, const double* q, hipStream_t s,
                       const int* only_if = nullptr, bool clear_first = false);
// The persistent solve kernel: a cooperative launch that runs rounds [P.round_begin,
// P.round_end) with a grid barrier between rounds (coop = 1), or an ordinary launch of one
// round (coop = 0, P.single_round = 1).
hipError_t launch_solve_rounds(const SolveParams& P, int cell, int f_dtype, hipStream_t s,
                               int workers, int* used, int coop);
// The persistent solve kernel without rounds (cooperative launch): cells queued in round
// P.round_begin's list are visited as they are popped from a ring, neighbours pushed as they
// are tagged, and the launch ends when no cell is queued or being visited and a verification
// pass over every cell finds eq. (2) satisfied.
hipError_t launch_solve_async(const SolveParams& P, int cell, int f_dtype, hipStream_t s,
                              int workers, int* used);
// Host-driven loop: *P.halted <- 0 before the first one-round launch; after the last one, the
// round cap is checked for round `end` (EIK_ENOCONV if its list is not empty).
hipError_t launch_halt_reset(const SolveParams& P, hipStream_t s);
hipError_t launch_hostloop_end(const SolveParams& P, int64_t end, hipStream_t s);
hipError_t launch_output(const Slot& S, int cell, double* u_out, hipStream_t s,
                         const int* only_if = nullptr);
// *redo <- 1 (and stats[ST_REDONE] += 1 once) if the FP64 row-major result u_out of slot S
// violates eq. (2) at some node beyond rounding (see k_polish_check).  *redo must be 0 before.
hipError_t launch_polish_check(const Slot& S, int cell, int f_dtype, const double* u_out,
                               int* redo, unsigned long long* stats, hipStream_t s);
hipError_t launch_clear_ints(int* p, int n, hipStream_t s);
// Slot S restarted from +inf with its staged speeds and exit values (nothing of the caller's
// read) and its exit cells queued for `round`; does nothing unless *only_if (if given) is set.
hipError_t launch_restart_slot(const SolveParams& P, const Slot& S, int slot, int cell,
                               int f_dtype, int64_t round, hipStream_t s, const int* only_if);
// Mixed precision: FP64 values (and faces) of S64 <- FP32 ones of S32 times factor.
hipError_t launch_lift(const Slot& S32, const Slot& S64, int cell, double factor, hipStream_t s);
// Round lists emptied and the round counter reset (launch status and counters kept).
hipError_t launch_reset_rounds(const SolveParams& P, hipStream_t s);
// counts[slot] <- 1 if the slot has a cell queued for the first round of the next launch
// (P.next_round), else 0.
hipError_t launch_slot_counts(const SolveParams& P, int* counts, int nslots, hipStream_t s);

}  // namespace eik
