// eik_api.hip -- the C ABI of libeik: argument validation, workspaces, launches, the server.
//
// Every entry point is declared, with its contract, in include/eik.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "eik_internal.h"

// Workspace of eik_solve_noalloc (see NoallocDevice below).
constexpr size_t kScratchBytes = size_t(384) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

using eik::kSmallBar;
using eik::kSmallCtl;
using eik::kSmallNextRound;
using eik::kSmallStats;
using eik::kSmallStatus;
using eik::Slot;
using eik::SolveParams;

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int hip_fail(hipError_t e) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return EIK_ENOMEM;
    return EIK_EHIP;
}

// Cell sides with kernels: 4, 8 and 16.
bool valid_cell(int cell) { return cell == 4 || cell == 8 || cell == 16; }

bool valid_dims(const int64_t* dims) {
    if (!dims) return false;
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 2) return false;
    const int64_t m = dims[0] * dims[1];
    if (m >= (int64_t(1) << 31)) return false;
    return m * dims[2] < (int64_t(1) << 31);
}

// Cells and array sizes of one grid.
// Mixed precision keeps FP32 copies of the values and faces (u32_bytes, faces32_bytes) for the
// single-precision phase beside the FP64 ones.
struct GridSize {
    int ncx = 0, ncy = 0, ncz = 0;
    int64_t ncell = 0;
    size_t u_bytes = 0, f_bytes = 0, faces_bytes = 0, u32_bytes = 0, faces32_bytes = 0;
    size_t bytes() const {
        return align_up(u_bytes) + align_up(f_bytes) + align_up(faces_bytes) +
               align_up(u32_bytes) + align_up(faces32_bytes);
    }
};

// Storage of a mode: FP32 values for EIK_MODE_FP32, FP64 otherwise (plus FP32 copies if mixed).
bool grid_size(const int64_t dims[3], int cell, int f_dtype, int mode, GridSize* g) {
    const int64_t r = cell;
    g->ncx = (int)((dims[0] + r - 1) / r);
    g->ncy = (int)((dims[1] + r - 1) / r);
    g->ncz = (int)((dims[2] + r - 1) / r);
    g->ncell = (int64_t)g->ncx * g->ncy * g->ncz;
    if (g->ncell * r * r * r >= (int64_t(1) << 31)) return false;
    const size_t n = (size_t)g->ncell, r3 = (size_t)(r * r * r), r2 = (size_t)(r * r);
    const size_t su = mode == EIK_MODE_FP32 ? 4 : 8;
    g->u_bytes = n * r3 * su;
    g->f_bytes = n * r3 * (f_dtype == EIK_F32 ? 4 : 8);
    g->faces_bytes = n * 6 * r2 * su;
    g->u32_bytes = mode == EIK_MODE_MIXED ? n * r3 * 4 : 0;
    g->faces32_bytes = mode == EIK_MODE_MIXED ? n * 6 * r2 * 4 : 0;
    return true;
}

// Shared part of a workspace: control area, slot table, per-slot status and counts, and the
// global per-cell arrays for `cells` cells.
struct CommonLayout {
    size_t off_small = 0, off_slots = 0, off_slot_status = 0, off_counts = 0, off_redo = 0,
           off_key = 0, off_flags = 0, off_list = 0, off_cell_slot = 0, off_keep = 0,
           off_slot_minkey = 0, off_bq = 0, total = 0;
    int nslots = 1;
    int64_t bq_cap = 0;  // entries per bucket ring (0: no buckets)
};

// buckets: room for the bucketed rings of the solve without rounds with a band.
CommonLayout common_layout(int64_t cells, int slots, bool buckets = false) {
    CommonLayout L;
    size_t o = 0;
    const size_t n = (size_t)std::max<int64_t>(cells, 1), ns = (size_t)std::max(slots, 1);
    L.off_small = o; o = align_up(o + eik::kSmallBytes);
    L.off_slots = o; o = align_up(o + ns * sizeof(Slot));
    L.off_slot_status = o; o = align_up(o + ns * sizeof(int));
    L.off_counts = o; o = align_up(o + ns * sizeof(int));
    L.off_redo = o; o = align_up(o + ns * sizeof(int));
    L.off_key = o; o = align_up(o + 2 * n * 8);
    L.off_flags = o; o = align_up(o + 2 * n * 4);
    L.off_list = o; o = align_up(o + (2 * n + (size_t)eik::kRingExtra) * 4);
    L.off_cell_slot = o; o = align_up(o + n * 4);
    L.off_keep = o; o = align_up(o + n * 8);
    L.off_slot_minkey = o; o = align_up(o + 4 * ns * 8);
    if (buckets) {
        L.bq_cap = (int64_t)n + eik::kRingExtra;
        L.off_bq = o;
        o = align_up(o + eik::kBucketCtlBytes + (size_t)eik::kBuckets * (size_t)L.bq_cap * 8);
    }
    L.nslots = (int)ns;
    L.total = o;
    return L;
}

// Fills the launch parameters that point into a workspace.
void bind_common(SolveParams* P, unsigned char* base, const CommonLayout& L, int64_t cells) {
    P->slots = (const Slot*)(base + L.off_slots);
    P->cell_slot = (const int*)(base + L.off_cell_slot);
    P->key_keep = (uint64_t*)(base + L.off_keep);
    P->key[0] = (uint64_t*)(base + L.off_key);
    P->key[1] = P->key[0] + cells;
    P->flags[0] = (uint32_t*)(base + L.off_flags);
    P->flags[1] = P->flags[0] + cells;
    P->list[0] = (int32_t*)(base + L.off_list);
    P->list[1] = P->list[0] + cells;
    P->ctl = (eik::RoundCtl*)(base + L.off_small + kSmallCtl);
    P->seg_cursor = (uint32_t*)(base + L.off_small + eik::kSmallSegCursor);
    P->bar = (uint32_t*)(base + L.off_small + kSmallBar);
    P->status = (int*)(base + L.off_small + kSmallStatus);
    P->stats = (unsigned long long*)(base + L.off_small + kSmallStats);
    P->next_round = (int64_t*)(base + L.off_small + kSmallNextRound);
    P->halted = (uint32_t*)(base + L.off_small + eik::kSmallHalted);
    P->ncells = cells;
    P->async_head = (unsigned long long*)(base + L.off_small + eik::kSmallAsyncHead);
    P->async_tail = (unsigned long long*)(base + L.off_small + eik::kSmallAsyncTail);
    P->async_pending = (unsigned long long*)(base + L.off_small + eik::kSmallAsyncPending);
    P->async_done = (uint32_t*)(base + L.off_small + eik::kSmallAsyncDone);
    P->bq_ctl = L.bq_cap ? (unsigned long long*)(base + L.off_bq) : nullptr;
    P->bq_ring = L.bq_cap ? (int32_t*)(base + L.off_bq + eik::kBucketCtlBytes) : nullptr;
    P->bq_cap = L.bq_cap;
    P->slot_minkey = (uint64_t*)(base + L.off_slot_minkey);
    P->nslots = L.nslots;
}

// Options common to single solves, batches and servers.
int parse_options(const eik_options* options, int cell, eik_options* opt, SolveParams* P) {
    std::memset(opt, 0, sizeof(*opt));
    if (options) *opt = *options;
    if (opt->mode != EIK_MODE_FP64 && opt->mode != EIK_MODE_FP32 && opt->mode != EIK_MODE_MIXED)
        return EIK_EINVAL;
    if (std::isnan(opt->delta) || opt->max_rounds < 0 || opt->max_sweeps < 0 || opt->workers < 0)
        return EIK_EINVAL;
    if (opt->round_log_len < 0 || (opt->round_log_len > 0 && !opt->round_log)) return EIK_EINVAL;
    if (opt->inner < 0 || opt->inner > EIK_INNER_PAIR) return EIK_EINVAL;
    if (opt->cell_value != EIK_CELL_VALUE_NEW && opt->cell_value != EIK_CELL_VALUE_OLD)
        return EIK_EINVAL;
    if (opt->schedule < EIK_SCHED_AUTO || opt->schedule > EIK_SCHED_ASYNC) return EIK_EINVAL;
    std::memset(P, 0, sizeof(*P));
    P->max_rounds = opt->max_rounds > 0 ? opt->max_rounds : (int64_t(1) << 20);
    // default in-cell solver: sweeps at r = 8 and 16, the list relaxation at r = 4 (measured
    // fastest); two sweep streams need both planes in one wave, which r = 16 does not allow
    const int inner = opt->inner ? opt->inner : (cell == 4 ? EIK_INNER_LIST : EIK_INNER_SWEEP);
    if ((inner == EIK_INNER_DUAL || inner == EIK_INNER_PAIR) && cell == 16) return EIK_EINVAL;
    if (inner == EIK_INNER_PAIR && opt->schedule == EIK_SCHED_ASYNC) return EIK_EINVAL;
    // default sweep cap: 8 directional sweeps (one Gray cycle) per visit for the sweeps -- a
    // longer visit publishes what it has and resumes next round, which keeps rounds short --
    // and effectively none for the others (their passes are short)
    P->max_sweeps = opt->max_sweeps > 0 ? opt->max_sweeps : (inner == EIK_INNER_SWEEP ? 8 : 512);
    P->inner = inner == EIK_INNER_SWEEP ? 0
             : inner == EIK_INNER_LIST ? 1
             : inner == EIK_INNER_DUAL ? 2 : 3;
    P->delta = opt->delta > 0.0 ? opt->delta : 0.0;
    P->fp32 = opt->mode == EIK_MODE_FP32 ? 1 : 0;
    P->cell_value = opt->cell_value;
    P->shuffle = opt->shuffle;
    P->watchdog_polls = 1ull << 23;  // several seconds of polling
    P->jitter = opt->jitter;
    P->round_log = opt->round_log;
    P->round_log_len = opt->round_log ? opt->round_log_len : 0;
    return EIK_OK;
}

// The approximation a problem starts from, or nullptr: none given, or no exits (the solution is
// +inf everywhere, which no polish from finite values reaches).
const double* start_values(const eik_problem& pb) {
    return pb.sources.n > 0 ? pb.u_approx : nullptr;
}

// Synchronous validation of one problem (host-side sources are checked here).
int validate_problem(const eik_problem& pb, int f_dtype) {
    if (!valid_dims(pb.dims) || !pb.F || !pb.u_out) return EIK_EINVAL;
    if (!(pb.h > 0.0) || !std::isfinite(pb.h)) return EIK_EINVAL;
    if (!(pb.tol >= 0.0) || !std::isfinite(pb.tol)) return EIK_EINVAL;
    if (f_dtype != EIK_F32 && f_dtype != EIK_F64) return EIK_EINVAL;
    const eik_sources& src = pb.sources;
    if (src.n < 0 || (src.n > 0 && (!src.idx3 || !src.q))) return EIK_EINVAL;
    if (src.n > (int64_t(1) << 24)) return EIK_EINVAL;
    if (!src.on_device) {
        for (int64_t n = 0; n < src.n; ++n) {
            const int64_t* p = src.idx3 + 3 * n;
            for (int a = 0; a < 3; ++a)
                if (p[a] < 0 || p[a] >= pb.dims[a]) return EIK_EINVAL;
            const double qv = src.q[n];
            if (!(qv >= 0.0) || !std::isfinite(qv)) return EIK_EINVAL;
        }
    }
    return EIK_OK;
}

Slot make_slot(const eik_problem& pb, const GridSize& g, int cell_base, unsigned char* mem,
               int* status_dev, int fp32) {
    Slot S;
    std::memset(&S, 0, sizeof(S));
    S.nx = (int)pb.dims[0];
    S.ny = (int)pb.dims[1];
    S.nz = (int)pb.dims[2];
    S.ncx = g.ncx;
    S.ncy = g.ncy;
    S.ncz = g.ncz;
    S.cell_base = cell_base;
    S.ncell = (int)g.ncell;
    S.h = pb.h;
    S.tol = pb.tol;
    S.u = (double*)mem;
    S.f = mem + align_up(g.u_bytes);
    S.faces = (double*)(mem + align_up(g.u_bytes) + align_up(g.f_bytes));
    S.status = status_dev;
    S.fp32 = fp32;
    return S;
}

// The single-precision twin of a mixed-precision slot: same grid, speeds and cells, FP32 values.
Slot fp32_twin(const Slot& S64, const GridSize& g) {
    Slot S = S64;
    unsigned char* mem = (unsigned char*)S64.u;
    S.u = mem + align_up(g.u_bytes) + align_up(g.f_bytes) + align_up(g.faces_bytes);
    S.faces = (unsigned char*)S.u + align_up(g.u32_bytes);
    S.fp32 = 1;
    return S;
}

// Factor that lifts an FP32-accurate result of a problem above its FP64 solution: 1 + the larger
// of 2^-12 (about twenty times the largest relative FP32 error measured on the grids here,
// 1.3e-5) and n 2^-20 with n the longest side (four times the bound 4 n 2^-24 that the FP32
// error is tested against: rounding at each local solve, accumulated along a characteristic of
// at most a few n nodes).  Any larger factor polishes to the same solution.
double lift_factor(const int64_t dims[3]) {
    const double n = (double)std::max(dims[0], std::max(dims[1], dims[2]));
    return 1.0 + std::max(1.0 / 4096.0, n / 1048576.0);
}

// Pinned staging of host-side data (sources, slot tables); one buffer, reused after its last
// copy finished.
struct Staging {
    void* host = nullptr;
    size_t host_bytes = 0;
    void* dev = nullptr;
    size_t dev_bytes = 0;
    hipEvent_t done = nullptr;
    bool recorded = false;

    int reserve(size_t bytes, hipStream_t stream) {
        hipError_t e;
        if (!done && (e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e);
        if (recorded && (e = hipEventSynchronize(done)) != hipSuccess) return hip_fail(e);
        if (host_bytes < bytes) {
            if (host) (void)hipHostFree(host);
            host = nullptr;
            host_bytes = 0;
            if ((e = hipHostMalloc(&host, bytes, hipHostMallocDefault)) != hipSuccess)
                return hip_fail(e);
            host_bytes = bytes;
        }
        if (dev_bytes < bytes) {
            if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e);
            if (dev) (void)hipFree(dev);
            dev = nullptr;
            dev_bytes = 0;
            if ((e = hipMalloc(&dev, bytes)) != hipSuccess) return hip_fail(e);
            dev_bytes = bytes;
        }
        return EIK_OK;
    }
    void release() {
        if (done) {
            if (recorded) (void)hipEventSynchronize(done);
            (void)hipEventDestroy(done);
        }
        if (host) (void)hipHostFree(host);
        if (dev) (void)hipFree(dev);
        *this = Staging();
    }
};

struct SourceRefs {
    const int64_t* idx3;
    const double* q;
};

// Copies `extra` (a slot table) and the host-side sources of a set of problems to the device
// through one pinned buffer; returns device pointers per problem and the table's offset.
int stage_sources(Staging& st, const std::vector<const eik_problem*>& pbs,
                  std::vector<SourceRefs>* refs, const void* extra, size_t extra_bytes,
                  hipStream_t stream) {
    size_t bytes = align_up(extra_bytes);
    for (const eik_problem* pb : pbs)
        if (!pb->sources.on_device) bytes += align_up((size_t)pb->sources.n * 32);
    refs->assign(pbs.size(), SourceRefs{nullptr, nullptr});
    if (bytes == 0) return EIK_OK;
    int rc = st.reserve(bytes, stream);
    if (rc != EIK_OK) return rc;
    unsigned char* h = (unsigned char*)st.host;
    unsigned char* d = (unsigned char*)st.dev;
    size_t o = 0;
    if (extra_bytes) {
        std::memcpy(h, extra, extra_bytes);
        o = align_up(extra_bytes);
    }
    for (size_t i = 0; i < pbs.size(); ++i) {
        const eik_sources& s = pbs[i]->sources;
        if (s.on_device) {
            (*refs)[i] = SourceRefs{s.idx3, s.q};
            continue;
        }
        if (s.n == 0) continue;
        std::memcpy(h + o, s.idx3, (size_t)s.n * 24);
        std::memcpy(h + o + (size_t)s.n * 24, s.q, (size_t)s.n * 8);
        (*refs)[i] = SourceRefs{(const int64_t*)(d + o), (const double*)(d + o + (size_t)s.n * 24)};
        o += align_up((size_t)s.n * 32);
    }
    hipError_t e = hipMemcpyAsync(d, h, o, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e);
    e = hipEventRecord(st.done, stream);
    if (e != hipSuccess) return hip_fail(e);
    st.recorded = true;
    return EIK_OK;
}

// Per device: the event recorded after the most recently enqueued persistent solve kernel.
// Each new solve kernel waits for it, so solve kernels of different streams run one at a time
// (a grid barrier needs its whole launch resident); the other kernels still overlap.
struct DeviceOrder {
    std::mutex mu;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int next = 0;
    bool any = false;
    uint32_t halted_word = 0;  // the halted word, read back by the host-driven loop
};
std::mutex g_mu;
std::map<int, DeviceOrder*> g_order;

DeviceOrder* device_order(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_order.find(dev);
    if (it != g_order.end()) return it->second;
    DeviceOrder* d = new DeviceOrder();
    g_order[dev] = d;
    return d;
}

// Host-driven loop over rounds [P.round_begin, P.round_end): one ordinary launch per round (no
// grid barrier, so no co-residency is needed), enqueued in growing batches; after each batch the
// host waits for the stream and reads the halted word.  Blocks the calling thread.
int host_loop_rounds(DeviceOrder* dord, SolveParams P, int cell, int f_dtype, hipStream_t stream,
                     int workers) {
    hipError_t e;
    if ((e = eik::launch_halt_reset(P, stream)) != hipSuccess) return hip_fail(e);
    const int64_t begin = P.round_begin, end = P.round_end;
    P.single_round = 1;
    int64_t t = begin;
    int batch = 4;
    while (t < end) {
        for (int i = 0; i < batch && t < end; ++i, ++t) {
            P.round_begin = t;
            P.round_end = t + 1;
            P.count_workers = t == begin;
            int used = 0;
            if ((e = eik::launch_solve_rounds(P, cell, f_dtype, stream, workers, &used, 0)) !=
                hipSuccess)
                return hip_fail(e);
        }
        if ((e = hipMemcpyAsync(&dord->halted_word, P.halted, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return hip_fail(e);
        if (dord->halted_word) break;
        batch = std::min(2 * batch, 64);
    }
    if ((e = eik::launch_hostloop_end(P, end, stream)) != hipSuccess) return hip_fail(e);
    return EIK_OK;
}

// Launches the persistent solve kernel for rounds [P.round_begin, P.round_end), ordered after
// every earlier solve kernel of the device.  EIK_SCHED_AUTO falls back to the host-driven loop
// when the runtime refuses the cooperative launch (e.g. another process on the device holds
// one).
int ordered_solve(int dev, const SolveParams& P, int cell, int f_dtype, hipStream_t stream,
                  int workers, int schedule) {
    DeviceOrder* dord = device_order(dev);
    std::lock_guard<std::mutex> lk(dord->mu);
    for (auto& ev : dord->ev) {
        if (!ev) {
            hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(e);
        }
    }
    hipError_t e;
    if (dord->any && (e = hipStreamWaitEvent(stream, dord->ev[dord->next ^ 1], 0)) != hipSuccess)
        return hip_fail(e);
    bool done = false;
    if (schedule == EIK_SCHED_ASYNC) {
        SolveParams Pc = P;
        Pc.single_round = 0;
        Pc.count_workers = 1;
        int used = 0;
        e = eik::launch_solve_async(Pc, cell, f_dtype, stream, workers, &used);
        if (e == hipSuccess) done = true;
        else (void)hipGetLastError();  // refused: the host-driven loop below
    } else if (schedule != EIK_SCHED_HOST_LOOP) {
        SolveParams Pc = P;
        Pc.single_round = 0;
        Pc.count_workers = 1;
        int used = 0;
        e = eik::launch_solve_rounds(Pc, cell, f_dtype, stream, workers, &used, 1);
        if (e == hipSuccess) done = true;
        else if (schedule == EIK_SCHED_COOPERATIVE) return hip_fail(e);
        else (void)hipGetLastError();  // refused: clear the error and take the host loop
    }
    if (!done) {
        int rc = host_loop_rounds(dord, P, cell, f_dtype, stream, workers);
        if (rc != EIK_OK) return rc;
    }
    if ((e = hipEventRecord(dord->ev[dord->next], stream)) != hipSuccess) return hip_fail(e);
    dord->any = true;
    dord->next ^= 1;
    return EIK_OK;
}

// ------------------------------------------------------------------------------------------
// Per-stream workspace of eik_solve / eik_solve_batch.

struct Workspace {
    int device = -1;
    void* base = nullptr;
    size_t bytes = 0;
    Staging staging;
    bool used = false;
    int64_t cells = 0;
    int nslots = 0;
    CommonLayout layout;
    std::mutex mu;  // serialises enqueues that share this workspace
    static constexpr int kRing = 256;
    std::vector<hipEvent_t> ring;  // 4 events per timed solve
    int64_t timed = 0;
    int64_t seq = 0;  // order of the last solve enqueued with this workspace (see g_seq)
    // Cancel word in host memory mapped into the device (eik_cancel): solve k of this
    // workspace stops once the word is >= k.  eik_cancel reads these without the workspace's
    // mutex, which a host-driven solve holds for its whole duration.
    std::atomic<uint32_t*> cancel_host{nullptr};
    uint32_t* cancel_dev = nullptr;
    std::atomic<uint32_t> cancel_seq{0};
};

// Sequence number of solves enqueued by the process: tells which of a stream's workspace solve
// and allocation-free solve came last.
std::atomic<int64_t> g_seq{0};

std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

Workspace* get_workspace(hipStream_t stream, int* rc) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { *rc = hip_fail(e); return nullptr; }
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) return it->second;
    Workspace* w = new Workspace();
    w->device = dev;
    g_ws[key] = w;
    return w;
}

Workspace* find_workspace(hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find(std::make_pair(dev, stream));
    return it == g_ws.end() ? nullptr : it->second;
}

int ensure_device(void** p, size_t* have, size_t need, hipStream_t stream) {
    if (*have >= need && *p) return EIK_OK;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e);
    if (*p) { (void)hipFree(*p); *p = nullptr; *have = 0; }
    e = hipMalloc(p, need);
    if (e != hipSuccess) { *p = nullptr; return hip_fail(e); }
    *have = need;
    return EIK_OK;
}

// The kernel sequence of a solve of n problems whose workspace (common part at `base`, layout L,
// grids' arrays where `slots` point) and device slot table are in place; refs holds each
// problem's exits as device pointers.  ev: 4 events to record (or null).
int enqueue_solve(int device, int n, const eik_problem* pbs, int f_dtype, int cell,
                  const eik_options& opt, SolveParams P, const Slot* slots,
                  const SourceRefs* refs, unsigned char* base, const CommonLayout& L,
                  int64_t nsrc_total, hipEvent_t* ev, hipStream_t stream) {
    hipError_t e;
    int rc;
    const bool mixed = opt.mode == EIK_MODE_MIXED;
    bool polish = false;  // some problem starts from a given approximation
    for (int i = 0; i < n; ++i) polish = polish || start_values(pbs[i]) != nullptr;
    // Mixed precision runs the method twice: in FP32 on the twins, then in FP64 from the FP32
    // result lifted above the FP64 solution, with the exits re-seeded at their exact values.  A
    // given approximation is polished the same way.  Nothing else is queued: the exact exit
    // values decrease the cells around them, whose changed faces tag their downwind neighbours,
    // so the polish reaches every cell whose boundary changes, in the order of a solve from
    // +inf, and visits no other.
    SolveParams P1 = P;
    const Slot* first = slots;
    if (mixed) {
        P1.fp32 = 1;
        P1.slots = P.slots + n;
        first = slots + n;
    }
    if (ev && (e = hipEventRecord(ev[0], stream)) != hipSuccess) return hip_fail(e);
    if ((e = eik::launch_init_global(P, stream)) != hipSuccess) return hip_fail(e);
    for (int i = 0; i < n; ++i) {
        const double* u0 = start_values(pbs[i]);
        e = eik::launch_init_slot(P1, first[i], i, cell, f_dtype, pbs[i].F, u0,
                                  lift_factor(pbs[i].dims), stream);
        if (e != hipSuccess) return hip_fail(e);
        e = eik::launch_seed(P1, first[i], cell, f_dtype, 0, pbs[i].sources.n, refs[i].idx3,
                             refs[i].q, stream, nullptr, u0 != nullptr);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (ev && (e = hipEventRecord(ev[1], stream)) != hipSuccess) return hip_fail(e);
    if (nsrc_total > 0) {
        P1.round_begin = 0;
        P1.round_end = P1.max_rounds;
        rc = ordered_solve(device, P1, cell, f_dtype, stream, opt.workers, opt.schedule);
        if (rc != EIK_OK) return rc;
        if (mixed) {
            if ((e = eik::launch_reset_rounds(P, stream)) != hipSuccess) return hip_fail(e);
            for (int i = 0; i < n; ++i) {
                if ((e = eik::launch_lift(first[i], slots[i], cell, lift_factor(pbs[i].dims),
                                          stream)) !=
                        hipSuccess ||
                    (e = eik::launch_seed(P, slots[i], cell, f_dtype, 0, pbs[i].sources.n,
                                          refs[i].idx3, refs[i].q, stream, nullptr, true)) !=
                        hipSuccess)
                    return hip_fail(e);
            }
            P.round_begin = 0;
            P.round_end = P.max_rounds;
            rc = ordered_solve(device, P, cell, f_dtype, stream, opt.workers, opt.schedule);
            if (rc != EIK_OK) return rc;
        }
    }
    if (ev && (e = hipEventRecord(ev[2], stream)) != hipSuccess) return hip_fail(e);
    for (int i = 0; i < n; ++i)
        if ((e = eik::launch_output(slots[i], cell, pbs[i].u_out, stream)) != hipSuccess)
            return hip_fail(e);
    // A polished result (mixed precision, or a given approximation) is checked against eq. (2)
    // at every node; a grid that fails (its start lay below the solution somewhere) is solved
    // again from +inf in FP64.  Everything stays on the stream: the re-solve's kernels do
    // nothing for grids that passed, and its solve launch finds an empty list if all did.
    if ((mixed || polish) && nsrc_total > 0) {
        int* redo = (int*)(base + L.off_redo);
        if ((e = eik::launch_clear_ints(redo, n, stream)) != hipSuccess) return hip_fail(e);
        for (int i = 0; i < n; ++i) {
            if (!mixed && !start_values(pbs[i])) continue;
            if ((e = eik::launch_polish_check(slots[i], cell, f_dtype, pbs[i].u_out, redo + i,
                                              P.stats, stream)) != hipSuccess)
                return hip_fail(e);
        }
        if ((e = eik::launch_reset_rounds(P, stream)) != hipSuccess) return hip_fail(e);
        for (int i = 0; i < n; ++i) {
            if (!mixed && !start_values(pbs[i])) continue;
            if ((e = eik::launch_restart_slot(P, slots[i], i, cell, f_dtype, 0, stream,
                                              redo + i)) != hipSuccess)
                return hip_fail(e);
        }
        P.round_begin = 0;
        P.round_end = P.max_rounds;
        rc = ordered_solve(device, P, cell, f_dtype, stream, opt.workers, opt.schedule);
        if (rc != EIK_OK) return rc;
        for (int i = 0; i < n; ++i) {
            if (!mixed && !start_values(pbs[i])) continue;
            if ((e = eik::launch_output(slots[i], cell, pbs[i].u_out, stream, redo + i)) !=
                hipSuccess)
                return hip_fail(e);
        }
    }
    if (ev && (e = hipEventRecord(ev[3], stream)) != hipSuccess) return hip_fail(e);
    return EIK_OK;
}

int solve_batch_impl(int n, const eik_problem* pbs, int f_dtype, int cell, hipStream_t stream,
                     const eik_options* options) {
    if (n < 1 || n > (1 << 20) || !pbs) return EIK_EINVAL;
    if (!valid_cell(cell)) return EIK_EINVAL;
    eik_options opt;
    SolveParams P;
    int rc = parse_options(options, cell, &opt, &P);
    if (rc != EIK_OK) return rc;
    std::vector<GridSize> gs((size_t)n);
    int64_t cells = 0;
    size_t grid_bytes = 0;
    int64_t nsrc_total = 0;
    for (int i = 0; i < n; ++i) {
        if ((rc = validate_problem(pbs[i], f_dtype)) != EIK_OK) return rc;
        if (!grid_size(pbs[i].dims, cell, f_dtype, opt.mode, &gs[i])) return EIK_EINVAL;
        cells += gs[i].ncell;
        grid_bytes += gs[i].bytes();
        nsrc_total += pbs[i].sources.n;
    }
    if (cells >= (int64_t(1) << 31)) return EIK_EINVAL;
    const bool mixed = opt.mode == EIK_MODE_MIXED;
    bool polish = false;  // some problem starts from a given approximation
    for (int i = 0; i < n; ++i) polish = polish || start_values(pbs[i]) != nullptr;
    if (polish && mixed) return EIK_EINVAL;
    const int ntab = mixed ? 2 * n : n;  // slot table entries (FP64 slots, then FP32 twins)
    const CommonLayout L =
        common_layout(cells, ntab, opt.schedule == EIK_SCHED_ASYNC && opt.delta > 0.0);

    Workspace* w = get_workspace(stream, &rc);
    if (!w) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    rc = ensure_device(&w->base, &w->bytes, L.total + grid_bytes, stream);
    if (rc != EIK_OK) return rc;
    if (!w->cancel_host.load()) {
        uint32_t* hostw = nullptr;
        hipError_t ec = hipHostMalloc((void**)&hostw, 64,
                                      hipHostMallocMapped | hipHostMallocCoherent);
        if (ec == hipSuccess) ec = hipHostGetDevicePointer((void**)&w->cancel_dev, hostw, 0);
        if (ec != hipSuccess) {
            if (hostw) (void)hipHostFree(hostw);
            return hip_fail(ec);
        }
        __atomic_store_n(hostw, 0u, __ATOMIC_SEQ_CST);
        w->cancel_host.store(hostw);
    }
    unsigned char* base = (unsigned char*)w->base;
    bind_common(&P, base, L, cells);
    P.cancel = w->cancel_dev;
    P.cancel_seq = ++w->cancel_seq;
    P.slot_band = n > 1;  // a band per grid: the grids of a batch advance side by side
    int* slot_status = (int*)(base + L.off_slot_status);

    // Slot table, built on the host and copied with the sources through one pinned buffer.
    std::vector<Slot> slots((size_t)ntab);
    size_t off = L.total;
    int64_t cell_base = 0;
    for (int i = 0; i < n; ++i) {
        slots[i] = make_slot(pbs[i], gs[i], (int)cell_base, base + off, slot_status + i, P.fp32);
        if (mixed) slots[(size_t)n + i] = fp32_twin(slots[i], gs[i]);
        off += gs[i].bytes();
        cell_base += gs[i].ncell;
    }
    std::vector<const eik_problem*> ptrs((size_t)n);
    for (int i = 0; i < n; ++i) ptrs[i] = &pbs[i];
    std::vector<SourceRefs> refs;
    rc = stage_sources(w->staging, ptrs, &refs, slots.data(), slots.size() * sizeof(Slot), stream);
    if (rc != EIK_OK) return rc;
    hipError_t e = hipMemcpyAsync(base + L.off_slots, w->staging.dev, slots.size() * sizeof(Slot),
                                  hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip_fail(e);

    hipEvent_t* ev = nullptr;
    if (opt.timing) {
        if (w->ring.empty()) {
            w->ring.assign(4 * Workspace::kRing, nullptr);
            for (auto& x : w->ring)
                if ((e = hipEventCreate(&x)) != hipSuccess) return hip_fail(e);
        }
        ev = &w->ring[4 * (w->timed % Workspace::kRing)];
        w->timed++;
    }
    rc = enqueue_solve(w->device, n, pbs, f_dtype, cell, opt, P, slots.data(), refs.data(), base,
                       L, nsrc_total, ev, stream);
    if (rc != EIK_OK) return rc;
    w->seq = ++g_seq;
    w->used = true;
    w->cells = cells;
    w->nslots = n;
    w->layout = L;
    return EIK_OK;
}

// ------------------------------------------------------------------------------------------
// Allocation-free solves (eik_solve_noalloc): the whole workspace of one solve lives in a static
// device array.  Each device that runs one holds its own copy of the array until the process
// ends; host code reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name in host code is a host-side stand-in).

constexpr int kMaxDevices = 64;

struct NoallocDevice {
    bool ready = false;
    unsigned char* ptr = nullptr;  // this device's copy of the scratch array
    std::mutex mu;                 // serialises the enqueues of allocation-free solves
    // the last allocation-free solve enqueued on the device (for eik_stream_status)
    hipStream_t stream = nullptr;
    bool used = false;
    int64_t seq = 0, cells = 0;
    CommonLayout layout;
};
std::mutex g_noalloc_mu;
NoallocDevice g_noalloc[kMaxDevices];

// Where the last solve enqueued on a stream keeps its status and counters: the stream's
// workspace, or this device's scratch if an allocation-free solve on that stream came later.
struct LastSolve {
    unsigned char* base = nullptr;
    CommonLayout layout;
    int nslots = 0;
    int64_t cells = 0;
};

bool last_solve(hipStream_t stream, LastSolve* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    Workspace* w = find_workspace(stream);
    int64_t wseq = -1;
    if (w) {
        std::lock_guard<std::mutex> lk(w->mu);
        if (w->used) {
            wseq = w->seq;
            out->base = (unsigned char*)w->base;
            out->layout = w->layout;
            out->nslots = w->nslots;
            out->cells = w->cells;
        }
    }
    if (dev >= 0 && dev < kMaxDevices) {
        NoallocDevice& d = g_noalloc[dev];
        std::lock_guard<std::mutex> lk(d.mu);
        if (d.ready && d.used && d.stream == stream && d.seq > wseq) {
            out->base = d.ptr;
            out->layout = d.layout;
            out->nslots = 1;
            out->cells = d.cells;
            return true;
        }
    }
    return wseq >= 0;
}

// One-time set-up of allocation-free solves on device `dev` (current): the address of this
// device's scratch array, and the events that order solve kernels on the device.
int noalloc_setup(int dev, NoallocDevice** out) {
    if (dev < 0 || dev >= kMaxDevices) return EIK_EINVAL;
    NoallocDevice& d = g_noalloc[dev];
    DeviceOrder* o = device_order(dev);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!d.ready) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return e != hipSuccess ? hip_fail(e) : EIK_EHIP;
        std::lock_guard<std::mutex> lo(o->mu);
        for (auto& ev : o->ev)
            if (!ev && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e);
        d.ptr = (unsigned char*)p;
        d.ready = true;
    }
    *out = &d;
    return EIK_OK;
}

template <typename T>
bool range_alloc(std::vector<std::pair<T, T>>& fl, T size, T align, T* out) {
    for (size_t i = 0; i < fl.size(); ++i) {
        const T start = (fl[i].first + align - 1) / align * align;
        const T end = fl[i].first + fl[i].second;
        if (start + size <= end) {
            const T pre = start - fl[i].first, post = end - (start + size);
            const T f0 = fl[i].first;
            fl.erase(fl.begin() + (long)i);
            if (post) fl.insert(fl.begin() + (long)i, {start + size, post});
            if (pre) fl.insert(fl.begin() + (long)i, {f0, pre});
            *out = start;
            return true;
        }
    }
    return false;
}

template <typename T>
void range_free(std::vector<std::pair<T, T>>& fl, T off, T size) {
    fl.push_back({off, size});
    std::sort(fl.begin(), fl.end());
    std::vector<std::pair<T, T>> merged;
    for (auto& r : fl) {
        if (!merged.empty() && merged.back().first + merged.back().second == r.first)
            merged.back().second += r.second;
        else
            merged.push_back(r);
    }
    fl.swap(merged);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Server state.

struct eik_server {
    int device = -1;
    hipStream_t stream = nullptr;
    int cell = 8, f_dtype = EIK_F32;
    eik_options opt;
    SolveParams P;
    CommonLayout layout;
    void* base = nullptr;  // common part
    void* pool = nullptr;  // grids' arrays
    size_t pool_bytes = 0;
    int64_t max_cells = 0;
    int max_problems = 0;
    Staging staging;
    struct Problem {
        int64_t ticket = -1;
        bool active = false;   // admitted and not yet retired
        bool started = false;  // seeded into a round
        eik_problem pb;
        GridSize g;
        Slot slot;
        size_t pool_off = 0;
        bool redone = false;   // restarted from +inf after its polish failed the check
    };
    std::vector<Problem> problems;                       // indexed by slot
    std::vector<std::pair<size_t, size_t>> free_pool;    // (offset, size), sorted
    std::vector<std::pair<int64_t, int64_t>> free_cells;
    std::vector<int> fresh;                              // slots admitted since the last step
    std::vector<std::pair<int64_t, int>> finished;       // (ticket, status) not yet polled
    int64_t next_ticket = 0;
    int64_t next_round = 0;
    int* host_words = nullptr;  // pinned: counts, statuses, next round, launch status
    size_t pool_used = 0;
    int64_t cells_used = 0;
    int64_t polish_redone = 0;
};

extern "C" {

const char* eik_strerror(int code) {
    switch (code) {
        case EIK_OK: return "EIK_OK";
        case EIK_EINVAL: return "EIK_EINVAL: invalid argument";
        case EIK_ENOMEM: return "EIK_ENOMEM: out of memory";
        case EIK_EHIP: return "EIK_EHIP: HIP runtime error";
        case EIK_ENOCONV: return "EIK_ENOCONV: round cap reached before convergence";
        case EIK_ECANCELLED: return "EIK_ECANCELLED: stopped by the device watchdog";
        case EIK_EBUSY: return "EIK_EBUSY: no room on the device now";
        case EIK_ETOOBIG:
            return "EIK_ETOOBIG: the problem's workspace exceeds the 384 MiB static scratch of "
                   "eik_solve_noalloc";
        default: return "EIK: unknown status";
    }
}

const char* eik_version(void) { return "eik-mi355x 0.2 (gfx950)"; }

int eik_problem_bytes(const int64_t dims[3], int cell, int f_dtype, int mode, size_t* bytes) {
    if (!bytes || !valid_dims(dims) || !valid_cell(cell) ||
        (f_dtype != EIK_F32 && f_dtype != EIK_F64) ||
        (mode != EIK_MODE_FP64 && mode != EIK_MODE_FP32 && mode != EIK_MODE_MIXED))
        return EIK_EINVAL;
    GridSize g;
    if (!grid_size(dims, cell, f_dtype, mode, &g)) return EIK_EINVAL;
    *bytes = g.bytes();
    return EIK_OK;
}

int eik_query_workspace(const int64_t dims[3], int cell, int f_dtype, int mode, size_t* bytes) {
    size_t grid = 0;
    int rc = eik_problem_bytes(dims, cell, f_dtype, mode, &grid);
    if (rc != EIK_OK) return rc;
    GridSize g;
    grid_size(dims, cell, f_dtype, mode, &g);
    *bytes = common_layout(g.ncell, mode == EIK_MODE_MIXED ? 2 : 1).total + grid;
    return EIK_OK;
}

int eik_solve_ex(const int64_t dims[3], double h, const void* F, int f_dtype,
                 const eik_sources* sources, double* u_out, int cell, double tol,
                 hipStream_t stream, const eik_options* options) {
    if (!dims || !sources) return EIK_EINVAL;
    eik_problem pb;
    std::memset(&pb, 0, sizeof(pb));
    for (int a = 0; a < 3; ++a) pb.dims[a] = dims[a];
    pb.h = h;
    pb.F = F;
    pb.sources = *sources;
    pb.u_out = u_out;
    pb.tol = tol;
    return solve_batch_impl(1, &pb, f_dtype, cell, stream, options);
}

int eik_solve(const int64_t dims[3], double h, const void* F, int f_dtype,
              const eik_sources* sources, double* u_out, int cell, double tol,
              hipStream_t stream) {
    return eik_solve_ex(dims, h, F, f_dtype, sources, u_out, cell, tol, stream, nullptr);
}

int eik_solve_batch(int n, const eik_problem* problems, int f_dtype, int cell, hipStream_t stream,
                    const eik_options* options) {
    return solve_batch_impl(n, problems, f_dtype, cell, stream, options);
}

int eik_solve_noalloc(const int64_t dims[3], double h, const void* F, int f_dtype,
                      const eik_sources* sources, double* u_out, int cell, double tol,
                      hipStream_t stream, const eik_options* options) {
    if (!dims || !sources || !valid_cell(cell)) return EIK_EINVAL;
    eik_problem pb;
    std::memset(&pb, 0, sizeof(pb));
    for (int a = 0; a < 3; ++a) pb.dims[a] = dims[a];
    pb.h = h;
    pb.F = F;
    pb.sources = *sources;
    pb.u_out = u_out;
    pb.tol = tol;
    eik_options opt;
    SolveParams P;
    int rc = parse_options(options, cell, &opt, &P);
    if (rc != EIK_OK) return rc;
    if (opt.timing) return EIK_EINVAL;  // timing would create events
    if ((rc = validate_problem(pb, f_dtype)) != EIK_OK) return rc;
    if (!sources->on_device && sources->n > eik::kHostExitsMax) return EIK_EINVAL;
    GridSize g;
    if (!grid_size(dims, cell, f_dtype, opt.mode, &g)) return EIK_EINVAL;
    const bool mixed = opt.mode == EIK_MODE_MIXED;
    const int ntab = mixed ? 2 : 1;
    const CommonLayout L =
        common_layout(g.ncell, ntab, opt.schedule == EIK_SCHED_ASYNC && opt.delta > 0.0);
    const size_t exits_off = L.total + g.bytes();
    const size_t need = exits_off + (sources->on_device ? 0 : align_up(eik::kHostExitsMax * 32));
    if (need > kScratchBytes) return EIK_ETOOBIG;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    NoallocDevice* d = nullptr;
    if ((rc = noalloc_setup(dev, &d)) != EIK_OK) return rc;
    std::lock_guard<std::mutex> lk(d->mu);
    unsigned char* base = d->ptr;
    bind_common(&P, base, L, g.ncell);
    int* slot_status = (int*)(base + L.off_slot_status);
    Slot slots[2];
    slots[0] = make_slot(pb, g, 0, base + L.total, slot_status, P.fp32);
    slots[1] = mixed ? fp32_twin(slots[0], g) : slots[0];
    if ((e = eik::launch_put_slots(slots[0], slots[1], ntab, (Slot*)(base + L.off_slots),
                                   stream)) != hipSuccess)
        return hip_fail(e);
    SourceRefs ref{sources->idx3, sources->q};
    if (!sources->on_device && sources->n > 0) {
        int64_t* di = (int64_t*)(base + exits_off);
        double* dq = (double*)(base + exits_off + eik::kHostExitsMax * 24);
        if ((e = eik::launch_put_exits(sources->idx3, sources->q, (int)sources->n, di, dq,
                                       stream)) != hipSuccess)
            return hip_fail(e);
        ref = SourceRefs{di, dq};
    }
    rc = enqueue_solve(dev, 1, &pb, f_dtype, cell, opt, P, slots, &ref, base, L, sources->n,
                       nullptr, stream);
    if (rc != EIK_OK) return rc;
    d->stream = stream;
    d->used = true;
    d->cells = g.ncell;
    d->layout = L;
    d->seq = ++g_seq;
    return EIK_OK;
}

int eik_autotune(const int64_t dims[3], double h, const void* F, int f_dtype,
                 const eik_sources* sources, double* u_out, double tol, hipStream_t stream,
                 int reps, eik_tune_entry* table, int cap, int* n_out, eik_tune_entry* best) {
    if (!best || reps < 1 || reps > 100 || cap < 0 || (cap > 0 && !table)) return EIK_EINVAL;
    int rc = EIK_OK;
    // Synchronous validation of the problem once (every cell size accepts the same problems).
    {
        eik_problem pb;
        std::memset(&pb, 0, sizeof(pb));
        if (!dims || !sources) return EIK_EINVAL;
        for (int a = 0; a < 3; ++a) pb.dims[a] = dims[a];
        pb.h = h;
        pb.F = F;
        pb.sources = *sources;
        pb.u_out = u_out;
        pb.tol = tol;
        if ((rc = validate_problem(pb, f_dtype)) != EIK_OK) return rc;
    }
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e);
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (auto& x : ev)
        if ((e = hipEventCreate(&x)) != hipSuccess) return hip_fail(e);
    std::vector<eik_tune_entry> cand;
    const int cells[3] = {8, 4, 16};
    const int inners[4] = {EIK_INNER_SWEEP, EIK_INNER_LIST, EIK_INNER_DUAL, EIK_INNER_PAIR};
    for (int cell : cells)
        for (int inner : inners)
            for (int workers : {0, ncu / 2}) {
                if ((inner == EIK_INNER_DUAL || inner == EIK_INNER_PAIR) && cell == 16) continue;
                eik_tune_entry t;
                std::memset(&t, 0, sizeof(t));
                t.cell = cell;
                t.inner = inner;
                t.workers = workers;
                t.delta = 0.0;
                cand.push_back(t);
            }
    auto run = [&](eik_tune_entry& t) -> int {
        eik_options o;
        std::memset(&o, 0, sizeof(o));
        o.inner = t.inner;
        o.workers = t.workers;
        o.delta = t.delta;
        t.ms = INFINITY;
        for (int k = 0; k <= reps; ++k) {  // run 0 warms up
            hipError_t ee = hipEventRecord(ev[0], stream);
            if (ee != hipSuccess) return hip_fail(ee);
            int r = eik_solve_ex(dims, h, F, f_dtype, sources, u_out, t.cell, tol, stream, &o);
            if (r != EIK_OK) return r;
            if ((ee = hipEventRecord(ev[1], stream)) != hipSuccess) return hip_fail(ee);
            const int st = eik_stream_status(stream, nullptr);
            t.status = st;
            if (st != EIK_OK) return EIK_OK;  // recorded; this candidate is not eligible
            float ms = 0.f;
            if ((ee = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) return hip_fail(ee);
            if (k > 0 && ms < t.ms) t.ms = ms;
        }
        return EIK_OK;
    };
    int ibest = -1;
    for (size_t i = 0; i < cand.size() && rc == EIK_OK; ++i) {
        rc = run(cand[i]);
        if (rc == EIK_OK && cand[i].status == EIK_OK &&
            (ibest < 0 || cand[i].ms < cand[(size_t)ibest].ms))
            ibest = (int)i;
    }
    // Priority bands around the best configuration: widths of 4, 16 and 64 cell crossings (r h).
    if (rc == EIK_OK && ibest >= 0) {
        const eik_tune_entry b = cand[(size_t)ibest];
        for (double m : {4.0, 16.0, 64.0}) {
            eik_tune_entry t = b;
            t.delta = m * b.cell * h;
            rc = run(t);
            if (rc != EIK_OK) break;
            cand.push_back(t);
            if (t.status == EIK_OK && t.ms < cand[(size_t)ibest].ms) ibest = (int)cand.size() - 1;
        }
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (rc != EIK_OK) return rc;
    if (ibest < 0) return EIK_ECANCELLED;
    *best = cand[(size_t)ibest];
    const int n = std::min<int>(cap, (int)cand.size());
    for (int i = 0; i < n; ++i) table[i] = cand[(size_t)i];
    if (n_out) *n_out = n;
    return EIK_OK;
}

int eik_stream_status(hipStream_t stream, eik_stats* stats) {
    LastSolve ls;
    if (!last_solve(stream, &ls)) return EIK_EINVAL;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e);
    unsigned char* base = ls.base;
    int status = 0;
    unsigned long long st[eik::ST_TOTAL];
    e = hipMemcpy(&status, base + ls.layout.off_small + kSmallStatus, sizeof(int),
                  hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    e = hipMemcpy(st, base + ls.layout.off_small + kSmallStats, sizeof(st), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    if (status == 0) {
        // otherwise the first failing grid's status
        std::vector<int> ss((size_t)ls.nslots);
        e = hipMemcpy(ss.data(), base + ls.layout.off_slot_status, ss.size() * sizeof(int),
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e);
        for (int v : ss)
            if (v != 0) { status = v; break; }
    }
    if (stats) {
        stats->rounds = (int64_t)st[eik::ST_ROUNDS];
        stats->visits = (int64_t)st[eik::ST_VISITS];
        stats->sweeps = (int64_t)st[eik::ST_SWEEPS];
        stats->updates = (int64_t)st[eik::ST_UPDATES];
        stats->deferred = (int64_t)st[eik::ST_DEFERRED];
        stats->requeued = (int64_t)st[eik::ST_REQUEUED];
        stats->cells = ls.cells;
        stats->status = status;
        stats->workers = (int64_t)st[eik::ST_WORKERS];
        stats->cycles_pop = (int64_t)st[eik::ST_CYC_POP];
        stats->cycles_stage = (int64_t)st[eik::ST_CYC_STAGE];
        stats->cycles_sweep = (int64_t)st[eik::ST_CYC_SWEEP];
        stats->cycles_write = (int64_t)st[eik::ST_CYC_WRITE];
        stats->cycles_wait = (int64_t)st[eik::ST_CYC_WAIT];
        stats->polish_redone = (int64_t)st[eik::ST_REDONE];
        for (int i = 0; i < 32; ++i) {
            stats->sweep_hist[i] = (int64_t)st[eik::ST_HIST_SWEEPS + i];
            stats->visit_cycles_log2_hist[i] = (int64_t)st[eik::ST_HIST_CYCLES + i];
        }
    }
    return status;
}

int eik_batch_status(hipStream_t stream, int n, int* status) {
    LastSolve ls;
    if (!last_solve(stream, &ls) || n < 0 || (n > 0 && !status)) return EIK_EINVAL;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e);
    int launch = 0;
    unsigned char* base = ls.base;
    e = hipMemcpy(&launch, base + ls.layout.off_small + kSmallStatus, sizeof(int),
                  hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    n = std::min(n, ls.nslots);
    e = hipMemcpy(status, base + ls.layout.off_slot_status, (size_t)n * sizeof(int),
                  hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    for (int i = 0; i < n; ++i)
        if (status[i] == 0) status[i] = launch;
    return n;
}

int eik_cancel(hipStream_t stream) {
    Workspace* w = find_workspace(stream);
    if (!w) return EIK_EINVAL;
    uint32_t* word = w->cancel_host.load();
    if (!word) return EIK_EINVAL;
    __atomic_store_n(word, w->cancel_seq.load(), __ATOMIC_SEQ_CST);
    return EIK_OK;
}

int eik_kernel_times(hipStream_t stream, int n, double* solve_ms, double* total_ms) {
    if (n < 0) return EIK_EINVAL;
    Workspace* w = find_workspace(stream);
    if (!w || w->timed == 0) return 0;
    std::lock_guard<std::mutex> lk(w->mu);
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e);
    const int64_t have = std::min<int64_t>(w->timed, Workspace::kRing);
    if (n > have) n = (int)have;
    for (int i = 0; i < n; ++i) {
        const int64_t k = w->timed - n + i;
        hipEvent_t* q4 = &w->ring[4 * (k % Workspace::kRing)];
        float a = 0.f, b = 0.f;
        if ((e = hipEventElapsedTime(&a, q4[1], q4[2])) != hipSuccess) return hip_fail(e);
        if ((e = hipEventElapsedTime(&b, q4[0], q4[3])) != hipSuccess) return hip_fail(e);
        if (solve_ms) solve_ms[i] = a;
        if (total_ms) total_ms[i] = b;
    }
    return n;
}

void eik_release(void) {
    // Allocation-free solves run their set-up again after this (their ordering events are
    // freed below); the scratch arrays themselves stay until the process ends.
    {
        std::lock_guard<std::mutex> ln(g_noalloc_mu);
        for (auto& d : g_noalloc) {
            std::lock_guard<std::mutex> ld(d.mu);
            d.ready = false;
            d.used = false;
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    // Wait for each device that holds library state (not for the streams themselves: a
    // caller may already have destroyed a stream it solved on).
    std::vector<int> devs;
    for (auto& kv : g_ws) devs.push_back(kv.second->device);
    for (auto& kv : g_order) devs.push_back(kv.first);
    std::sort(devs.begin(), devs.end());
    devs.erase(std::unique(devs.begin(), devs.end()), devs.end());
    for (int d : devs)
        if (hipSetDevice(d) == hipSuccess) (void)hipDeviceSynchronize();
    for (auto& kv : g_ws) {
        Workspace* w = kv.second;
        (void)hipSetDevice(w->device);
        w->staging.release();
        if (w->base) (void)hipFree(w->base);
        if (w->cancel_host.load()) (void)hipHostFree(w->cancel_host.load());
        for (auto& x : w->ring)
            if (x) (void)hipEventDestroy(x);
        delete w;
    }
    g_ws.clear();
    // The events that order solve kernels across streams of a device.
    for (auto& kv : g_order) {
        DeviceOrder* d = kv.second;
        (void)hipSetDevice(kv.first);
        for (auto& ev : d->ev)
            if (ev) (void)hipEventDestroy(ev);
        delete d;
    }
    g_order.clear();
    (void)hipSetDevice(cur);
}

// ---------------------------------- server ------------------------------------------------

int eik_server_create(eik_server** out, size_t pool_bytes, int64_t max_cells, int max_problems,
                      int cell, int f_dtype, hipStream_t stream, const eik_options* options) {
    if (!out || pool_bytes == 0 || max_cells < 1 || max_cells >= (int64_t(1) << 31) ||
        max_problems < 1 || max_problems > (1 << 16) || !valid_cell(cell) ||
        (f_dtype != EIK_F32 && f_dtype != EIK_F64))
        return EIK_EINVAL;
    eik_server* s = new eik_server();
    int rc = parse_options(options, cell, &s->opt, &s->P);
    if (rc == EIK_OK && s->opt.mode == EIK_MODE_MIXED) rc = EIK_EINVAL;  // one precision per server
    if (rc == EIK_OK && s->opt.schedule == EIK_SCHED_ASYNC) rc = EIK_EINVAL;  // steps are rounds
    if (rc != EIK_OK) { delete s; return rc; }
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) { delete s; return hip_fail(e); }
    s->stream = stream;
    s->cell = cell;
    s->f_dtype = f_dtype;
    s->max_cells = max_cells;
    s->max_problems = max_problems;
    s->pool_bytes = pool_bytes;
    s->layout = common_layout(max_cells, max_problems);
    // counts [0, n), statuses [n, 2n), next round and launch status [2n, 2n + 8), redo words
    // [2n + 8, 3n + 8)
    const size_t hb = ((size_t)max_problems * 3 + 8) * sizeof(int) + 64;
    if ((e = hipMalloc(&s->base, s->layout.total)) != hipSuccess ||
        (e = hipMalloc(&s->pool, pool_bytes)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s->host_words, hb, hipHostMallocDefault)) != hipSuccess) {
        eik_server_destroy(s);
        return hip_fail(e);
    }
    bind_common(&s->P, (unsigned char*)s->base, s->layout, max_cells);
    // A band per problem, so that problems admitted later (values near their exits) do not
    // hold back the ones whose fronts are further on.
    s->P.slot_band = max_problems > 1;
    s->problems.resize((size_t)max_problems);
    s->free_pool.push_back({0, pool_bytes});
    s->free_cells.push_back({0, max_cells});
    if ((e = eik::launch_init_global(s->P, stream)) != hipSuccess) {
        eik_server_destroy(s);
        return hip_fail(e);
    }
    *out = s;
    return EIK_OK;
}

int eik_server_submit(eik_server* s, const eik_problem* pb, int64_t* ticket) {
    if (!s || !pb || !ticket) return EIK_EINVAL;
    int rc = validate_problem(*pb, s->f_dtype);
    if (rc != EIK_OK) return rc;
    GridSize g;
    if (!grid_size(pb->dims, s->cell, s->f_dtype, s->opt.mode, &g)) return EIK_EINVAL;
    if (g.ncell > s->max_cells || g.bytes() > s->pool_bytes) return EIK_EINVAL;  // never fits
    int slot = -1;
    for (int i = 0; i < s->max_problems; ++i)
        if (!s->problems[i].active) { slot = i; break; }
    if (slot < 0) return EIK_EBUSY;
    size_t poff = 0;
    int64_t cbase = 0;
    if (!range_alloc<size_t>(s->free_pool, g.bytes(), kAlign, &poff)) return EIK_EBUSY;
    if (!range_alloc<int64_t>(s->free_cells, g.ncell, 1, &cbase)) {
        range_free<size_t>(s->free_pool, poff, g.bytes());
        return EIK_EBUSY;
    }
    eik_server::Problem& p = s->problems[slot];
    p.ticket = s->next_ticket++;
    p.active = true;
    p.started = false;
    p.pb = *pb;
    p.g = g;
    p.pool_off = poff;
    int* slot_status = (int*)((unsigned char*)s->base + s->layout.off_slot_status) + slot;
    p.slot = make_slot(*pb, g, (int)cbase, (unsigned char*)s->pool + poff, slot_status, s->P.fp32);
    s->fresh.push_back(slot);
    s->pool_used += g.bytes();
    s->cells_used += g.ncell;
    *ticket = p.ticket;
    return EIK_OK;
}

int eik_server_step(eik_server* s, int64_t rounds, int* finished) {
    if (!s || rounds < 1) return EIK_EINVAL;
    hipStream_t st = s->stream;
    unsigned char* base = (unsigned char*)s->base;
    const int ns = s->max_problems;
    hipError_t e;
    int rc;
    // 1. Admit: slot table, sources, init and seeding into the list of the next round.
    if (!s->fresh.empty()) {
        std::vector<const eik_problem*> ptrs;
        for (int slot : s->fresh) ptrs.push_back(&s->problems[slot].pb);
        std::vector<Slot> table((size_t)ns);
        for (int i = 0; i < ns; ++i) table[i] = s->problems[i].slot;
        std::vector<SourceRefs> refs;
        rc = stage_sources(s->staging, ptrs, &refs, table.data(), table.size() * sizeof(Slot), st);
        if (rc != EIK_OK) return rc;
        e = hipMemcpyAsync(base + s->layout.off_slots, s->staging.dev, table.size() * sizeof(Slot),
                           hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e);
        for (size_t k = 0; k < s->fresh.size(); ++k) {
            eik_server::Problem& p = s->problems[s->fresh[k]];
            const double* u0 = start_values(p.pb);
            e = eik::launch_init_slot(s->P, p.slot, s->fresh[k], s->cell, s->f_dtype, p.pb.F, u0,
                                      lift_factor(p.pb.dims), st);
            if (e != hipSuccess) return hip_fail(e);
            e = eik::launch_seed(s->P, p.slot, s->cell, s->f_dtype, s->next_round,
                                 p.pb.sources.n, refs[k].idx3, refs[k].q, st, nullptr,
                                 u0 != nullptr);
            if (e != hipSuccess) return hip_fail(e);
            p.started = true;
        }
        s->fresh.clear();
    }
    // 2. Up to `rounds` rounds of every problem on the device, in one persistent launch.
    SolveParams P = s->P;
    P.round_begin = s->next_round;
    P.round_end = s->next_round + rounds;
    P.max_rounds = int64_t(1) << 62;
    P.round_log_len = 0;
    rc = ordered_solve(s->device, P, s->cell, s->f_dtype, st, s->opt.workers, s->opt.schedule);
    if (rc != EIK_OK) return rc;
    // 3. Per problem: whether a cell is still queued, status; the round where the launch
    //    stopped.
    int* counts_dev = (int*)(base + s->layout.off_counts);
    e = eik::launch_slot_counts(P, counts_dev, ns, st);
    if (e != hipSuccess) return hip_fail(e);
    int* hw = s->host_words;
    if ((e = hipMemcpyAsync(hw, counts_dev, (size_t)ns * sizeof(int), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(hw + ns, base + s->layout.off_slot_status, (size_t)ns * sizeof(int),
                            hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(hw + 2 * ns, base + s->layout.off_small + kSmallNextRound,
                            sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(hw + 2 * ns + 2, base + s->layout.off_small + kSmallStatus,
                            sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e);
    int64_t nr;
    std::memcpy(&nr, hw + 2 * ns, sizeof(nr));
    s->next_round = nr;
    const int launch_status = hw[2 * ns + 2];
    // 4. Retire converged problems: write their results, free their space.  A polished
    //    problem's result is first checked against eq. (2); one that fails is restarted from
    //    +inf (its staged speeds and exits) and stays on the device.
    int nfin = 0;
    std::vector<int> done, checked;
    for (int i = 0; i < ns; ++i) {
        eik_server::Problem& p = s->problems[i];
        if (!p.active || !p.started) continue;
        if (hw[i] != 0 && launch_status == 0) continue;
        if ((e = eik::launch_output(p.slot, s->cell, p.pb.u_out, st)) != hipSuccess)
            return hip_fail(e);
        const int status = hw[ns + i] != 0 ? hw[ns + i] : launch_status;
        if (status == 0 && start_values(p.pb) && !p.redone && s->opt.mode == EIK_MODE_FP64 &&
            p.pb.tol == 0.0) {
            checked.push_back(i);
            continue;
        }
        s->finished.push_back({p.ticket, status});
        done.push_back(i);
        ++nfin;
    }
    if (!checked.empty()) {
        int* redo_dev = (int*)(base + s->layout.off_redo);
        int* redo = hw + 2 * ns + 8;
        if ((e = eik::launch_clear_ints(redo_dev, ns, st)) != hipSuccess) return hip_fail(e);
        for (int i : checked) {
            eik_server::Problem& p = s->problems[i];
            if ((e = eik::launch_polish_check(p.slot, s->cell, s->f_dtype, p.pb.u_out,
                                              redo_dev + i, s->P.stats, st)) != hipSuccess)
                return hip_fail(e);
        }
        if ((e = hipMemcpyAsync(redo, redo_dev, (size_t)ns * sizeof(int),
                                hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(e);
        for (int i : checked) {
            eik_server::Problem& p = s->problems[i];
            if (redo[i]) {
                if ((e = eik::launch_restart_slot(s->P, p.slot, i, s->cell, s->f_dtype,
                                                  s->next_round, st, nullptr)) != hipSuccess)
                    return hip_fail(e);
                p.redone = true;
                ++s->polish_redone;
                continue;
            }
            s->finished.push_back({p.ticket, 0});
            done.push_back(i);
            ++nfin;
        }
    }
    if (!done.empty()) {
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e);
        for (int i : done) {
            eik_server::Problem& p = s->problems[i];
            range_free<size_t>(s->free_pool, p.pool_off, p.g.bytes());
            range_free<int64_t>(s->free_cells, p.slot.cell_base, p.g.ncell);
            s->pool_used -= p.g.bytes();
            s->cells_used -= p.g.ncell;
            p = eik_server::Problem();
        }
    }
    if (launch_status != 0) {
        // The launch was stopped (watchdog): every problem on the device was retired above with
        // that status; the next step starts from a clean control state.
        if ((e = eik::launch_init_global(s->P, st)) != hipSuccess) return hip_fail(e);
        s->next_round = 0;
    }
    if (finished) *finished = nfin;
    return launch_status;
}

int eik_server_poll(eik_server* s, int max, int64_t* tickets, int* status, int* n_out) {
    if (!s || max < 0 || !n_out || (max > 0 && (!tickets || !status))) return EIK_EINVAL;
    const int n = std::min<int>(max, (int)s->finished.size());
    for (int i = 0; i < n; ++i) {
        tickets[i] = s->finished[i].first;
        status[i] = s->finished[i].second;
    }
    s->finished.erase(s->finished.begin(), s->finished.begin() + n);
    *n_out = n;
    return EIK_OK;
}

int eik_server_load(eik_server* s, int* problems, int64_t* cells, size_t* pool_used) {
    if (!s) return EIK_EINVAL;
    int np = 0;
    for (auto& p : s->problems) np += p.active ? 1 : 0;
    if (problems) *problems = np;
    if (cells) *cells = s->cells_used;
    if (pool_used) *pool_used = s->pool_used;
    return EIK_OK;
}

int64_t eik_server_polish_redone(const eik_server* s) {
    return s ? s->polish_redone : (int64_t)EIK_EINVAL;
}

int eik_server_destroy(eik_server* s) {
    if (!s) return EIK_EINVAL;
    if (s->stream || s->base) (void)hipStreamSynchronize(s->stream);
    s->staging.release();
    if (s->host_words) (void)hipHostFree(s->host_words);
    if (s->base) (void)hipFree(s->base);
    if (s->pool) (void)hipFree(s->pool);
    delete s;
    return EIK_OK;
}

}  // extern "C"
