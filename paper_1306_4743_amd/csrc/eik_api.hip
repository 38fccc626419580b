// eik_api.hip -- the C ABI of libeik: argument validation, per-stream workspaces, launches.
//
// Every entry point is declared, with its contract, in include/eik.h.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "eik_internal.h"

namespace {

using eik::SolveParams;

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
    int ncx = 0, ncy = 0, ncz = 0;
    int64_t ncell = 0;
    size_t off_u = 0, off_f = 0, off_faces = 0, off_key = 0, off_flags = 0, off_list = 0,
           off_small = 0, total = 0;
};

// Device workspace of one solve: cell-blocked values, speeds, face copies, the double-buffered
// cell state, the lists and a small control area (round control blocks, barrier, status,
// counters).
bool make_layout(const int64_t dims[3], int cell, int f_dtype, Layout* L) {
    const int64_t r = cell;
    L->ncx = (int)((dims[0] + r - 1) / r);
    L->ncy = (int)((dims[1] + r - 1) / r);
    L->ncz = (int)((dims[2] + r - 1) / r);
    L->ncell = (int64_t)L->ncx * L->ncy * L->ncz;
    if (L->ncell * r * r * r >= (int64_t(1) << 31)) return false;
    const size_t n = (size_t)L->ncell;
    const size_t r3 = (size_t)(r * r * r), r2 = (size_t)(r * r);
    const size_t fsz = f_dtype == EIK_F32 ? 4 : 8;
    size_t o = 0;
    L->off_small = o; o = align_up(o + eik::kSmallBytes);
    L->off_u = o; o = align_up(o + n * r3 * 8);
    L->off_f = o; o = align_up(o + n * r3 * fsz);
    L->off_faces = o; o = align_up(o + n * 6 * r2 * 8);
    L->off_key = o; o = align_up(o + 2 * n * 8);
    L->off_flags = o; o = align_up(o + 2 * n * 4);
    L->off_list = o; o = align_up(o + 2 * n * 4);
    L->total = o;
    return true;
}

using eik::kSmallBar;
using eik::kSmallCtl;
using eik::kSmallStats;
using eik::kSmallStatus;

struct Workspace {
    int device = -1;
    void* base = nullptr;
    size_t bytes = 0;
    void* src_dev = nullptr;  // device copy of host-provided sources
    size_t src_bytes = 0;
    void* src_host = nullptr;  // pinned staging buffer
    size_t src_host_bytes = 0;
    hipEvent_t staged = nullptr;  // last copy out of src_host finished
    bool used = false;
    int64_t cells = 0;
    std::mutex mu;  // serialises enqueues that share this workspace
    // ring of event quadruples for timed solves
    static constexpr int kRing = 256;
    std::vector<eik::LaunchEvents> ring;
    int64_t timed = 0;  // timed solves enqueued so far
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

// Per device: the event recorded after the most recently enqueued persistent solve kernel.
// Each new solve kernel waits for it, so solve kernels of different streams run one at a time
// (each needs the whole device resident for its grid barrier); the other kernels still overlap.
struct DeviceOrder {
    std::mutex mu;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int next = 0;
    bool any = false;
};
std::map<int, DeviceOrder*> g_order;

DeviceOrder* device_order(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_order.find(dev);
    if (it != g_order.end()) return it->second;
    DeviceOrder* d = new DeviceOrder();
    g_order[dev] = d;
    return d;
}

int hip_fail(hipError_t e) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return EIK_ENOMEM;
    return EIK_EHIP;
}

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
    e = hipEventCreateWithFlags(&w->staged, hipEventDisableTiming);
    if (e != hipSuccess) { delete w; *rc = hip_fail(e); return nullptr; }
    g_ws[key] = w;
    return w;
}

// Grows a device buffer; waits for the stream first because the old buffer may be in use.
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

int ensure_host(Workspace* w, size_t need) {
    if (w->src_host_bytes >= need && w->src_host) return EIK_OK;
    if (w->src_host) {
        (void)hipEventSynchronize(w->staged);
        (void)hipHostFree(w->src_host);
        w->src_host = nullptr;
        w->src_host_bytes = 0;
    }
    hipError_t e = hipHostMalloc(&w->src_host, need, hipHostMallocDefault);
    if (e != hipSuccess) { w->src_host = nullptr; return hip_fail(e); }
    w->src_host_bytes = need;
    return EIK_OK;
}

bool valid_dims(const int64_t* dims) {
    if (!dims) return false;
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 2) return false;
    const int64_t m = dims[0] * dims[1];
    if (m >= (int64_t(1) << 31)) return false;
    return m * dims[2] < (int64_t(1) << 31);
}

}  // namespace

extern "C" {

const char* eik_strerror(int code) {
    switch (code) {
        case EIK_OK: return "EIK_OK";
        case EIK_EINVAL: return "EIK_EINVAL: invalid argument";
        case EIK_ENOMEM: return "EIK_ENOMEM: out of memory";
        case EIK_EHIP: return "EIK_EHIP: HIP runtime error";
        case EIK_ENOCONV: return "EIK_ENOCONV: round cap reached before convergence";
        case EIK_ECANCELLED: return "EIK_ECANCELLED: stopped by the device watchdog";
        default: return "EIK: unknown status";
    }
}

const char* eik_version(void) { return "eik-mi355x 0.1 (gfx950)"; }

int eik_query_workspace(const int64_t dims[3], int cell, int f_dtype, int mode, size_t* bytes) {
    if (!bytes || !valid_dims(dims) || (cell != 4 && cell != 8) ||
        (f_dtype != EIK_F32 && f_dtype != EIK_F64) || mode != EIK_MODE_FP64)
        return EIK_EINVAL;
    Layout L;
    if (!make_layout(dims, cell, f_dtype, &L)) return EIK_EINVAL;
    *bytes = L.total;
    return EIK_OK;
}

int eik_solve_ex(const int64_t dims[3], double h, const void* F, int f_dtype,
                 const eik_sources* sources, double* u_out, int cell, double tol,
                 hipStream_t stream, const eik_options* options) {
    eik_options opt;
    std::memset(&opt, 0, sizeof(opt));
    if (options) opt = *options;
    // ---- synchronous validation: nothing is enqueued on failure
    if (!valid_dims(dims) || !F || !u_out || !sources) return EIK_EINVAL;
    if (!(h > 0.0) || !std::isfinite(h)) return EIK_EINVAL;
    if (f_dtype != EIK_F32 && f_dtype != EIK_F64) return EIK_EINVAL;
    if (cell != 4 && cell != 8) return EIK_EINVAL;
    if (!(tol >= 0.0) || !std::isfinite(tol)) return EIK_EINVAL;
    if (opt.mode != EIK_MODE_FP64) return EIK_EINVAL;
    if (std::isnan(opt.delta) || opt.max_rounds < 0 || opt.max_sweeps < 0 || opt.workers < 0)
        return EIK_EINVAL;
    if (opt.round_log_len < 0 || (opt.round_log_len > 0 && !opt.round_log)) return EIK_EINVAL;
    if (opt.inner < 0 || opt.inner > EIK_INNER_DUAL) return EIK_EINVAL;
    const int64_t nsrc = sources->n;
    if (nsrc < 0 || (nsrc > 0 && (!sources->idx3 || !sources->q))) return EIK_EINVAL;
    if (nsrc > (int64_t(1) << 24)) return EIK_EINVAL;
    if (!sources->on_device) {
        for (int64_t n = 0; n < nsrc; ++n) {
            const int64_t* p = sources->idx3 + 3 * n;
            for (int a = 0; a < 3; ++a)
                if (p[a] < 0 || p[a] >= dims[a]) return EIK_EINVAL;
            const double qv = sources->q[n];
            if (!(qv >= 0.0) || !std::isfinite(qv)) return EIK_EINVAL;
        }
    }
    Layout L;
    if (!make_layout(dims, cell, f_dtype, &L)) return EIK_EINVAL;

    int rc = EIK_OK;
    Workspace* w = get_workspace(stream, &rc);
    if (!w) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    rc = ensure_device(&w->base, &w->bytes, L.total, stream);
    if (rc != EIK_OK) return rc;

    // ---- sources: host lists are staged through pinned memory into the workspace
    const int64_t* idx_dev = nullptr;
    const double* q_dev = nullptr;
    if (nsrc > 0) {
        if (sources->on_device) {
            idx_dev = sources->idx3;
            q_dev = sources->q;
        } else {
            const size_t sb = (size_t)nsrc * 32;
            rc = ensure_device(&w->src_dev, &w->src_bytes, sb, stream);
            if (rc != EIK_OK) return rc;
            rc = ensure_host(w, sb);
            if (rc != EIK_OK) return rc;
            hipError_t e = hipEventSynchronize(w->staged);
            if (e != hipSuccess) return hip_fail(e);
            unsigned char* hb = (unsigned char*)w->src_host;
            std::memcpy(hb, sources->idx3, (size_t)nsrc * 24);
            std::memcpy(hb + (size_t)nsrc * 24, sources->q, (size_t)nsrc * 8);
            e = hipMemcpyAsync(w->src_dev, hb, sb, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return hip_fail(e);
            e = hipEventRecord(w->staged, stream);
            if (e != hipSuccess) return hip_fail(e);
            idx_dev = (const int64_t*)w->src_dev;
            q_dev = (const double*)((unsigned char*)w->src_dev + (size_t)nsrc * 24);
        }
    }

    // ---- parameters
    unsigned char* base = (unsigned char*)w->base;
    SolveParams P;
    std::memset(&P, 0, sizeof(P));
    P.nx = (int)dims[0];
    P.ny = (int)dims[1];
    P.nz = (int)dims[2];
    P.ncx = L.ncx;
    P.ncy = L.ncy;
    P.ncz = L.ncz;
    P.ncell = (int)L.ncell;
    P.max_rounds = opt.max_rounds > 0 ? (int)std::min<int64_t>(opt.max_rounds, 1 << 30) : (1 << 20);
    P.max_sweeps = opt.max_sweeps > 0 ? opt.max_sweeps : 512;
    // default in-cell solver: sweeps at r = 8, the list relaxation at r = 4 (measured fastest)
    const int inner = opt.inner ? opt.inner : (cell == 8 ? EIK_INNER_SWEEP : EIK_INNER_LIST);
    P.inner = inner == EIK_INNER_SWEEP ? 0 : (inner == EIK_INNER_LIST ? 1 : 2);
    P.h = h;
    P.tol = tol;
    P.delta = opt.delta > 0.0 ? opt.delta : 0.0;
    P.shuffle = opt.shuffle;
    P.watchdog_polls = 1ull << 23;  // several seconds of polling
    P.u = (double*)(base + L.off_u);
    P.fw = base + L.off_f;
    P.f = P.fw;
    P.faces = (double*)(base + L.off_faces);
    P.key[0] = (uint64_t*)(base + L.off_key);
    P.key[1] = P.key[0] + L.ncell;
    P.flags[0] = (uint32_t*)(base + L.off_flags);
    P.flags[1] = P.flags[0] + L.ncell;
    P.list[0] = (int32_t*)(base + L.off_list);
    P.list[1] = P.list[0] + L.ncell;
    P.ctl = (eik::RoundCtl*)(base + L.off_small + kSmallCtl);
    P.bar = (uint32_t*)(base + L.off_small + kSmallBar);
    P.status = (int*)(base + L.off_small + kSmallStatus);
    P.stats = (unsigned long long*)(base + L.off_small + kSmallStats);
    P.round_log = opt.round_log;
    P.round_log_len = opt.round_log ? opt.round_log_len : 0;

    int used = 0;
    const eik::LaunchEvents* evp = nullptr;
    if (opt.timing) {
        if (w->ring.empty()) {
            w->ring.resize(Workspace::kRing);
            for (auto& q4 : w->ring)
                for (auto& ev : q4.ev) {
                    hipError_t ee = hipEventCreate(&ev);
                    if (ee != hipSuccess) return hip_fail(ee);
                }
        }
        evp = &w->ring[w->timed % Workspace::kRing];
        w->timed++;
    }
    DeviceOrder* dord = device_order(w->device);
    std::lock_guard<std::mutex> olk(dord->mu);
    for (auto& ev : dord->ev) {
        if (!ev) {
            hipError_t ee = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (ee != hipSuccess) return hip_fail(ee);
        }
    }
    // Alternate two events: the new launch waits on the previous one and records the other.
    eik::SolveOrder order;
    order.after = dord->any ? dord->ev[dord->next ^ 1] : nullptr;
    order.done = dord->ev[dord->next];
    hipError_t e = eik::launch_solve(P, cell, f_dtype, F, nsrc, idx_dev, q_dev, u_out, stream,
                                     opt.workers, &used, evp, &order);
    if (e == hipSuccess && nsrc > 0) {
        dord->any = true;
        dord->next ^= 1;
    }
    if (e != hipSuccess) return hip_fail(e);
    w->used = true;
    w->cells = L.ncell;
    return EIK_OK;
}

int eik_solve(const int64_t dims[3], double h, const void* F, int f_dtype,
              const eik_sources* sources, double* u_out, int cell, double tol,
              hipStream_t stream) {
    return eik_solve_ex(dims, h, F, f_dtype, sources, u_out, cell, tol, stream, nullptr);
}

int eik_stream_status(hipStream_t stream, eik_stats* stats) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return EIK_EHIP;
    Workspace* w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_ws.find(std::make_pair(dev, stream));
        if (it != g_ws.end()) w = it->second;
    }
    if (!w || !w->used) return EIK_EINVAL;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e);
    unsigned char* base = (unsigned char*)w->base;
    int status = 0;
    unsigned long long st[eik::ST_COUNT];
    e = hipMemcpy(&status, base + kSmallStatus, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    e = hipMemcpy(st, base + kSmallStats, sizeof(st), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    if (stats) {
        stats->rounds = (int64_t)st[eik::ST_ROUNDS];
        stats->visits = (int64_t)st[eik::ST_VISITS];
        stats->sweeps = (int64_t)st[eik::ST_SWEEPS];
        stats->updates = (int64_t)st[eik::ST_UPDATES];
        stats->deferred = (int64_t)st[eik::ST_DEFERRED];
        stats->requeued = (int64_t)st[eik::ST_REQUEUED];
        stats->cells = w->cells;
        stats->status = status;
        stats->workers = (int64_t)st[eik::ST_WORKERS];
        stats->cycles_pop = (int64_t)st[eik::ST_CYC_POP];
        stats->cycles_stage = (int64_t)st[eik::ST_CYC_STAGE];
        stats->cycles_sweep = (int64_t)st[eik::ST_CYC_SWEEP];
        stats->cycles_write = (int64_t)st[eik::ST_CYC_WRITE];
        stats->cycles_wait = (int64_t)st[eik::ST_CYC_WAIT];
    }
    return status;
}

int eik_kernel_times(hipStream_t stream, int n, double* solve_ms, double* total_ms) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return EIK_EHIP;
    if (n < 0) return EIK_EINVAL;
    Workspace* w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_ws.find(std::make_pair(dev, stream));
        if (it != g_ws.end()) w = it->second;
    }
    if (!w || w->timed == 0) return 0;
    std::lock_guard<std::mutex> lk(w->mu);
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e);
    int64_t have = std::min<int64_t>(w->timed, Workspace::kRing);
    if (n > have) n = (int)have;
    for (int i = 0; i < n; ++i) {
        const int64_t k = w->timed - n + i;
        const eik::LaunchEvents& q4 = w->ring[k % Workspace::kRing];
        float a = 0.f, b = 0.f;
        e = hipEventElapsedTime(&a, q4.ev[1], q4.ev[2]);
        if (e != hipSuccess) return hip_fail(e);
        e = hipEventElapsedTime(&b, q4.ev[0], q4.ev[3]);
        if (e != hipSuccess) return hip_fail(e);
        if (solve_ms) solve_ms[i] = a;
        if (total_ms) total_ms[i] = b;
    }
    return n;
}

void eik_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_ws) {
        Workspace* w = kv.second;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(w->device);
        (void)hipStreamSynchronize(kv.first.second);
        if (w->staged) { (void)hipEventSynchronize(w->staged); (void)hipEventDestroy(w->staged); }
        if (w->base) (void)hipFree(w->base);
        if (w->src_dev) (void)hipFree(w->src_dev);
        if (w->src_host) (void)hipHostFree(w->src_host);
        for (auto& q4 : w->ring)
            for (auto& ev : q4.ev)
                if (ev) (void)hipEventDestroy(ev);
        (void)hipSetDevice(cur);
        delete w;
    }
    g_ws.clear();
}

}  // extern "C"
