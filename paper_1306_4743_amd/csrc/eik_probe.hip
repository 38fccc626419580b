// Bandwidth probes (include/eik_probe.h): a plain HBM copy and LDS read / write streams, so
// that the solver's roofline fractions can be read against what simple kernels reach on the
// same device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eik_probe.h"

namespace {

constexpr int kThreads = 256;
constexpr int kLdsWords = 2048;  // 16-byte words: 32 KiB per workgroup

__global__ void __launch_bounds__(kThreads) k_copy(const uint4* __restrict__ a,
                                                    uint4* __restrict__ b, size_t n) {
    const size_t stride = (size_t)gridDim.x * kThreads;
    size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x;
    // Four independent 16-byte loads in flight per thread, then the ragged rest.
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 v0 = a[i], v1 = a[i + stride], v2 = a[i + 2 * stride], v3 = a[i + 3 * stride];
        b[i] = v0;
        b[i + stride] = v1;
        b[i + 2 * stride] = v2;
        b[i + 3 * stride] = v3;
    }
    for (; i < n; i += stride) b[i] = a[i];
}

__global__ void __launch_bounds__(kThreads) k_lds_read(int iters, unsigned int* __restrict__ out) {
    __shared__ uint4 s[kLdsWords];
    const int t = threadIdx.x;
    for (int j = t; j < kLdsWords; j += kThreads)
        s[j] = make_uint4((unsigned)j, 3u * j + 1u, 5u * j + 2u, 7u * j + 3u);
    __syncthreads();
    unsigned int acc = 0;
    int idx = t, k = 0;
    constexpr int M = kLdsWords - 1;
    // Four loads in flight per step.  A thread's words repeat every 8 iterations; without the
    // compiler barrier the loads would be hoisted out of the loop and LDS read only once.
    for (; k + 4 <= iters; k += 4) {
        const uint4 v0 = s[idx], v1 = s[(idx + kThreads) & M], v2 = s[(idx + 2 * kThreads) & M],
                    v3 = s[(idx + 3 * kThreads) & M];
        acc ^= v0.x ^ v0.y ^ v0.z ^ v0.w ^ v1.x ^ v1.y ^ v1.z ^ v1.w;
        acc ^= v2.x ^ v2.y ^ v2.z ^ v2.w ^ v3.x ^ v3.y ^ v3.z ^ v3.w;
        idx = (idx + 4 * kThreads) & M;
        __asm__ __volatile__("" ::: "memory");
    }
    for (; k < iters; ++k) {
        const uint4 v = s[idx];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
        idx = (idx + kThreads) & M;
        __asm__ __volatile__("" ::: "memory");
    }
    out[blockIdx.x * kThreads + t] = acc;
}

__global__ void __launch_bounds__(kThreads) k_lds_write(int iters, unsigned int* __restrict__ out) {
    __shared__ uint4 s[kLdsWords];
    const int t = threadIdx.x;
    int idx = t;
    for (int k = 0; k < iters; ++k) {
        s[idx] = make_uint4((unsigned)(t + k), (unsigned)k, (unsigned)t, 1u);
        idx = (idx + kThreads) & (kLdsWords - 1);
        __asm__ __volatile__("" ::: "memory");  // every store is kept (no store merging)
    }
    __syncthreads();
    unsigned int acc = 0;
    for (int j = t; j < kLdsWords; j += kThreads) {
        const uint4 v = s[j];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    out[blockIdx.x * kThreads + t] = acc;
}

int fail(hipError_t e) { return e == hipSuccess ? 0 : -3; }

// One untimed launch, then `reps` timed ones between two events; mean ms per launch.
template <typename Launch>
int timed(Launch launch, int reps, hipStream_t stream, float* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) { launch(); e = hipGetLastError(); }
    if (e == hipSuccess) e = hipEventRecord(e0, stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) { launch(); e = hipGetLastError(); }
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e == hipSuccess && ms) *ms = t / (float)reps;
    return fail(e);
}

}  // namespace

extern "C" {

int eikp_copy(const void* src, void* dst, size_t bytes, int reps, hipStream_t stream, float* ms) {
    if (!src || !dst || bytes == 0 || bytes % 16 || reps < 1 || reps > 1000 || !ms ||
        (uintptr_t)src % 16 || (uintptr_t)dst % 16)
        return -1;
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    if (a < b + bytes && b < a + bytes) return -1;  // overlapping buffers
    const size_t n = bytes / 16;
    size_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    const uint4* s = reinterpret_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(dst);
    return timed([&] {
        hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kThreads), 0, stream, s, d, n);
    }, reps, stream, ms);
}

int eikp_lds(int blocks, int iters, int write, int reps, unsigned int* out, hipStream_t stream,
             float* ms, double* bytes_moved) {
    if (blocks < 1 || blocks > 65536 || iters < 1 || iters > (1 << 20) || (write != 0 && write != 1) ||
        reps < 1 || reps > 1000 || !out || !ms)
        return -1;
    if (bytes_moved) *bytes_moved = (double)blocks * kThreads * (double)iters * 16.0;
    return timed([&] {
        if (write)
            hipLaunchKernelGGL(k_lds_write, dim3(blocks), dim3(kThreads), 0, stream, iters, out);
        else
            hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(kThreads), 0, stream, iters, out);
    }, reps, stream, ms);
}

}  // extern "C"
