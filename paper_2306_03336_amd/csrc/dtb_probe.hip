// dtb_probe.hip -- micro-benchmarks that measure the denominators the kernels'
// rooflines are stated against on the running part: LDS read and write
// bandwidth, device copy bandwidth (a buffer that fits in the Infinity Cache
// and one that does not), the latency of a device-wide barrier and of a
// neighbour flag exchange between persistent workgroups.  Not part of the
// stencil path; exposed through include/dtb_testing.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/dtb.h"
#include "../../include/dtb_testing.h"
#include "dtb_internal.h"
#include "dtb_tile.h"

namespace dtb {
namespace {

constexpr int kProbeThreads = 512;
constexpr int kLdsProbeBytes = 64 * 1024;
constexpr int kLdsUnroll = 8;

// LDS bandwidth: every thread moves 16 bytes per access, consecutive lanes on
// consecutive 16-byte slots (no bank conflicts), kLdsUnroll accesses per
// iteration.  The empty asm with a memory clobber keeps each iteration's
// accesses from being merged with the next one's.
template <bool WRITE>
__global__ __launch_bounds__(kProbeThreads) void k_probe_lds(int iters, uint32_t* sink)
{
    __shared__ __attribute__((aligned(16))) uint4 buf[kLdsProbeBytes / 16];
    const int tid = threadIdx.x;
    for (int i = tid; i < kLdsProbeBytes / 16; i += kProbeThreads) buf[i] = make_uint4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    uint4 acc = make_uint4(tid, 0, 0, 0);
    constexpr int kSlots = kLdsProbeBytes / 16;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kLdsUnroll; ++u) {
            const int slot = (tid + (u + it * kLdsUnroll) * kProbeThreads) & (kSlots - 1);
            if constexpr (WRITE) {
                buf[slot] = acc;
                acc.x += 1;
            } else {
                const uint4 v = buf[slot];
                acc.x ^= v.x;
                acc.y ^= v.y;
                acc.z ^= v.z;
                acc.w ^= v.w;
            }
        }
        asm volatile("" ::: "memory");
    }
    __syncthreads();
    if constexpr (WRITE) acc = buf[tid];
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x9e3779b9u) sink[blockIdx.x] = acc.x;  // almost never taken
}

// Device copy, 16 bytes per lane per access, four accesses in flight per lane.
__global__ __launch_bounds__(256) void k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// `iters` device-wide barriers (the two-level barrier of the tile-serial sweep).
__global__ __launch_bounds__(kProbeThreads) void k_probe_barrier(int iters, uint32_t* bar, int* err)
{
    for (int n = 1; n <= iters; ++n) grid_barrier(bar, (uint32_t)n, err, 1u << 22);
}

// `iters` neighbour exchange points without data: each workgroup raises its
// flag and waits for the workgroups listed in its descriptor (the resident
// kernel's synchronisation, without the strips).
__global__ __launch_bounds__(kProbeThreads) void k_probe_flags(int iters, const WgDesc* __restrict__ wgs,
                                                               uint32_t* flags, int* err)
{
    const int me = blockIdx.x;
    const uint32_t base = __hip_atomic_load(flags + (size_t)me * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int n = 1; n <= iters; ++n) exchange_point(flags, me, wgs[me], base + (uint32_t)n, err, 1u << 22);
}

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t st;
    explicit Timer(hipStream_t s) : st(s) {}
    bool start() { return hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess && hipEventRecord(e0, st) == hipSuccess; }
    bool stop(double* ms)
    {
        float f = 0;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&f, e0, e1) != hipSuccess)
            return false;
        *ms = f;
        return true;
    }
    ~Timer()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace
}  // namespace dtb

using namespace dtb;

extern "C" dtb_status dtb_probe(int32_t kind, int64_t size, int32_t iters, int32_t nwg, void* stream, double* out)
{
    if (!out || iters < 1 || nwg < 0) return DTB_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return DTB_ERR_HIP;
    if (nwg == 0) nwg = (kind == DTB_PROBE_LDS_READ || kind == DTB_PROBE_LDS_WRITE) ? 2 * ncu : ncu;
    dtb_status rc = DTB_OK;
    switch (kind) {
    case DTB_PROBE_LDS_READ:
    case DTB_PROBE_LDS_WRITE: {
        uint32_t* sink = nullptr;
        if (hipMalloc(&sink, (size_t)nwg * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        const void* f = kind == DTB_PROBE_LDS_READ ? (const void*)&k_probe_lds<false> : (const void*)&k_probe_lds<true>;
        void* args[] = {&iters, &sink};
        Timer t(st);
        double ms = 0;
        // One warm-up launch, then the timed one.
        if (hipLaunchKernel(f, dim3(nwg), dim3(kProbeThreads), args, 0, st) != hipSuccess || !t.start() ||
            hipLaunchKernel(f, dim3(nwg), dim3(kProbeThreads), args, 0, st) != hipSuccess || !t.stop(&ms))
            rc = DTB_ERR_HIP;
        else {
            out[0] = ms;
            out[1] = (double)nwg * kProbeThreads * 16.0 * kLdsUnroll * iters;  // bytes moved
        }
        (void)hipFree(sink);
        break;
    }
    case DTB_PROBE_COPY: {
        if (size < 16) return DTB_ERR_INVALID_ARG;
        const int64_t n = size / 16;
        uint4 *a = nullptr, *b = nullptr;
        if (hipMalloc(&a, (size_t)n * 16) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&b, (size_t)n * 16) != hipSuccess) {
            (void)hipFree(a);
            return DTB_ERR_OUT_OF_MEMORY;
        }
        const int grid = nwg * 8;
        Timer t(st);
        double ms = 0;
        bool ok = hipMemsetAsync(a, 0, (size_t)n * 16, st) == hipSuccess;
        if (ok) {
            hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(256), 0, st, (const uint4*)a, b, n);
            ok = hipGetLastError() == hipSuccess && t.start();
        }
        for (int i = 0; ok && i < iters; ++i) {
            hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(256), 0, st, (const uint4*)a, b, n);
            ok = hipGetLastError() == hipSuccess;
        }
        if (ok && t.stop(&ms)) {
            out[0] = ms;
            out[1] = 2.0 * (double)n * 16.0 * iters;  // bytes read + written
        } else {
            rc = DTB_ERR_HIP;
        }
        (void)hipFree(a);
        (void)hipFree(b);
        break;
    }
    case DTB_PROBE_BARRIER:
    case DTB_PROBE_FLAGS: {
        // Persistent launch: every workgroup must be resident at once.
        if (nwg > ncu) return DTB_ERR_NOT_CORESIDENT;
        uint32_t* words = nullptr;
        int* err = nullptr;
        WgDesc* wgs = nullptr;
        const size_t nwords = (size_t)std::max(nwg, kBarrierSlots) * kFlagStride;
        if (hipMalloc(&words, nwords * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&err, sizeof(int)) != hipSuccess) {
            (void)hipFree(words);
            return DTB_ERR_OUT_OF_MEMORY;
        }
        bool ok = hipMemset(words, 0, nwords * sizeof(uint32_t)) == hipSuccess && hipMemset(err, 0, sizeof(int)) == hipSuccess;
        if (ok && kind == DTB_PROBE_FLAGS) {
            // A ring of workgroups, each waiting for the 8 nearest in launch order (4 before, 4 after):
            // the neighbour count of an interior tile of the resident layout.
            std::vector<WgDesc> h(nwg);
            for (int b = 0; b < nwg; ++b) {
                h[b] = WgDesc{};
                for (int d = 1; d <= 4 && 2 * d <= nwg - 1; ++d) {
                    h[b].nb[h[b].nnb++] = (b + d) % nwg;
                    h[b].nb[h[b].nnb++] = (b + nwg - d) % nwg;
                }
            }
            ok = hipMalloc(&wgs, (size_t)nwg * sizeof(WgDesc)) == hipSuccess &&
                 hipMemcpy(wgs, h.data(), (size_t)nwg * sizeof(WgDesc), hipMemcpyHostToDevice) == hipSuccess;
        }
        Timer t(st);
        double ms = 0;
        if (ok) {
            const void* f = kind == DTB_PROBE_BARRIER ? (const void*)&k_probe_barrier : (const void*)&k_probe_flags;
            void* args_b[] = {&iters, &words, &err};
            void* args_f[] = {&iters, &wgs, &words, &err};
            ok = t.start() && hipLaunchCooperativeKernel(f, dim3(nwg), dim3(kProbeThreads),
                                                        kind == DTB_PROBE_BARRIER ? args_b : args_f, 0, st) == hipSuccess &&
                 t.stop(&ms);
        }
        int e = 0;
        if (ok) ok = hipMemcpy(&e, err, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess;
        if (!ok) rc = DTB_ERR_HIP;
        else if (e) rc = DTB_ERR_TIMEOUT;
        else {
            out[0] = ms;
            out[1] = (double)iters;
        }
        (void)hipFree(words);
        (void)hipFree(err);
        if (wgs) (void)hipFree(wgs);
        break;
    }
    default: return DTB_ERR_INVALID_ARG;
    }
    return rc;
}
