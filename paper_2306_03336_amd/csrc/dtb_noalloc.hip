// dtb_noalloc.hip -- dtb_run_noalloc: the resident deep-temporal-blocking
// path without any allocation, for callers that cannot allocate device memory.
//
// Everything the kernels need beyond the caller's grid -- the descriptor
// table, the epoch flags, the error word and the two exchange buffers -- lives
// in one file-scope device array, `scratch`, of kNoallocScratchBytes.  The
// loader reserves it on every GPU the library runs on; it is held until the
// process ends.  Host code never passes the array's name to a kernel: its
// device address is looked up once per device with hipGetSymbolAddress and
// that address is used from then on.
//
// Per call, on the caller's stream: k_noalloc_setup writes the descriptor
// table (from the layout passed by value), zeroes the epoch flags and the
// error word; the cooperative resident kernel runs every time step; if the
// caller passed an error word, k_noalloc_report ORs the run's error into it.
// The host plans with fixed-size arrays (no heap) and copies nothing.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/dtb.h"
#include "dtb_internal.h"
#include "dtb_launch.h"
#include "dtb_plan.h"

namespace dtb {
namespace {

// Layout of the scratch array: descriptor table, epoch flags (one per
// workgroup, kFlagStride words apart), the error word, then the two exchange
// buffers (each a copy of the grid's storage shape).
constexpr size_t kTableBytes = (size_t)kFixedMaxWg * sizeof(WgDesc);
constexpr size_t kFlagsOffset = (kTableBytes + 255) / 256 * 256;
constexpr size_t kFlagsBytes = (size_t)kFixedMaxWg * kFlagStride * sizeof(uint32_t);
constexpr size_t kErrOffset = kFlagsOffset + kFlagsBytes;
constexpr size_t kBufOffset = kErrOffset + 256;
constexpr size_t kBufBytes = DTB_NOALLOC_MAX_BUFFER_BYTES;
constexpr size_t kNoallocScratchBytes = kBufOffset + 2 * kBufBytes;
static_assert(kNoallocScratchBytes == DTB_NOALLOC_SCRATCH_BYTES, "scratch size stated in dtb.h");

__device__ __align__(256) static unsigned char scratch[kNoallocScratchBytes];

// The layout, by value (about 1 KiB of kernel arguments).
struct TableArgs {
    int32_t rows, cols, k, pr, pc, nwg;
    int32_t rb[kFixedMaxParts + 1], re0[kFixedMaxParts];
    int32_t cb[kFixedMaxParts + 1], ce0[kFixedMaxParts];
    int16_t slot_of_tile[kFixedMaxWg];
};

// One workgroup: the descriptor of every launch slot (as the host planner
// builds it for a resident grid: whole interior computed and stored,
// neighbours = tiles whose owned cells lie within k, in slot order), the
// epoch flags and the error word zeroed.
__global__ __launch_bounds__(256) void k_noalloc_setup(TableArgs a, WgDesc* table, uint32_t* flags, int* err)
{
    __shared__ int16_t tile_of_slot[kFixedMaxWg];
    for (int t = threadIdx.x; t < a.nwg; t += blockDim.x) tile_of_slot[a.slot_of_tile[t]] = (int16_t)t;
    for (int b = threadIdx.x; b < a.nwg; b += blockDim.x)
        __hip_atomic_store(flags + (size_t)b * kFlagStride, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) __hip_atomic_store(err, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    for (int slot = threadIdx.x; slot < a.nwg; slot += blockDim.x) {
        const int t = tile_of_slot[slot];
        const int tr = t / a.pc, tc = t % a.pc;
        WgDesc d{};
        d.prob = 0;
        d.ext_r0 = a.re0[tr];
        d.ext_c0 = a.ce0[tc];
        d.own_r0 = a.rb[tr];
        d.own_r1 = a.rb[tr + 1];
        d.own_c0 = a.cb[tc];
        d.own_c1 = a.cb[tc + 1];
        d.cr_r0 = d.st_r0 = 1;
        d.cr_r1 = d.st_r1 = a.rows + 1;
        d.cr_c0 = d.st_c0 = 1;
        d.cr_c1 = d.st_c1 = a.cols + 1;
        d.nnb = 0;
        for (int b = 0; b < a.nwg; ++b) {
            if (b == slot) continue;
            const int u = tile_of_slot[b];
            const int ur = u / a.pc, uc = u % a.pc;
            const bool meet = a.rb[ur] < d.own_r1 + a.k && a.rb[ur + 1] > d.own_r0 - a.k &&
                              a.cb[uc] < d.own_c1 + a.k && a.cb[uc + 1] > d.own_c0 - a.k;
            if (meet && d.nnb < kMaxNeighbours) d.nb[d.nnb++] = b;
        }
        table[slot] = d;
    }
}

__global__ void k_noalloc_report(const int* err, int32_t* out)
{
    const int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0 && e != 0) __hip_atomic_fetch_or(out, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kMaxDevices = 64;
constexpr int kNumXcd = 8;
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kRowsPerLane[] = {8, 12, 16, 24, 28};
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// The scratch array's device address on the current device (looked up once per device).
dtb_status scratch_address(int dev, unsigned char** out)
{
    if (dev < 0 || dev >= kMaxDevices) return DTB_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return DTB_ERR_HIP;
        }
        g_scratch[dev] = (unsigned char*)ptr;
    }
    *out = g_scratch[dev];
    return DTB_OK;
}

// The resident plan dtb_run would choose (same candidates, same cost model),
// built without allocation.
bool choose(int64_t rows, int64_t cols, int dtype, int n_cu, FixedLayout* best, const void** best_f)
{
    const int eb = dtype == DTB_F64 ? 8 : 4;
    double best_cost = 1e300;
    bool found = false;
    for (int R : kRowsPerLane) {
        int C = 0, waves = 0;
        if (!dtb_kernel(dtype, R, true, false, false, &C, &waves)) continue;
        const bool rc = rows < (int64_t)waves * R, cm = cols < (int64_t)kWaveSize * C;
        const void* f = dtb_kernel(dtype, R, true, cm, rc, &C, &waves);
        hipFuncAttributes fa{};
        if (!f || hipFuncGetAttributes(&fa, f) != hipSuccess || fa.localSizeBytes != 0) continue;
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, waves * kWaveSize, 0) != hipSuccess) continue;
        for (int k = 2; k <= 24; ++k) {
            FixedLayout L;
            if (!build_fixed_layout(rows, cols, R, C, waves, k, kNumXcd, &L)) continue;
            if (L.nwg > occ * n_cu) continue;
            const double cost = layout_cost_of(L.nwg, R, C, L.ER, L.EC, k, occ, n_cu, eb);
            if (cost < best_cost) {
                best_cost = cost;
                *best = L;
                *best_f = f;
                found = true;
            }
        }
    }
    return found;
}

}  // namespace
}  // namespace dtb

using namespace dtb;

extern "C" dtb_status dtb_run_noalloc(const dtb_grid* grid, const double coeffs[5], int64_t T, dtb_dtype dtype,
                                      int32_t* err_flag, void* stream)
{
    if (!grid || !coeffs || !grid->data || T < 0) return DTB_ERR_INVALID_ARG;
    if (grid->rows < 1 || grid->cols < 1 || grid->pitch < grid->cols + 2) return DTB_ERR_INVALID_ARG;
    if (dtype != DTB_F64 && dtype != DTB_F32) return DTB_ERR_INVALID_ARG;
    const size_t eb = dtype == DTB_F64 ? 8 : 4;
    if ((double)(grid->rows + 2) * (double)grid->pitch * eb > (double)kBufBytes) return DTB_ERR_UNSUPPORTED;
    if (T == 0) return DTB_OK;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return DTB_ERR_HIP;
    unsigned char* base = nullptr;
    if (dtb_status rc = scratch_address(dev, &base); rc != DTB_OK) return rc;

    FixedLayout L;
    const void* f = nullptr;
    if (!choose(grid->rows, grid->cols, (int)dtype, ncu, &L, &f)) return DTB_ERR_NOT_CORESIDENT;

    TableArgs a{};
    a.rows = (int32_t)grid->rows;
    a.cols = (int32_t)grid->cols;
    a.k = L.k;
    a.pr = L.pr;
    a.pc = L.pc;
    a.nwg = L.nwg;
    for (int i = 0; i <= L.pr; ++i) a.rb[i] = L.rb[i];
    for (int i = 0; i < L.pr; ++i) a.re0[i] = L.re0[i];
    for (int i = 0; i <= L.pc; ++i) a.cb[i] = L.cb[i];
    for (int i = 0; i < L.pc; ++i) a.ce0[i] = L.ce0[i];
    for (int i = 0; i < L.nwg; ++i) a.slot_of_tile[i] = (int16_t)L.slot_of_tile[i];

    WgDesc* table = (WgDesc*)base;
    uint32_t* flags = (uint32_t*)(base + kFlagsOffset);
    int* err = (int*)(base + kErrOffset);
    hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, st, a, table, flags, err);
    if (hipGetLastError() != hipSuccess) return DTB_ERR_HIP;

    ProbDesc P{};
    P.grid = grid->data;
    P.xbuf[0] = base + kBufOffset;
    P.xbuf[1] = base + kBufOffset + kBufBytes;
    P.pitch = grid->pitch;
    P.T = T;
    P.rows = (int32_t)grid->rows;
    P.cols = (int32_t)grid->cols;
    P.k = L.k;
    P.wg0 = 0;
    P.nwg = L.nwg;
    P.dtype = (int32_t)dtype;
    P.fma = 1;
    P.narrow_cols = L.narrow_cols ? 1 : 0;
    P.narrow_rows = L.narrow_rows ? 1 : 0;
    P.debug = 0;
    P.timing = nullptr;
    P.direct_xchg = 0;
    for (int i = 0; i < 5; ++i) P.coeffs[i] = coeffs[i];
    const WgDesc* wgs = table;
    uint32_t spin = kSpinLimit;
    void* args[] = {&P, (void*)&wgs, (void*)&flags, (void*)&err, &spin};
    if (hipLaunchCooperativeKernel(f, dim3(L.nwg), dim3(L.waves * kWaveSize), args, 0, st) != hipSuccess)
        return DTB_ERR_HIP;
    if (err_flag) {
        hipLaunchKernelGGL(k_noalloc_report, dim3(1), dim3(64), 0, st, (const int*)err, err_flag);
        if (hipGetLastError() != hipSuccess) return DTB_ERR_HIP;
    }
    return DTB_OK;
}
