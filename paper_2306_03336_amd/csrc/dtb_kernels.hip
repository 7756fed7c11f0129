// dtb_kernels.hip -- gfx950 kernels for the j2d5pt iterative stencil.
//
// The update (Listing 1 of Zhang et al., GPGPU '23): every interior cell
// becomes w*W + e*E + s*S + c*C + n*N of the previous step's values, with
// W = (i, j-1), E = (i, j+1), S = (i-1, j), N = (i+1, j) (x = column j is the
// contiguous index, y = row i).  Reads and writes never alias within a step
// (Jacobi).  The one-cell ring around the interior is a fixed Dirichlet halo.
//
// Two kernels:
//
//  * k_step: one time step per launch, global memory to global memory.  It is
//    the untiled baseline the paper starts from before the time loop moves
//    into the kernel (Section 3.1).  Bound by HBM (or the Infinity Cache when
//    the two buffers fit in it): one read and one write per cell-update.
//
//  * k_dtb: deep temporal blocking (Sections 1, 3.1-3.3, Figure 1).  One
//    persistent cooperative launch runs every time step.  Each workgroup keeps
//    an extended tile -- its owned cells plus a ghost ring k cells deep -- in
//    the VGPR file (two register sets, ping-ponged between steps), advances it
//    k steps without touching HBM, then exchanges the k-deep border strips with
//    the workgroups around it through global memory and per-workgroup epoch
//    flags (bulk-synchronous, Section 3.2; a neighbour-wise form of the grid
//    barrier).  Inside a workgroup the waves are stacked vertically; each step
//    they swap their top and bottom rows through LDS and meet at one s_barrier.
//    East/west neighbours across lanes come from DPP wave shifts.
//
// Arithmetic: with fma == 0 every product is rounded and the sum is taken
// left to right in the order W, E, S, C, N (the printed order of Listing 1);
// with fma == 1 the same chain uses fused multiply-adds.  The library is built
// with -ffp-contract=off so the compiler never fuses on its own.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtb_internal.h"

namespace dtb {

template <typename T>
struct Coef {
    T c, n, s, e, w;
};

template <typename T>
__device__ __forceinline__ Coef<T> load_coef(const double* k)
{
    return Coef<T>{(T)k[0], (T)k[1], (T)k[2], (T)k[3], (T)k[4]};
}

template <bool FMA, typename T>
__device__ __forceinline__ T j2d5pt(T W, T E, T S, T C, T N, const Coef<T>& k)
{
    if constexpr (FMA) {
        T acc = k.w * W;
        acc = __builtin_fma(k.e, E, acc);
        acc = __builtin_fma(k.s, S, acc);
        acc = __builtin_fma(k.c, C, acc);
        acc = __builtin_fma(k.n, N, acc);
        return acc;
    } else {
        T acc = k.w * W;
        acc = acc + k.e * E;
        acc = acc + k.s * S;
        acc = acc + k.c * C;
        acc = acc + k.n * N;
        return acc;
    }
}

// ============================================================================ one-step baseline

// Block: 64 x 4 threads.  Thread (tx, ty) owns column j and STEP_ILP
// consecutive rows; it keeps the column's vertical neighbours in registers
// (the column cache of Listing 1) and reads W/E from memory (cache hits).
constexpr int kStepIlp = 8;

template <typename T, bool FMA>
__global__ __launch_bounds__(256) void k_step(const T* __restrict__ in, T* __restrict__ out,
                                              int64_t pitch, int rows, int cols,
                                              Coef<T> k)
{
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i0 = (blockIdx.y * 4 + threadIdx.y) * kStepIlp + 1;
    if (j > cols || i0 > rows) return;
    T col[kStepIlp + 2];
#pragma unroll
    for (int q = 0; q < kStepIlp + 2; ++q) {
        const int i = i0 - 1 + q;
        col[q] = (i <= rows + 1) ? in[(int64_t)i * pitch + j] : T(0);
    }
#pragma unroll
    for (int q = 0; q < kStepIlp; ++q) {
        const int i = i0 + q;
        if (i <= rows) {
            const T* mid = in + (int64_t)i * pitch;
            out[(int64_t)i * pitch + j] = j2d5pt<FMA>(mid[j - 1], mid[j + 1], col[q], col[q + 1], col[q + 2], k);
        }
    }
}

// Copies the interior of src into dst (used when an odd number of one-step
// launches leaves the result in the workspace).
template <typename T>
__global__ __launch_bounds__(256) void k_copy_interior(const T* __restrict__ src, T* __restrict__ dst,
                                                       int64_t pitch, int rows, int cols)
{
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i = blockIdx.y * 4 + threadIdx.y + 1;
    if (j <= cols && i <= rows) dst[(int64_t)i * pitch + j] = src[(int64_t)i * pitch + j];
}

// ============================================================================ deep temporal blocking

// DPP wave shifts (GFX9 wave_shr:1 / wave_shl:1).  Lanes whose source lane
// does not exist (lane 0 for shr, lane 63 for shl) keep `old`.
template <typename T>
__device__ __forceinline__ T wave_shr1(T old, T v)
{
    return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);
}
template <typename T>
__device__ __forceinline__ T wave_shl1(T old, T v)
{
    return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xf, 0xf, false);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Wrap-safe "counter a has reached b".
__device__ __forceinline__ bool reached(uint32_t a, uint32_t b) { return (int32_t)(a - b) >= 0; }

// Geometry of one kernel instance: C columns x R rows per lane, WAVES waves
// stacked vertically.  Extended tile: (WAVES * R) x (64 * C) cells.
template <typename T, int C, int R, int WAVES>
struct Geo {
    static constexpr int ER = WAVES * R;
    static constexpr int EC = kWaveSize * C;
    // LDS: edge rows [parity][slot = wave + 1][top/bottom][64 * C] and, per
    // extended row, the west/east halo values for lanes 0 and 63.
    static constexpr int kEdgeElems = 2 * (WAVES + 2) * 2 * EC;
    static constexpr int kHaloElems = ER * 2;
    static constexpr size_t kLdsBytes = (size_t)(kEdgeElems + kHaloElems) * sizeof(T);
};

template <typename T, int C, int R, int WAVES, bool FMA, bool COLMASK, bool ROWCHECK>
struct Tile {
    using G = Geo<T, C, R, WAVES>;
    static constexpr int ER = G::ER;
    static constexpr int EC = G::EC;

    T a[R][C];
    T b[R][C];

    T* edge;   // LDS
    T* halo;   // LDS
    int wave, lane;
    int g0;        // storage row of this wave's row 0
    int col0;      // storage column of this lane's slot 0
    bool colact[C];
    Coef<T> k;

    __device__ __forceinline__ T* edge_row(int parity, int slot, int bottom)
    {
        return edge + ((size_t)((parity * (WAVES + 2) + slot) * 2 + bottom)) * EC;
    }

    // One time step: src -> dst.  `parity` selects the LDS edge buffer.
    __device__ __forceinline__ void step(T (&src)[R][C], T (&dst)[R][C], int parity, int rows)
    {
        // Publish this wave's current top and bottom rows for the waves above and below.
        T* mytop = edge_row(parity, wave + 1, 0) + lane * C;
        T* mybot = edge_row(parity, wave + 1, 1) + lane * C;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            mytop[c] = src[0][c];
            mybot[c] = src[R - 1][c];
        }
        __syncthreads();
        T top[C], bot[C];
        const T* above = edge_row(parity, wave, 1) + lane * C;      // bottom row of the wave above
        const T* below = edge_row(parity, wave + 2, 0) + lane * C;  // top row of the wave below
#pragma unroll
        for (int c = 0; c < C; ++c) {
            top[c] = above[c];
            bot[c] = below[c];
        }
        const T* hrow = halo + (size_t)wave * R * 2;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (ROWCHECK) {
                const int g = g0 + r;
                if (g < 1 || g > rows) continue;
            }
            const T hw = hrow[2 * r];
            const T he = hrow[2 * r + 1];
            const T wlane = wave_shr1(hw, src[r][C - 1]);  // west neighbour of slot 0
            const T elane = wave_shl1(he, src[r][0]);      // east neighbour of slot C-1
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T Wv = (c == 0) ? wlane : src[r][c - 1];
                const T Ev = (c == C - 1) ? elane : src[r][c + 1];
                const T Sv = (r == 0) ? top[c] : src[r - 1][c];
                const T Nv = (r == R - 1) ? bot[c] : src[r + 1][c];
                T v = j2d5pt<FMA>(Wv, Ev, Sv, src[r][c], Nv, k);
                if constexpr (COLMASK) v = colact[c] ? v : dst[r][c];
                dst[r][c] = v;
            }
        }
    }

    // The owned cells within k of an owned edge: what the neighbours need.
    __device__ __forceinline__ void publish(T (&x)[R][C], T* __restrict__ xb, int64_t pitch,
                                            const WgDesc& d, int kk)
    {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int g = g0 + r;
            if (g < d.own_r0 || g >= d.own_r1) continue;
            const bool row_near = (g < d.own_r0 + kk) || (g >= d.own_r1 - kk);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int col = col0 + c;
                const bool own = col >= d.own_c0 && col < d.own_c1;
                const bool near = row_near || col < d.own_c0 + kk || col >= d.own_c1 - kk;
                if (own && near) xb[(int64_t)g * pitch + col] = x[r][c];
            }
        }
    }

    // Refresh the ghost ring (cells within k of the owned region, inside the interior, not owned).
    __device__ __forceinline__ void load_ghost(T (&x)[R][C], const T* __restrict__ xb, int64_t pitch,
                                               const WgDesc& d, int kk, int rows, int cols)
    {
        const int r_lo = max(d.own_r0 - kk, 1), r_hi = min(d.own_r1 + kk, rows + 1);
        const int c_lo = max(d.own_c0 - kk, 1), c_hi = min(d.own_c1 + kk, cols + 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int g = g0 + r;
            if (g < r_lo || g >= r_hi) continue;
            const bool row_own = g >= d.own_r0 && g < d.own_r1;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int col = col0 + c;
                const bool in_ring = col >= c_lo && col < c_hi;
                const bool own = row_own && col >= d.own_c0 && col < d.own_c1;
                if (in_ring && !own) x[r][c] = xb[(int64_t)g * pitch + col];
            }
        }
    }

    __device__ __forceinline__ void store_owned(T (&x)[R][C], T* __restrict__ grid, int64_t pitch,
                                                const WgDesc& d)
    {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int g = g0 + r;
            if (g < d.own_r0 || g >= d.own_r1) continue;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int col = col0 + c;
                if (col >= d.own_c0 && col < d.own_c1) grid[(int64_t)g * pitch + col] = x[r][c];
            }
        }
    }
};

// Neighbour-wise bulk-synchronous exchange point.  Every thread's prior global
// stores are released at agent scope, one thread raises this workgroup's
// epoch flag, and the first nnb threads of wave 0 wait (bounded) until each
// neighbour's flag has reached the same epoch.  On timeout the error word is
// set and the wait is abandoned, so the grid always drains.
__device__ __forceinline__ void exchange_point(uint32_t* flags, int me, const WgDesc& d, uint32_t target,
                                               int* err, uint32_t spin_limit)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flags + me, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if ((int)threadIdx.x < d.nnb) {
        const int nb = d.nb[threadIdx.x];
        uint32_t spins = 0;
        while (!reached(__hip_atomic_load(flags + nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), target)) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > spin_limit) {
                __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <typename T, int C, int R, int WAVES, bool FMA, bool COLMASK, bool ROWCHECK>
__device__ __forceinline__ void run_tile(const ProbDesc& P, const WgDesc& d, int me, uint32_t* flags, int* err,
                                         uint32_t spin_limit, char* lds)
{
    using Tl = Tile<T, C, R, WAVES, FMA, COLMASK, ROWCHECK>;
    using G = typename Tl::G;
    Tl t;
    T* grid = (T*)P.grid;
    const int64_t pitch = P.pitch;
    const int rows = P.rows, cols = P.cols;
    const int kk = P.k;
    t.edge = (T*)lds;
    t.halo = (T*)lds + G::kEdgeElems;
    t.wave = uniform(threadIdx.x >> 6);
    t.lane = threadIdx.x & 63;
    t.g0 = d.ext_r0 + t.wave * R;
    t.col0 = d.ext_c0 + t.lane * C;
    t.k = load_coef<T>(P.coeffs);
#pragma unroll
    for (int c = 0; c < C; ++c) t.colact[c] = (t.col0 + c) <= cols;

    // ---- load the extended tile (both register sets) and the fixed boundary values
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int g = t.g0 + r;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int col = t.col0 + c;
            const T v = (g <= rows + 1 && col <= cols + 1) ? grid[(int64_t)g * pitch + col] : T(0);
            t.a[r][c] = v;
            t.b[r][c] = v;
        }
    }
    // Rows just above and below the extended tile (the halo rows for edge tiles), both parities.
    {
        const int gt = d.ext_r0 - 1;
        const int gb = d.ext_r0 + G::ER;
        for (int idx = threadIdx.x; idx < G::EC; idx += WAVES * kWaveSize) {
            const int col = d.ext_c0 + idx;
            const T vt = (col <= cols + 1) ? grid[(int64_t)gt * pitch + col] : T(0);
            const T vb = (gb <= rows + 1 && col <= cols + 1) ? grid[(int64_t)gb * pitch + col] : T(0);
            for (int p = 0; p < 2; ++p) {
                t.edge_row(p, 0, 1)[idx] = vt;
                t.edge_row(p, WAVES + 1, 0)[idx] = vb;
            }
        }
        // Columns just west and east of the extended tile, per extended row.
        for (int idx = threadIdx.x; idx < G::ER; idx += WAVES * kWaveSize) {
            const int g = d.ext_r0 + idx;
            const int cw = d.ext_c0 - 1, ce = d.ext_c0 + G::EC;
            const bool grow = g <= rows + 1;
            t.halo[2 * idx] = (grow && cw >= 0) ? grid[(int64_t)g * pitch + cw] : T(0);
            t.halo[2 * idx + 1] = (grow && ce <= cols + 1) ? grid[(int64_t)g * pitch + ce] : T(0);
        }
    }
    __syncthreads();

    uint32_t base = __hip_atomic_load(flags + me, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t epoch = 0;
    int64_t done = 0;
    bool exchanged = false;
    // The state is in register set a at every epoch boundary: steps go in
    // pairs a -> b -> a (LDS edge parity 0 then 1); an odd tail step is copied
    // back.  A run of k steps is followed by an exchange point (a workgroup
    // barrier), so an odd k never lets two consecutive steps share a parity.
    while (done < P.T) {
        const int64_t left = P.T - done;
        const int nsteps = (int)(left < kk ? left : kk);
        for (int s = 0; s + 1 < nsteps; s += 2) {
            t.step(t.a, t.b, 0, rows);
            t.step(t.b, t.a, 1, rows);
        }
        if (nsteps & 1) {
            t.step(t.a, t.b, 0, rows);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < C; ++c) t.a[r][c] = t.b[r][c];
        }
        done += nsteps;
        if (done < P.T) {
            T* xb = (T*)P.xbuf[epoch & 1];
            t.publish(t.a, xb, pitch, d, kk);
            ++epoch;
            exchange_point(flags, me, d, base + epoch, err, spin_limit);
            exchanged = true;
            t.load_ghost(t.a, xb, pitch, d, kk, rows, cols);
        }
    }
    // Neighbours read their initial ghost ring from the grid; make sure they all
    // have before the owned cells are written back in place.
    if (!exchanged) {
        ++epoch;
        exchange_point(flags, me, d, base + epoch, err, spin_limit);
    }
    t.store_owned(t.a, grid, pitch, d);
}

// LDS for the largest instance a kernel can run.
template <typename T, int C, int R, int WAVES>
__device__ __forceinline__ char* dtb_lds()
{
    __shared__ __attribute__((aligned(16))) char lds[Geo<T, C, R, WAVES>::kLdsBytes];
    return lds;
}

template <typename T, int C, int R, int WAVES, bool FMA, bool COLMASK, bool ROWCHECK>
__global__ __launch_bounds__(WAVES * 64) void k_dtb(ProbDesc P, const WgDesc* __restrict__ wgs,
                                                    uint32_t* flags, int* err, uint32_t spin_limit)
{
    const int me = blockIdx.x;
    const WgDesc& d = wgs[me];
    char* lds = dtb_lds<T, C, R, WAVES>();
    run_tile<T, C, R, WAVES, FMA, COLMASK, ROWCHECK>(P, d, me, flags, err, spin_limit, lds);
}

// Copies the halo ring of src into dst (so a one-step workspace sees the grid's boundary).
template <typename T>
__global__ __launch_bounds__(256) void k_copy_halo(const T* __restrict__ src, T* __restrict__ dst,
                                                   int64_t pitch, int rows, int cols)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const int nrow = cols + 2, ncol = rows;
    if (idx < nrow) {
        dst[idx] = src[idx];
        dst[(int64_t)(rows + 1) * pitch + idx] = src[(int64_t)(rows + 1) * pitch + idx];
    } else if (idx < nrow + ncol) {
        const int64_t i = idx - nrow + 1;
        dst[i * pitch] = src[i * pitch];
        dst[i * pitch + cols + 1] = src[i * pitch + cols + 1];
    }
}

// ============================================================================ host-side launchers

template <typename T>
static hipError_t launch_step_t(bool fma, const void* in, void* out, int64_t pitch, int rows, int cols,
                                const double* coeffs, hipStream_t st)
{
    Coef<T> k{(T)coeffs[0], (T)coeffs[1], (T)coeffs[2], (T)coeffs[3], (T)coeffs[4]};
    dim3 block(64, 4);
    dim3 grid((cols + 63) / 64, (rows + 4 * kStepIlp - 1) / (4 * kStepIlp));
    if (fma) hipLaunchKernelGGL((k_step<T, true>), grid, block, 0, st, (const T*)in, (T*)out, pitch, rows, cols, k);
    else hipLaunchKernelGGL((k_step<T, false>), grid, block, 0, st, (const T*)in, (T*)out, pitch, rows, cols, k);
    return hipGetLastError();
}

hipError_t launch_step(int dtype, bool fma, const void* in, void* out, int64_t pitch, int rows, int cols,
                       const double* coeffs, hipStream_t st)
{
    return dtype == 0 ? launch_step_t<double>(fma, in, out, pitch, rows, cols, coeffs, st)
                      : launch_step_t<float>(fma, in, out, pitch, rows, cols, coeffs, st);
}

hipError_t launch_copy_interior(int dtype, const void* src, void* dst, int64_t pitch, int rows, int cols,
                                hipStream_t st)
{
    dim3 block(64, 4);
    dim3 grid((cols + 63) / 64, (rows + 3) / 4);
    if (dtype == 0) hipLaunchKernelGGL((k_copy_interior<double>), grid, block, 0, st, (const double*)src, (double*)dst, pitch, rows, cols);
    else hipLaunchKernelGGL((k_copy_interior<float>), grid, block, 0, st, (const float*)src, (float*)dst, pitch, rows, cols);
    return hipGetLastError();
}

hipError_t launch_copy_halo(int dtype, const void* src, void* dst, int64_t pitch, int rows, int cols,
                            hipStream_t st)
{
    const int n = cols + 2 + rows;
    dim3 grid((n + 255) / 256);
    if (dtype == 0) hipLaunchKernelGGL((k_copy_halo<double>), grid, dim3(256), 0, st, (const double*)src, (double*)dst, pitch, rows, cols);
    else hipLaunchKernelGGL((k_copy_halo<float>), grid, dim3(256), 0, st, (const float*)src, (float*)dst, pitch, rows, cols);
    return hipGetLastError();
}

// Instantiated DTB kernels: FP64 with 2 columns per lane, FP32 with 4 (16 bytes
// of a row per lane either way), 8 waves per workgroup, R rows per lane.
constexpr int kDtbWaves = 8;

template <typename T, int C, int R>
static const void* pick(bool fma, bool colmask, bool rowcheck)
{
    const int v = (fma ? 4 : 0) | (colmask ? 2 : 0) | (rowcheck ? 1 : 0);
    switch (v) {
    case 0: return (const void*)&k_dtb<T, C, R, kDtbWaves, false, false, false>;
    case 1: return (const void*)&k_dtb<T, C, R, kDtbWaves, false, false, true>;
    case 2: return (const void*)&k_dtb<T, C, R, kDtbWaves, false, true, false>;
    case 3: return (const void*)&k_dtb<T, C, R, kDtbWaves, false, true, true>;
    case 4: return (const void*)&k_dtb<T, C, R, kDtbWaves, true, false, false>;
    case 5: return (const void*)&k_dtb<T, C, R, kDtbWaves, true, false, true>;
    case 6: return (const void*)&k_dtb<T, C, R, kDtbWaves, true, true, false>;
    default: return (const void*)&k_dtb<T, C, R, kDtbWaves, true, true, true>;
    }
}

// Returns the kernel for (dtype, R, variant) or nullptr if not instantiated;
// fills the instance geometry.
const void* dtb_kernel(int dtype, int R, bool fma, bool colmask, bool rowcheck, int* C, int* waves)
{
    *waves = kDtbWaves;
    if (dtype == 0) {
        *C = 2;
        switch (R) {
        case 8: return pick<double, 2, 8>(fma, colmask, rowcheck);
        case 16: return pick<double, 2, 16>(fma, colmask, rowcheck);
        case 24: return pick<double, 2, 24>(fma, colmask, rowcheck);
        default: return nullptr;
        }
    } else {
        *C = 4;
        switch (R) {
        case 8: return pick<float, 4, 8>(fma, colmask, rowcheck);
        case 16: return pick<float, 4, 16>(fma, colmask, rowcheck);
        case 24: return pick<float, 4, 24>(fma, colmask, rowcheck);
        default: return nullptr;
        }
    }
}

}  // namespace dtb
