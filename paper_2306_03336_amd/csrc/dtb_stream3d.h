// dtb_stream3d.h -- the 3-D seven-point stencil (j3d7pt) by 2.5D streaming
// with temporal blocking.
//
// The update: every interior cell of a (depth + 2) x (rows + 2) x pitch grid
// becomes w*W + e*E + s*S + c*C + n*N + b*B + t*T of the previous step's
// values (W/E columns j-1/j+1, S/N rows i-1/i+1, B/T planes z-1/z+1), products
// summed in that order; the one-cell shell around the interior is a fixed
// Dirichlet halo.  This is Listing 1's update with the two neighbours of the
// third axis, repeated T times (Section 3.1, Figure 1); Section 2 names 2.5D
// tiling of 3-D stencils among the related designs.
//
// Design.  A 3-D grid does not fit on chip, so each workgroup owns a column
// of the grid: an (x, y) tile, ER = WAVES * R rows by EC = 64 * C columns,
// over a block of Zb planes, and streams it plane by plane.  One launch
// advances the grid K steps: the workgroup keeps, for every time level l =
// 0 .. K-1, the three most recent planes of that level in registers (the
// "2.5D" window: rows across waves, columns across lanes, planes across
// registers), so that level l+1 of plane q is computed as soon as level l of
// plane q+1 exists.  Level 0 is loaded from HBM (one or two planes ahead, so
// that the loads overlap the compute), level K is stored.  Neighbouring workgroups do
// not synchronise: each tile carries a K-deep ring of redundant cells in x and
// y, and each z-block K planes below and above (overlapped, or trapezoidal,
// blocking in all three axes; stale values from a tile's open edges move one
// cell per level and never reach the owned cells).  Cells outside the interior
// (the halo shell, where a tile meets the grid boundary) keep their values at
// every level.  Within a plane, W/E neighbours come from the neighbouring lane
// (DPP), S/N from the neighbouring row of the same lane or, at a wave's first
// and last row, from the wave above or below through LDS: every level
// publishes its newest plane's edge rows once per plane, and one workgroup
// barrier per plane separates publishing from reading (two LDS buffers,
// alternating).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtb_internal.h"
#include "dtb_stencil.h"

namespace dtb {

// Seven weights; the order of the products is W, E, S, C, N, B, T.
template <typename T>
struct Coef7 {
    T c, n, s, e, w, t, b;
};

template <bool FMA, typename T>
__device__ __forceinline__ T j3d7pt(T W, T E, T S, T Cv, T N, T B, T Tv, const Coef7<T>& k)
{
    T acc = k.w * W;
    if constexpr (FMA) {
        acc = fma_t(k.e, E, acc);
        acc = fma_t(k.s, S, acc);
        acc = fma_t(k.c, Cv, acc);
        acc = fma_t(k.n, N, acc);
        acc = fma_t(k.b, B, acc);
        acc = fma_t(k.t, Tv, acc);
    } else {
        acc = acc + k.e * E;
        acc = acc + k.s * S;
        acc = acc + k.c * Cv;
        acc = acc + k.n * N;
        acc = acc + k.b * B;
        acc = acc + k.t * Tv;
    }
    return acc;
}

template <typename T>
__device__ __forceinline__ T wave_shr1_3(T v)  // lane l gets lane l-1's value (lane 0: 0)
{
    return __builtin_amdgcn_update_dpp((T)0, v, 0x138, 0xf, 0xf, true);
}
template <typename T>
__device__ __forceinline__ T wave_shl1_3(T v)  // lane l gets lane l+1's value (lane 63: 0)
{
    return __builtin_amdgcn_update_dpp((T)0, v, 0x130, 0xf, 0xf, true);
}

// v in the lanes whose bit is set in `mask`, x in the others (one v_cndmask per 32 bits, the mask in SGPRs).
__device__ __forceinline__ uint32_t keep_or32(uint64_t mask, uint32_t x, uint32_t v)
{
    uint32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(v), "s"(mask));
    return r;
}
__device__ __forceinline__ float keep_or(uint64_t mask, float x, float v)
{
    return __builtin_bit_cast(float, keep_or32(mask, __builtin_bit_cast(uint32_t, x), __builtin_bit_cast(uint32_t, v)));
}
__device__ __forceinline__ double keep_or(uint64_t mask, double x, double v)
{
    const uint64_t xb = __builtin_bit_cast(uint64_t, x), vb = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = keep_or32(mask, (uint32_t)xb, (uint32_t)vb);
    const uint32_t hi = keep_or32(mask, (uint32_t)(xb >> 32), (uint32_t)(vb >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <typename T, int C, int R, int K, int WAVES>
struct Stream3Geo {
    static constexpr int ER = WAVES * R;
    static constexpr int EC = 64 * C;
    // LDS: [parity 2][level K][wave][top/bottom 2][EC], then one row of zeros:
    // what the first wave reads above its first row and the last wave below
    // its last row (the tile's open edges; any value would do, since stale
    // values there never reach the owned cells).
    static constexpr size_t kEdgeElems = (size_t)2 * K * WAVES * 2 * EC;
    static constexpr size_t kLdsBytes = (kEdgeElems + EC) * sizeof(T);
};

// The register pipeline of one workgroup.
template <typename T, int C, int R, int K, int WAVES, bool FMA, bool EDGE, int PF>
struct Stream3 {
    using G = Stream3Geo<T, C, R, K, WAVES>;
    using Elem = T;
    static constexpr int kC = C, kR = R, kK = K, kWaves = WAVES, kPF = PF;
    T win[K][3][R][C];   // level l's three most recent planes (slot: the plane's offset from the first, mod 3)
    T next[PF][R][C];    // the level-0 planes being loaded 1 .. PF iterations ahead
    Coef7<T> k;
    T* lds;
    int wave, lane;
    int g0;              // storage row of this wave's row 0
    int col0;            // storage column of this lane's slot 0
    bool rowact[R];      // EDGE: row inside the interior (uniform over the wave)
    uint64_t colact[C];  // EDGE: the lanes whose column c is inside the interior (a wave-wide mask)
    bool rowown[R];      // row owned by this tile (stored)
    bool colown[C];      // column owned by this tile
    bool allown;         // all C columns owned

    __device__ __forceinline__ T* edge_row(int parity, int level, int w, int bottom)
    {
        return lds + ((size_t)(((parity * K + level) * WAVES + w) * 2 + bottom)) * G::EC;
    }
    __device__ __forceinline__ const T* zero_row() const { return lds + G::kEdgeElems; }

    // Load plane z of the source (cells outside the stored grid read as 0).
    __device__ __forceinline__ void load_plane(const T* src, const Stream3Args& A, int z, T (&dst)[R][C])
    {
        const T* plane = src + (int64_t)z * A.plane_pitch;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int g = g0 + r;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int col = col0 + c;
                T v = T(0);
                if (!EDGE || (g <= A.rows + 1 && col <= A.cols + 1)) v = plane[(int64_t)g * A.pitch + col];
                dst[r][c] = v;
            }
        }
    }

    // Publish a plane's first and last rows for the waves above and below.
    __device__ __forceinline__ void publish(int parity, int level, const T (&x)[R][C])
    {
        T* top = edge_row(parity, level, wave, 0);
        T* bot = edge_row(parity, level, wave, 1);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            top[c * 64 + lane] = x[0][c];
            bot[c * 64 + lane] = x[R - 1][c];
        }
    }

    // Store the owned cells of plane q (level K) to the destination.
    __device__ __forceinline__ void store_plane(T* dst, const Stream3Args& A, int q, const T (&out)[R][C])
    {
        T* plane = dst + (int64_t)q * A.plane_pitch;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!rowown[r]) continue;  // uniform over the wave
            T* row = plane + (int64_t)(g0 + r) * A.pitch + col0;
            if (allown) {
                // every cell of the lane owned: one wide store of its C cells (aligned to the element only: the
                // hardware takes unaligned wide accesses to global memory)
                typedef T Vec __attribute__((ext_vector_type(C), aligned(sizeof(T))));
                Vec v;
#pragma unroll
                for (int c = 0; c < C; ++c) v[c] = out[r][c];
                *(Vec*)row = v;
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (colown[c]) row[c] = out[r][c];
            }
        }
    }

    // Level `level` + 1 of plane q from level `level`'s planes q-1 (bw), q (cw), q+1 (aw): writes out.
    // above/below: the neighbouring waves' edge rows of plane q (zeros at the tile's first / last row).
    __device__ __forceinline__ void compute(const T (&bw)[R][C], const T (&cw)[R][C], const T (&aw)[R][C],
                                            const T (&above)[C], const T (&below)[C], bool plane_interior,
                                            T (&out)[R][C])
    {
        if (!plane_interior) {  // a halo plane (uniform): it keeps its values at every level
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < C; ++c) out[r][c] = cw[r][c];
            return;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T wl = wave_shr1_3(cw[r][C - 1]);
            const T el = wave_shl1_3(cw[r][0]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T W = c == 0 ? wl : cw[r][c - 1];
                const T E = c == C - 1 ? el : cw[r][c + 1];
                const T S = r == 0 ? above[c] : cw[r - 1][c];
                const T N = r == R - 1 ? below[c] : cw[r + 1][c];
                T v = j3d7pt<FMA>(W, E, S, cw[r][c], N, bw[r][c], aw[r][c], k);
                // Cells outside the interior keep their value: one select by a scalar lane mask, no branch.
                if constexpr (EDGE) v = keep_or(rowact[r] ? colact[c] : 0ull, cw[r][c], v);
                out[r][c] = v;
            }
        }
    }
};

// Slot of plane p0 + Um + u - l in a level's three-slot window (U a multiple of 3; u, l known at compile time
// after unrolling).
__host__ __device__ constexpr int stream_slot(int u, int l) { return ((u - l) % 3 + 3) % 3; }

// U iterations of the streaming loop from iteration pb (see stream3_run).  FAST: every iteration of the
// block has its level-0 plane and the plane PF ahead to load (pb + U + PF <= p_end), and every level
// produces a plane of the interior inside its range (pb >= zo0 + K, so p - K >= zo0 >= 1; and p <= p_end -
// PF - 1 with p_end <= depth + 2, so p - 1 <= depth - 1): the conditions below are then all true and
// compiled out.
template <bool FAST, int U, typename S3>
__device__ __forceinline__ void stream3_block(S3& s, const Stream3Args& A, const typename S3::Elem* src,
                                              typename S3::Elem* dst, int pb, int p_end, int p_stop, int zo0,
                                              int zo1)
{
    using T = typename S3::Elem;
    constexpr int C = S3::kC, R = S3::kR, K = S3::kK, WAVES = S3::kWaves, PF = S3::kPF;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int p = pb + u;
        if constexpr (!FAST) {
            if (p >= p_stop) break;
        }
        // Keep the scheduler from interleaving iterations of the branch-free block (its live ranges would no
        // longer fit the register file).
        __builtin_amdgcn_sched_barrier(0);
        const int par = p & 1;
        if (FAST || p < p_end) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < C; ++c) s.win[0][stream_slot(u, 0)][r][c] = s.next[u % PF][r][c];
            if (FAST || p + PF < p_end) s.load_plane(src, A, p + PF, s.next[u % PF]);
        }
        // The centre planes' edge rows were published last iteration (the other LDS buffer).
        __syncthreads();
#pragma unroll
        for (int l = 1; l <= K; ++l) {
            const int q = p - l;
            if constexpr (!FAST) {
                const int lo = zo0 - K + l > 0 ? zo0 - K + l : 0;
                const int hi = zo1 + K - l < A.depth + 2 ? zo1 + K - l : A.depth + 2;
                if (q < lo || q >= hi) continue;
            }
            // The neighbouring waves' edge rows of plane q at level l - 1 (the zero row past the tile's
            // first and last rows: a scalar choice of address, no per-lane select).
            const T* ab = s.wave > 0 ? s.edge_row(par ^ 1, l - 1, s.wave - 1, 1) : s.zero_row();
            const T* be = s.wave < WAVES - 1 ? s.edge_row(par ^ 1, l - 1, s.wave + 1, 0) : s.zero_row();
            T above[C], below[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                above[c] = ab[c * 64 + s.lane];
                below[c] = be[c * 64 + s.lane];
            }
            const bool interior = FAST || (q >= 1 && q <= A.depth);
            if (l < K) {
                s.compute(s.win[l - 1][stream_slot(u, l + 1)], s.win[l - 1][stream_slot(u, l)],
                          s.win[l - 1][stream_slot(u, l - 1)], above, below, interior, s.win[l][stream_slot(u, l)]);
            } else {
                T out[R][C];
                s.compute(s.win[l - 1][stream_slot(u, l + 1)], s.win[l - 1][stream_slot(u, l)],
                          s.win[l - 1][stream_slot(u, l - 1)], above, below, interior, out);
                s.store_plane(dst, A, q, out);
            }
        }
        // Publish every level's newest plane (the centre planes of the next iteration).
#pragma unroll
        for (int l = 0; l < K; ++l) s.publish(par, l, s.win[l][stream_slot(u, l)]);
    }
}

// One K-step launch of one workgroup: tile `d`, owned planes [zo0, zo1).
// PF: planes loaded ahead (1 or 2).  Measured at 512^3 with the branch-free steady state: swapping the
// depths (FP64 two, FP32 one) lost in both (FP64 682 -> 678, FP32 893 -> 879 GCells/s), so FP32 loads two
// planes ahead and FP64, whose three levels of eight cells per lane leave fewer free registers, one.
template <typename T, int C, int R, int K, int WAVES, bool FMA, bool EDGE, int PF = (sizeof(T) == 4 ? 2 : 1)>
__device__ __forceinline__ void stream3_run(const Stream3Args& A, const Tile3Desc& d, int zo0, int zo1, T* lds)
{
    static_assert(PF == 1 || PF == 2, "one or two planes ahead");
    Stream3<T, C, R, K, WAVES, FMA, EDGE, PF> s;
    s.lds = lds;
    s.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    s.lane = threadIdx.x & 63;
    s.g0 = d.ext_r0 + s.wave * R;
    s.col0 = d.ext_c0 + s.lane * C;
    s.k = Coef7<T>{(T)A.coeffs[0], (T)A.coeffs[1], (T)A.coeffs[2], (T)A.coeffs[3],
                   (T)A.coeffs[4], (T)A.coeffs[5], (T)A.coeffs[6]};
#pragma unroll
    for (int r = 0; r < R; ++r) s.rowact[r] = s.g0 + r >= 1 && s.g0 + r <= A.rows;
#pragma unroll
    for (int c = 0; c < C; ++c) s.colact[c] = __builtin_amdgcn_ballot_w64(s.col0 + c >= 1 && s.col0 + c <= A.cols);
#pragma unroll
    for (int r = 0; r < R; ++r) s.rowown[r] = s.g0 + r >= d.own_r0 && s.g0 + r < d.own_r1;
#pragma unroll
    for (int c = 0; c < C; ++c) s.colown[c] = s.col0 + c >= d.own_c0 && s.col0 + c < d.own_c1;
    s.allown = s.col0 >= d.own_c0 && s.col0 + C <= d.own_c1;
    const T* src = (const T*)A.src;
    T* dst = (T*)A.dst;
    // Level 0 (loaded) covers planes [p0, p_end); level l covers [lo(l), hi(l)), one plane less on each
    // side per level, clipped to the stored planes 0 .. depth + 1; level K is [zo0, zo1).
    const int p0 = zo0 - K > 0 ? zo0 - K : 0;
    const int p_end = zo1 + K < A.depth + 2 ? zo1 + K : A.depth + 2;
    s.load_plane(src, A, p0, s.next[0]);
    if constexpr (PF == 2) {
        if (p0 + 1 < p_end) s.load_plane(src, A, p0 + 1, s.next[1]);
    }
    // The zero row (read by the outermost waves) is visible after the first
    // barrier of the loop, before any read.
    using G = Stream3Geo<T, C, R, K, WAVES>;
    for (int i = threadIdx.x; i < G::EC; i += WAVES * 64) lds[G::kEdgeElems + i] = T(0);
    // Iteration p: level 0 takes plane p, level l = 1 .. K produces plane p - l (when it has one); the
    // last owned plane, zo1 - 1, leaves level K at iteration zo1 - 1 + K.
    // Unrolled by three (six with two prefetch buffers): window slots repeat every three planes.  Blocks of
    // iterations in which every one loads its plane and the plane PF ahead, and every level produces an
    // interior plane, run without any of the per-iteration conditions (stream3_block<true>): no branches,
    // so the window stays in place (no register copies at branch joins) and the loads are counted exactly.
    // They form one run in the middle of the z-block (the conditions hold from pb = zo0 + K until
    // pb + U + PF > p_end), with the general form before and after it, each in a loop of its own.
    constexpr int U = PF == 2 ? 6 : 3;
    const int p_stop = zo1 + K;
    int pb = p0;
    for (; pb < p_stop && pb < zo0 + K; pb += U) stream3_block<false, U>(s, A, src, dst, pb, p_end, p_stop, zo0, zo1);
    for (; pb + U + PF <= p_end; pb += U) stream3_block<true, U>(s, A, src, dst, pb, p_end, p_stop, zo0, zo1);
    for (; pb < p_stop; pb += U) stream3_block<false, U>(s, A, src, dst, pb, p_end, p_stop, zo0, zo1);
}

// The K-step streaming kernel.  Workgroup b: tile b % ntiles, z-block b / ntiles.
template <typename T, int C, int R, int K, int WAVES, bool FMA>
__global__ __launch_bounds__(WAVES * 64, 1) void k_stream3d(Stream3Args A, const Tile3Desc* __restrict__ tiles)
{
    using G = Stream3Geo<T, C, R, K, WAVES>;
    __shared__ __attribute__((aligned(16))) char lds_raw[G::kLdsBytes];
    const Tile3Desc d = tiles[blockIdx.x % A.ntiles];
    const int zblk = blockIdx.x / A.ntiles;
    const int zo0 = 1 + zblk * A.zb;
    const int zo1 = zo0 + A.zb < A.depth + 1 ? zo0 + A.zb : A.depth + 1;
    if (d.edge) stream3_run<T, C, R, K, WAVES, FMA, true>(A, d, zo0, zo1, (T*)lds_raw);
    else stream3_run<T, C, R, K, WAVES, FMA, false>(A, d, zo0, zo1, (T*)lds_raw);
}

}  // namespace dtb
