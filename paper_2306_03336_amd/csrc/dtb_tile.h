// dtb_tile.h -- device templates of the deep-temporal-blocking kernels
// (register tile, steps, exchange, sweep); instantiated per (precision,
// rows per lane) in the dtb_inst_*.hip translation units.
//
// The update (Listing 1 of Zhang et al., GPGPU '23): every interior cell
// becomes w*W + e*E + s*S + c*C + n*N of the previous step's values, with
// W = (i, j-1), E = (i, j+1), S = (i-1, j), N = (i+1, j) (x = column j is the
// contiguous index, y = row i).  Reads and writes never alias within a step
// (Jacobi).  The one-cell ring around the interior is a fixed Dirichlet halo.
//
// The kernels here:
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
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dtb_internal.h"
#include "dtb_launch.h"
#include "dtb_stencil.h"

namespace dtb {

// ============================================================================ deep temporal blocking

// Border strips travel between workgroups with device-scope (sc1) relaxed
// atomic stores and loads, which are coherent across XCDs without an L2
// write-back or invalidate; their order is enforced by s_waitcnt at the
// exchange point.
template <typename T>
__device__ __forceinline__ void xchg_store(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T xchg_load(T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// DPP wave shifts (GFX9 wave_shr:1 / wave_shl:1) with bound_ctrl: a lane
// whose source lane does not exist (lane 0 for shr, lane 63 for shl) reads 0.
template <typename T>
__device__ __forceinline__ T wave_shr1(T v)
{
    return __builtin_amdgcn_update_dpp((T)0, v, 0x138, 0xf, 0xf, true);
}
template <typename T>
__device__ __forceinline__ T wave_shl1(T v)
{
    return __builtin_amdgcn_update_dpp((T)0, v, 0x130, 0xf, 0xf, true);
}

// The same shifts without bound_ctrl: the lane without a source lane keeps
// `old` (lane 0 for shr, lane 63 for shl) -- how the box stencil's edge lanes
// receive the west/east halo.
template <typename T>
__device__ __forceinline__ T wave_shr1_or(T old, T v)
{
    return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);
}
template <typename T>
__device__ __forceinline__ T wave_shl1_or(T old, T v)
{
    return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xf, 0xf, false);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Per-lane choice without a branch: lanes whose bit is set in `mask` (a
// wave-wide lane mask) get v, the others keep x.  Written as v_cndmask so the
// compiler cannot turn it into a branch around the instruction producing v
// (which for an LDS load would then wait on every one).
__device__ __forceinline__ uint32_t lane_pick32(uint64_t mask, uint32_t x, uint32_t v)
{
    uint32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(v), "s"(mask));
    return r;
}
__device__ __forceinline__ float lane_pick(uint64_t mask, float x, float v)
{
    return __builtin_bit_cast(float, lane_pick32(mask, __builtin_bit_cast(uint32_t, x), __builtin_bit_cast(uint32_t, v)));
}
__device__ __forceinline__ double lane_pick(uint64_t mask, double x, double v)
{
    const uint64_t xb = __builtin_bit_cast(uint64_t, x), vb = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = lane_pick32(mask, (uint32_t)xb, (uint32_t)vb);
    const uint32_t hi = lane_pick32(mask, (uint32_t)(xb >> 32), (uint32_t)(vb >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Wrap-safe "counter a has reached b".
__device__ __forceinline__ bool reached(uint32_t a, uint32_t b) { return (int32_t)(a - b) >= 0; }

// The update with the west and east products given an addend: lane 0 of a
// west-edge tile reads W = 0 from the shift and gets the halo product w*hW
// as the addend of its first product; lane 63 of an east-edge tile likewise
// gets e*hE.  Everywhere else the addends are 0, so fma(w, W, 0) is just the
// rounded product and both modes keep their operation order:
//   FMA:   acc = fma(w, W, bw + be); then e, s, c, n by fused multiply-adds;
//   exact: acc = fma(w, W, bw); p = fma(e, E, be); acc += p; acc += s*S; acc += c*C; acc += n*N.
template <bool FMA, bool BW, bool BE, typename T>
__device__ __forceinline__ T j2d5pt_edge(T W, T E, T S, T C, T N, T bw, T be, T bwe, const Coef<T>& k)
{
    if constexpr (FMA) {
        T acc;
        if constexpr (BW && BE) acc = fma_t(k.w, W, bwe);
        else if constexpr (BW) acc = fma_t(k.w, W, bw);
        else if constexpr (BE) acc = fma_t(k.w, W, be);
        else acc = k.w * W;
        acc = fma_t(k.e, E, acc);
        acc = fma_t(k.s, S, acc);
        acc = fma_t(k.c, C, acc);
        acc = fma_t(k.n, N, acc);
        return acc;
    } else {
        T acc;
        if constexpr (BW) acc = fma_t(k.w, W, bw);
        else acc = k.w * W;
        T pe;
        if constexpr (BE) pe = fma_t(k.e, E, be);
        else pe = k.e * E;
        acc = acc + pe;
        acc = acc + k.s * S;
        acc = acc + k.c * C;
        acc = acc + k.n * N;
        return acc;
    }
}

// Geometry of one kernel instance: C columns x R rows per lane, WAVES waves
// stacked vertically.  Extended tile: (WAVES * R) x (64 * C) cells.
template <typename T, int C, int R, int WAVES>
struct Geo {
    static constexpr int ER = WAVES * R;
    static constexpr int EC = kWaveSize * C;
    // LDS: edge rows [parity][slot = wave + 1][top/bottom][64 * C], then per
    // extended row the west and east halo products (w*hW, e*hE) and a row of
    // zeros (what every other lane reads on the row-by-row halo path) -- for
    // the box stencil the halo values themselves, of the rows -1 .. ER.
    static constexpr int kEdgeElems = 2 * (WAVES + 2) * 2 * EC;
    // West/east halo values of the ER + 2 rows a tile's box stencil reaches (three
    // slots; the 5-point stencil uses three of ER), rounded up to 16 bytes so
    // that the staging area after it stays 16-byte aligned.
    static constexpr int kHaloElems = ((ER + 2) * 3 * (int)sizeof(T) + 15) / 16 * 16 / (int)sizeof(T);
    // Exchange staging area for rings up to kStageK deep (deeper rings take
    // the direct per-lane path): a block of up to 2 * kStageK full-width rows
    // (EC cells each) and a block of ER side rows (kSide left cells, then
    // kSide right cells each).
    static constexpr bool kStaged = tile_stages(R, C, (int)sizeof(T));
    static constexpr int kStageK = stage_k(R);
    static constexpr int kSide = kStageK <= 8 ? 8 : 16;
    static constexpr int kStageRows = 2 * kStageK * EC;
    static constexpr int kStageElems = kStaged ? kStageRows + ER * 2 * kSide : 0;
    // ... followed by one spare slot per lane (see stage_cells).
    static constexpr int kStageSpare = kStaged ? kWaveSize : 0;
    static constexpr size_t kLdsBytes = (size_t)(kEdgeElems + kHaloElems + kStageElems + kStageSpare) * sizeof(T);
};

// What one exchange moves, laid out for the LDS staging area: the full-width
// rows [n0, n1) and [s0, s1) over the columns [c0, c1) (each stored as a whole
// tile row of EC cells), then the side rows [m0, m1) over the columns
// [w0, w1) (left part) and [e0, e1) (right part).
// The rim a tile publishes is its owned cells within k of an owned edge; the
// ring it loads is the cells within k of its owned region, inside its
// computed region, that it does not own.
struct StageMap {
    int n0, n1, s0, s1, c0, c1;
    int m0, m1, w0, w1, e0, e1;
    int tc0;  // c0 - the tile's first column: full rows are stored by tile column
};

__device__ __forceinline__ StageMap rim_map(const WgDesc& d, int kk)
{
    StageMap m;
    m.n0 = d.own_r0;
    m.n1 = min(d.own_r0 + kk, d.own_r1);
    m.s0 = max(d.own_r1 - kk, m.n1);
    m.s1 = d.own_r1;
    m.c0 = d.own_c0;
    m.c1 = d.own_c1;
    m.m0 = m.n1;
    m.m1 = m.s0;
    m.w0 = d.own_c0;
    m.w1 = min(d.own_c0 + kk, d.own_c1);
    m.e0 = max(d.own_c1 - kk, m.w1);
    m.e1 = d.own_c1;
    m.tc0 = m.c0 - d.ext_c0;
    return m;
}

__device__ __forceinline__ StageMap ring_map(const WgDesc& d, int kk)
{
    StageMap m;
    m.n0 = max(d.own_r0 - kk, d.cr_r0);
    m.n1 = d.own_r0;
    m.s0 = d.own_r1;
    m.s1 = min(d.own_r1 + kk, d.cr_r1);
    m.c0 = max(d.own_c0 - kk, d.cr_c0);
    m.c1 = min(d.own_c1 + kk, d.cr_c1);
    m.m0 = d.own_r0;
    m.m1 = d.own_r1;
    m.w0 = m.c0;
    m.w1 = d.own_c0;
    m.e0 = d.own_c1;
    m.e1 = m.c1;
    m.tc0 = m.c0 - d.ext_c0;
    return m;
}

template <typename T, int C, int R, int WAVES, bool FMA, bool COLMASK, bool ROWCHECK, int PTS = 5>
struct Tile {
    using G = Geo<T, C, R, WAVES>;
    static constexpr int kPts = PTS;  // 5: j2d5pt (Listing 1); 9: j2d9pt, the 3 x 3 box
    static constexpr int ER = G::ER;
    static constexpr int EC = G::EC;
    static constexpr int kWaves = WAVES;
    static constexpr bool kColmask = COLMASK;
    // Some cells are never written by a step (those outside the grid).
    static constexpr bool kKeepsCells = COLMASK || ROWCHECK;
    using LdsT = __attribute__((address_space(3))) T;  // a cell addressed by its LDS byte address

    T a[R][C];
    T b[R][C];

    T* edge;         // LDS edge rows
    T* stage;        // LDS exchange staging area (Geo::kStageElems)
    const T* hbw;    // LDS, per lane: the west products (lane 0) or zeros
    const T* hbe;    // LDS, per lane: the east products (lane 63) or zeros
    const T* hbwe;   // LDS, per lane: lane 0 west, lane 63 east, zeros elsewhere
    int wave, lane;
    int g0;          // storage row of this wave's row 0
    int col0;        // storage column of this lane's slot 0
    bool colact[C];
    std::conditional_t<PTS == 9, Coef9<T>, Coef<T>> k;
    T bw, be, bwe;   // halo addends when they are the same for every row (box: the halo values of lanes 0 / 63)

    __device__ __forceinline__ T* edge_row(int parity, int slot, int bottom)
    {
        return edge + ((size_t)((parity * (WAVES + 2) + slot) * 2 + bottom)) * EC;
    }

    // Position of (lane, column slot c) in an edge row: 16-byte groups, lane
    // fastest, so that each 16-byte LDS access of a wave covers one
    // contiguous kilobyte (no bank conflicts when a lane holds more than 16
    // bytes of a row, as FP64 with 4 columns does).
    static constexpr int kVec = 16 / (int)sizeof(T) < C ? 16 / (int)sizeof(T) : C;
    __device__ __forceinline__ static int edge_pos(int ln, int c)
    {
        return ((c / kVec) * kWaveSize + ln) * kVec + c % kVec;
    }

    // One time step: src -> dst.  `parity` selects the LDS edge buffer.
    // HALO_ROWS: the halo addends change from row to row (an edge tile of a
    // grid whose west/east halo is not constant) and are read from LDS.
    template <bool HALO_ROWS>
    __device__ __forceinline__ void step(T (&src)[R][C], T (&dst)[R][C], int parity, int rows)
    {
        static_assert(R >= 2, "a wave holds at least two rows");
        if constexpr (PTS == 9) step9<HALO_ROWS>(src, dst, parity, rows);
        else step5<HALO_ROWS>(src, dst, parity, rows);
    }

    // One j2d5pt step (Listing 1's update on every cell of the register tile).
    template <bool HALO_ROWS>
    __device__ __forceinline__ void step5(T (&src)[R][C], T (&dst)[R][C], int parity, int rows)
    {
        // Publish this wave's current top and bottom rows for the waves above and below.
        T* mytop = edge_row(parity, wave + 1, 0);
        T* mybot = edge_row(parity, wave + 1, 1);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            mytop[edge_pos(lane, c)] = src[0][c];
            mybot[edge_pos(lane, c)] = src[R - 1][c];
        }
        __builtin_amdgcn_sched_barrier(0);  // the stores issue first
        // Rows 1 .. R-2 need only this wave's cells: the first ones go
        // before the barrier (covering the LDS stores above), the rest after
        // it (covering the loads of the neighbours' rows), and the first and
        // last rows come last.
        T top[C], bot[C];
        // Inner rows [1, kHalf) go before the barrier.  Measured: the 12-row
        // tile (FP64, 4 columns) is fastest with just one row there (an early
        // barrier lets less wave skew build up in front of it; 2195 -> 2213
        // GCells/s at 2048^2), the 24-row tiles with half of their rows
        // (one row there costs them 1 %).
        constexpr int kHalf = R == 12 ? 2 : R / 2;
#pragma unroll
        for (int r = 1; r < kHalf; ++r) any_row<HALO_ROWS>(src, dst, r, top, bot, rows);
        __syncthreads();
        const T* above = edge_row(parity, wave, 1);      // bottom row of the wave above
        const T* below = edge_row(parity, wave + 2, 0);  // top row of the wave below
#pragma unroll
        for (int c = 0; c < C; ++c) {
            top[c] = above[edge_pos(lane, c)];
            bot[c] = below[edge_pos(lane, c)];
        }
        __builtin_amdgcn_sched_barrier(0);  // the loads issue before the rows that do not need them
#pragma unroll
        for (int r = kHalf; r < R - 1; ++r) any_row<HALO_ROWS>(src, dst, r, top, bot, rows);
        any_row<HALO_ROWS>(src, dst, 0, top, bot, rows);
        any_row<HALO_ROWS>(src, dst, R - 1, top, bot, rows);
    }

    template <bool HALO_ROWS>
    __device__ __forceinline__ void any_row(T (&src)[R][C], T (&dst)[R][C], int r, const T (&top)[C],
                                            const T (&bot)[C], int rows)
    {
        row<HALO_ROWS>(src, dst, r, top, bot, rows);
    }

    // West/east halo value a lane's row shifts fall back to, of the storage row
    // at halo index q (rows ext_r0 - 1 .. ext_r0 + ER): lane 0 of a west-edge
    // tile and lane 63 of an east-edge tile get the halo, every other lane 0.
    template <bool HALO_ROWS>
    __device__ __forceinline__ T halo_w(int q) const { return HALO_ROWS ? hbw[q] : bw; }
    template <bool HALO_ROWS>
    __device__ __forceinline__ T halo_e(int q) const { return HALO_ROWS ? hbe[q] : be; }

    // One box-stencil step: src -> dst.  Same schedule as step() (edge rows
    // published first, inner rows around the barrier, the wave's first and
    // last rows last), but every source row's west and east lane shifts are
    // taken once and shared by the three output rows that read them: two
    // shifts per source row instead of six per output row.
    template <bool HALO_ROWS>
    __device__ __forceinline__ void step9(T (&src)[R][C], T (&dst)[R][C], int parity, int rows)
    {
        T* mytop = edge_row(parity, wave + 1, 0);
        T* mybot = edge_row(parity, wave + 1, 1);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            mytop[edge_pos(lane, c)] = src[0][c];
            mybot[edge_pos(lane, c)] = src[R - 1][c];
        }
        __builtin_amdgcn_sched_barrier(0);  // the stores issue first
        const int q0 = wave * R + 1;  // halo index of this wave's row 0
        T xw[R], xe[R];               // per source row: west neighbour of slot 0, east neighbour of slot C-1
#pragma unroll
        for (int q = 0; q < R; ++q) {
            xw[q] = wave_shr1_or(halo_w<HALO_ROWS>(q0 + q), src[q][C - 1]);
            xe[q] = wave_shl1_or(halo_e<HALO_ROWS>(q0 + q), src[q][0]);
        }
        constexpr int kHalf = R / 2;
#pragma unroll
        for (int r = 1; r < kHalf; ++r)
            box_row(src[r - 1], xw[r - 1], xe[r - 1], src[r], xw[r], xe[r], src[r + 1], xw[r + 1], xe[r + 1], dst[r],
                    r, rows);
        __syncthreads();
        const T* above = edge_row(parity, wave, 1);      // bottom row of the wave above
        const T* below = edge_row(parity, wave + 2, 0);  // top row of the wave below
        T top[C], bot[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            top[c] = above[edge_pos(lane, c)];
            bot[c] = below[edge_pos(lane, c)];
        }
        __builtin_amdgcn_sched_barrier(0);  // the loads issue before the rows that do not need them
#pragma unroll
        for (int r = kHalf; r < R - 1; ++r)
            box_row(src[r - 1], xw[r - 1], xe[r - 1], src[r], xw[r], xe[r], src[r + 1], xw[r + 1], xe[r + 1], dst[r],
                    r, rows);
        const T tw = wave_shr1_or(halo_w<HALO_ROWS>(q0 - 1), top[C - 1]);
        const T te = wave_shl1_or(halo_e<HALO_ROWS>(q0 - 1), top[0]);
        box_row(top, tw, te, src[0], xw[0], xe[0], src[1], xw[1], xe[1], dst[0], 0, rows);
        const T dw = wave_shr1_or(halo_w<HALO_ROWS>(q0 + R), bot[C - 1]);
        const T de = wave_shl1_or(halo_e<HALO_ROWS>(q0 + R), bot[0]);
        box_row(src[R - 2], xw[R - 2], xe[R - 2], src[R - 1], xw[R - 1], xe[R - 1], bot, dw, de, dst[R - 1], R - 1,
                rows);
    }

    // Row r of one box-stencil step: the three source rows s (r-1), m (r), n
    // (r+1) with their west/east lane neighbours; the nine products in the
    // weights' order (sw, s, se, w, c, e, nw, n, ne), as the oracle sums them.
    __device__ __forceinline__ void box_row(const T (&sr)[C], T sW, T sE, const T (&mr)[C], T mW, T mE,
                                            const T (&nr)[C], T nW, T nE, T (&out)[C], int r, int rows)
    {
        if constexpr (ROWCHECK) {
            const int g = g0 + r;
            if (g < 1 || g > rows) return;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const T a[9] = {c == 0 ? sW : sr[c - 1], sr[c], c == C - 1 ? sE : sr[c + 1],
                            c == 0 ? mW : mr[c - 1], mr[c], c == C - 1 ? mE : mr[c + 1],
                            c == 0 ? nW : nr[c - 1], nr[c], c == C - 1 ? nE : nr[c + 1]};
            T v = j2d9pt<FMA>(a, k);
            if constexpr (COLMASK) v = colact[c] ? v : out[c];
            out[c] = v;
        }
        if constexpr (sizeof(T) == 4 && R > 8) {
            if (r % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
    }

    // Row r of one step: src -> dst.  top / bot are the neighbouring waves'
    // rows (read only by rows 0 and R-1).
    template <bool HALO_ROWS>
    __device__ __forceinline__ void row(T (&src)[R][C], T (&dst)[R][C], int r, const T (&top)[C], const T (&bot)[C],
                                        int rows)
    {
        if constexpr (ROWCHECK) {
            const int g = g0 + r;
            if (g < 1 || g > rows) return;
        }
        T rbw = bw, rbe = be, rbwe = bwe;
        if constexpr (HALO_ROWS) {
            rbw = hbw[wave * R + r];
            rbe = hbe[wave * R + r];
            rbwe = hbwe[wave * R + r];
        }
        const T wlane = wave_shr1(src[r][C - 1]);  // west neighbour of slot 0
        const T elane = wave_shl1(src[r][0]);      // east neighbour of slot C-1
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const T Wv = (c == 0) ? wlane : src[r][c - 1];
            const T Ev = (c == C - 1) ? elane : src[r][c + 1];
            const T Sv = (r == 0) ? top[c] : src[r - 1][c];
            const T Nv = (r == R - 1) ? bot[c] : src[r + 1][c];
            T v;
            if (c == 0 && c == C - 1)
                v = j2d5pt_edge<FMA, true, true>(Wv, Ev, Sv, src[r][c], Nv, rbw, rbe, rbwe, k);
            else if (c == 0)
                v = j2d5pt_edge<FMA, true, false>(Wv, Ev, Sv, src[r][c], Nv, rbw, rbe, rbwe, k);
            else if (c == C - 1)
                v = j2d5pt_edge<FMA, false, true>(Wv, Ev, Sv, src[r][c], Nv, rbw, rbe, rbwe, k);
            else
                v = j2d5pt_edge<FMA, false, false>(Wv, Ev, Sv, src[r][c], Nv, rbw, rbe, rbwe, k);
            if constexpr (COLMASK) v = colact[c] ? v : dst[r][c];
            dst[r][c] = v;
        }
        // The row-by-row halo path is rare (edge tiles with a varying halo);
        // keep the scheduler from hoisting every row's LDS reads, which would
        // cost a register pair per row.
        if constexpr (HALO_ROWS) __builtin_amdgcn_sched_barrier(0);
        // Tall FP32 tiles (more than 16 rows of 4 columns) leave no registers
        // for the scheduler to run ahead over many rows: fence it every four.
        if constexpr (sizeof(T) == 4 && R > 16) {
            if (r % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
    }

    // The owned cells within k of an owned edge: what the neighbours need.
    // Written with device-scope (sc1) stores, which are coherent across XCDs
    // without an L2 write-back.
    __device__ __forceinline__ void publish(T (&x)[R][C], T* xb, int64_t pitch, const WgDesc& d, int kk)
    {
        // An opaque copy of the pitch: the per-row offsets are not hoisted out
        // of the epoch loop (where they would hold registers through the steps).
        asm volatile("" : "+v"(pitch));
        // Every store below sits in its own exec-masked block, so the
        // compiler's wait-count tracking cannot see that the tile registers
        // are no longer the target of an outstanding load (the paths into the
        // step loop include the ghost loads) and would otherwise put a
        // vmcnt(0) wait before each store, serialising them.  One explicit
        // wait here (nothing is outstanding by now) clears that state.
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt/lgkmcnt untouched
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
                if (own && near) xchg_store(xb + (int64_t)g * pitch + col, x[r][c]);
            }
        }
    }

    // Refresh the ghost ring (cells within k of the owned region, inside the
    // computed region, not owned) with device-scope (sc1) loads.
    __device__ __forceinline__ void load_ghost(T (&x)[R][C], T* xb, int64_t pitch, const WgDesc& d, int kk)
    {
        asm volatile("" : "+v"(pitch));  // as in publish
        const int r_lo = max(d.own_r0 - kk, d.cr_r0), r_hi = min(d.own_r1 + kk, d.cr_r1);
        const int c_lo = max(d.own_c0 - kk, d.cr_c0), c_hi = min(d.own_c1 + kk, d.cr_c1);
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
                if (in_ring && !own) x[r][c] = xchg_load(xb + (int64_t)g * pitch + col);
            }
        }
    }

    // Move this lane's cells of a stage map between registers and the
    // staging area (LOAD: stage -> registers).  A full row is stored as the
    // whole tile row (in the edge-row order, edge_pos), so every lane has a
    // slot there;
    // side rows hold only the side columns, and a lane with nothing to move
    // in a side row uses a spare slot of its own past the staging area.
    // Branch-free: lane r works out the kind and first slot of row r, read
    // back as a scalar, so each cell costs one select and one LDS access,
    // and the accesses issue back to back.
    template <bool LOAD>
    __device__ __forceinline__ void stage_cells(T (&x)[R][C], const StageMap& m)
    {
        constexpr int kSide = G::kSide;
        // An opaque copy of col0: keeps the compiler from hoisting the column
        // offsets out of the epoch loop, where they would stay live (and
        // spill) through the steps.
        int lcol0 = col0;
        asm volatile("" : "+v"(lcol0));
        if constexpr (!LOAD) __builtin_amdgcn_s_waitcnt(0x0F70);  // as in publish: no wait per LDS store
        const int spare = G::kStageElems + lane;
        // Per column slot (once per call): the lanes whose column is one of
        // the map's full-row columns (nmask) or side columns (wmask), as
        // wave-wide masks, and the side slot of each lane (its spare slot
        // when it has none).
        // A side row's cell c sits at the LDS byte address sbyte[c] +
        // sinc[c] * (the row's first slot): its side slot for a lane that has
        // one.  A lane without one loads the row's first slot (the same
        // address for all such lanes: a broadcast, no bank conflict; the
        // value is not picked) and stores to its own spare slot (sinc 0: a
        // store must not land in a live slot).  One 24-bit multiply-add per
        // cell (slots are far below 2^24).
        const uint32_t stage_lds = (uint32_t)(uintptr_t)stage;  // low half of an LDS pointer: its LDS address
        uint64_t nmask[C], wmask[C];
        uint32_t sbyte[C], sinc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int col = lcol0 + c;
            const bool w = col >= m.w0 && col < m.w1, e = col >= m.e0 && col < m.e1;
            nmask[c] = __builtin_amdgcn_ballot_w64(col >= m.c0 && col < m.c1);
            wmask[c] = __builtin_amdgcn_ballot_w64(w || e);
            const int slot = w ? col - m.w0 : (e ? kSide + col - m.e0 : (LOAD ? 0 : spare));
            sbyte[c] = stage_lds + (uint32_t)slot * (uint32_t)sizeof(T);
            sinc[c] = (w || e || LOAD) ? (uint32_t)sizeof(T) : 0u;
        }
        // Row r of this wave: bit 31 set for a full row (low bits: its first
        // slot), a side row's first slot, or -1 when the row moves nothing.
        int rowinfo;
        {
            const int g = g0 + (lane < R ? lane : 0);
            const int nn = m.n1 - m.n0;
            const bool in_n = g >= m.n0 && g < m.n1, in_s = g >= m.s0 && g < m.s1, in_m = g >= m.m0 && g < m.m1;
            rowinfo = in_n ? (int)(0x80000000u | (uint32_t)((g - m.n0) * EC))
                    : in_s ? (int)(0x80000000u | (uint32_t)((nn + g - m.s0) * EC))
                    : in_m ? G::kStageRows + (g - m.m0) * 2 * kSide
                           : -1;
        }
        // Row kinds are uniform, so each row takes one branch: a full row is
        // one address per lane (the C cells at fixed offsets), a side row one
        // address per cell (the side slot, or the spare).  Loads go in groups
        // of four rows, all issued before any result is picked into the tile.
        constexpr int kGroup = 4;
#pragma unroll
        for (int r0 = 0; r0 < R; r0 += kGroup) {
            T v[kGroup][C];
            uint64_t pick[kGroup][C];
#pragma unroll
            for (int rr = 0; rr < kGroup && r0 + rr < R; ++rr) {
                const int r = r0 + rr;
                const int info = __builtin_amdgcn_readlane(rowinfo, r);
#pragma unroll
                for (int c = 0; c < C; ++c) pick[rr][c] = 0;
                if (info == -1) continue;
                if (info < 0) {
                    T* const p = stage + (info & 0x7fffffff);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        if constexpr (LOAD) {
                            v[rr][c] = p[edge_pos(lane, c)];
                            pick[rr][c] = nmask[c];
                        } else {
                            p[edge_pos(lane, c)] = x[r][c];
                        }
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        uint32_t addr;
                        asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(addr) : "s"(info), "v"(sinc[c]), "v"(sbyte[c]));
                        LdsT* const p = (LdsT*)addr;
                        if constexpr (LOAD) {
                            v[rr][c] = *p;
                            pick[rr][c] = wmask[c];
                        } else {
                            *p = x[r][c];
                        }
                    }
                }
            }
            if constexpr (LOAD) {
#pragma unroll
                for (int rr = 0; rr < kGroup && r0 + rr < R; ++rr)
#pragma unroll
                    for (int c = 0; c < C; ++c) x[r0 + rr][c] = lane_pick(pick[rr][c], x[r0 + rr][c], v[rr][c]);
            }
        }
    }

    // Copy a stage map between the staging area and the exchange buffer
    // (STORE: stage -> buffer) with the whole workgroup: full rows with EC
    // consecutive lanes per row (a wave covers part of one row, so the row is
    // scalar), side rows with 2 * kSide lanes per row.  Buffer addresses step
    // by scalar strides and staging slots by immediate offsets; all loads (or
    // LDS reads) are issued before any of their results is used, so one
    // memory latency covers the lot.
    template <bool STORE>
    __device__ __forceinline__ void stage_copy(T* xb, int64_t pitch, const StageMap& m)
    {
        constexpr int kThreads = WAVES * kWaveSize;
        constexpr int kSide = G::kSide, SW = 2 * kSide;
        constexpr int kRowsPass = kThreads / EC, kSidePass = kThreads / SW;
        constexpr int kNP = (2 * G::kStageK + kRowsPass - 1) / kRowsPass;
        constexpr int kSP = (ER + kSidePass - 1) / kSidePass;
        static_assert(kThreads % EC == 0 && kThreads % SW == 0 && EC % kWaveSize == 0, "staging copy shape");
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));  // as in stage_cells: no hoisting out of the epoch loop
        asm volatile("" : "+v"(pitch));
        const int nn = m.n1 - m.n0, nrows = nn + (m.s1 - m.s0);
        const int cc = tid % EC;
        const int rr = uniform(tid / EC);  // the same for the whole wave
        const bool cact = cc < m.c1 - m.c0;
        T* const fbase = xb + m.c0 + cc;
        T* const fslot = stage + rr * EC + edge_pos((m.tc0 + cc) / C, (m.tc0 + cc) % C);  // as in stage_cells
        const int sc = tid % SW, sr = tid / SW;
        const bool left = sc < kSide;
        const int scol = left ? m.w0 + sc : m.e0 + (sc - kSide);
        const bool sact = left ? sc < m.w1 - m.w0 : (sc - kSide) < m.e1 - m.e0;
        const int nm = m.m1 - m.m0;
        T* const sbase = xb + (int64_t)(m.m0 + sr) * pitch + scol;
        T* const sslot = stage + G::kStageRows + sr * SW + sc;
        const int64_t sstride = (int64_t)kSidePass * pitch;
        T v[kNP + kSP];
        if constexpr (STORE) {
#pragma unroll
            for (int j = 0; j < kNP; ++j) v[j] = fslot[j * kRowsPass * EC];
#pragma unroll
            for (int j = 0; j < kSP; ++j) v[kNP + j] = sslot[j * kSidePass * SW];
#pragma unroll
            for (int j = 0; j < kNP; ++j) {
                const int ri = rr + j * kRowsPass;
                if (ri < nrows && cact) {
                    const int g = ri < nn ? m.n0 + ri : m.s0 + (ri - nn);
                    xchg_store(fbase + (int64_t)g * pitch, v[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < kSP; ++j)
                if (sr + j * kSidePass < nm && sact) xchg_store(sbase + j * sstride, v[kNP + j]);
        } else {
#pragma unroll
            for (int j = 0; j < kNP; ++j) {
                const int ri = rr + j * kRowsPass;
                const int g = ri < nn ? m.n0 + ri : m.s0 + (ri - nn);
                v[j] = (ri < nrows && cact) ? xchg_load(fbase + (int64_t)g * pitch) : T(0);
            }
#pragma unroll
            for (int j = 0; j < kSP; ++j)
                v[kNP + j] = (sr + j * kSidePass < nm && sact) ? xchg_load(sbase + j * sstride) : T(0);
            // Only live positions write: a full-row slot of a lane past the
            // row's columns can lie in the next row, and past the last row in
            // the side block.
#pragma unroll
            for (int j = 0; j < kNP; ++j)
                if (rr + j * kRowsPass < nrows && cact) fslot[j * kRowsPass * EC] = v[j];
#pragma unroll
            for (int j = 0; j < kSP; ++j)
                if (sr + j * kSidePass < nm && sact) sslot[j * kSidePass * SW] = v[kNP + j];
        }
    }

    // Debug: set every interior cell of the register tile outside the fresh
    // region (owned cells grown by k, clipped to the computed region) to NaN.
    // Those cells are expendable by construction; a NaN reaching an owned
    // cell within the next k steps would expose a hole in that argument.
    __device__ __forceinline__ void poison(T (&x)[R][C], const WgDesc& d, int kk, int rows, int cols)
    {
        const int r_lo = max(d.own_r0 - kk, d.cr_r0), r_hi = min(d.own_r1 + kk, d.cr_r1);
        const int c_lo = max(d.own_c0 - kk, d.cr_c0), c_hi = min(d.own_c1 + kk, d.cr_c1);
        const T nan = __builtin_nan("");
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int g = g0 + r;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int col = col0 + c;
                const bool interior = g >= 1 && g <= rows && col >= 1 && col <= cols;
                const bool fresh = g >= r_lo && g < r_hi && col >= c_lo && col < c_hi;
                if (interior && !fresh) x[r][c] = nan;
            }
        }
    }

    // Owned cells inside the stored region -> dst, with plain stores: the four
    // cells of a lane in a row share 32 bytes, and plain stores of one wave
    // meet in the L2 as whole lines (device-scope stores would each go to
    // memory on their own, four partial writes per 32 bytes).  When the
    // readers are other workgroups of the same launch (the tile-serial sweep),
    // the caller makes the stores visible device-wide with an agent-scope
    // release before it signals them (grid_barrier / group_point with
    // release = true).
    __device__ __forceinline__ void store_owned(T (&x)[R][C], T* __restrict__ dst, int64_t pitch, const WgDesc& d)
    {
        const int r0 = max(d.own_r0, d.st_r0), r1 = min(d.own_r1, d.st_r1);
        const int c0 = max(d.own_c0, d.st_c0), c1 = min(d.own_c1, d.st_c1);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // as in publish: keeps the stores from being serialised
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int g = g0 + r;
            if (g < r0 || g >= r1) continue;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int col = col0 + c;
                if (col >= c0 && col < c1) dst[(int64_t)g * pitch + col] = x[r][c];
            }
        }
    }
};

// Neighbour-wise bulk-synchronous exchange point.
//
// The border strips were written with device-scope atomic stores; waiting for
// them to complete (vmcnt 0) makes them visible to every XCD, so no L2
// write-back is needed before this workgroup raises its epoch flag.  The
// first nnb threads of wave 0 then wait (bounded) until each neighbour's flag
// has reached the same epoch; the ghost ring is read afterwards with
// device-scope loads, so no L2 invalidate is needed either.  The inline
// waits double as compiler barriers (memory clobber).  On timeout the error
// word is set and the wait is abandoned, so the grid always drains.
__device__ __forceinline__ void exchange_point(uint32_t* flags, int me, const WgDesc& d, uint32_t target,
                                               int* err, uint32_t spin_limit)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flags + (size_t)me * kFlagStride, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((int)threadIdx.x < d.nnb) {
        const int nb = d.nb[threadIdx.x];
        uint32_t spins = 0;
        while (!reached(__hip_atomic_load(flags + (size_t)nb * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), target)) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > spin_limit) {
                __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            // Someone else already gave up: stop waiting so the grid drains quickly.
            if ((spins & 1023) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}

// Device-wide barrier for the sweep, two levels deep so that no address has
// more than one XCD's workgroups polling it.  Counters (each in its own
// kFlagStride slot, all reset to 0 before the launch): slot 0 counts XCDs,
// slots 1..8 count arrivals per XCD, slots 9..16 are per-XCD release words.
// Workgroup b runs on XCD b % 8.  Barrier number n (1-based): the last
// arrival of an XCD bumps the XCD counter, waits for every XCD, then releases
// its own XCD by writing n.  Prior device-scope stores are complete (vmcnt 0)
// before arriving.  Bounded waits as in exchange_point.
// Slot 17 (of kBarrierSlots): the tile-serial sweep's count of tile-boundary
// arrivals (the split-phase barrier between the big tiles of a round, below).
constexpr int kTileCountSlot = 17;
static_assert(kTileCountSlot < kBarrierSlots, "barrier slots");

__device__ __forceinline__ bool spin_until(uint32_t* p, uint32_t target, int* err, int code, uint32_t spin_limit)
{
    uint32_t spins = 0;
    while (!reached(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), target)) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > spin_limit) {
            __hip_atomic_fetch_or(err, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if ((spins & 1023) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    }
    return true;
}

__device__ __forceinline__ void grid_barrier(uint32_t* bar, uint32_t n, int* err, uint32_t spin_limit,
                                             bool release = false, bool wait_stores = true, bool acquire = false)
{
    // wait_stores == false: the workgroup's outstanding stores need not be
    // complete at the barrier (the caller's memory accesses that the barrier
    // orders -- exchange strips and flags -- have completed already), so the
    // waves meet with a bare s_barrier and no vmcnt wait, and the stores keep
    // draining behind it.
    if (wait_stores) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    } else {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    }
    if (threadIdx.x == 0) {
        // release: the workgroup's plain stores (all complete in this XCD's L2
        // by now) are written back so that every XCD sees them after the barrier.
        if (release) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t x = blockIdx.x % 8u;
        const uint32_t per_xcd = (gridDim.x - x + 7u) / 8u;  // workgroups on this XCD
        const uint32_t nxcd = gridDim.x < 8u ? gridDim.x : 8u;
        uint32_t* xcnt = bar + (size_t)(1 + x) * kFlagStride;
        uint32_t* xrel = bar + (size_t)(9 + x) * kFlagStride;
        const uint32_t old = __hip_atomic_fetch_add(xcnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == per_xcd * n) {
            __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            spin_until(bar, nxcd * n, err, 2, spin_limit);
            __hip_atomic_store(xrel, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        spin_until(xrel, n, err, 2, spin_limit);
    }
    if (wait_stores) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    } else {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    }
    // acquire: what other workgroups released before the barrier is visible to
    // this workgroup's plain loads after it (no stale line of this XCD's caches).
    if (acquire) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Split-phase barrier between two big tiles of one round of a sweep.  The
// only thing it orders is the reuse of the exchange buffers: no workgroup may
// store the strips of big tile m while another one may still read strips of
// big tile m - 1 (tile m reads buffer A, which no one writes in this round,
// and stores its own cells of buffer B, so nothing else needs it).  Every
// workgroup signals when it is done with a big tile (its ring loads have all
// returned by then) and, before its first strip store in the next big tile of
// the round, waits for the others' signals (n words, each to reach `target`).
// The tile-serial sweep counts arrivals in one word (n = 1,
// target nwg * m: the first time the count reaches nwg * m every workgroup has
// arrived exactly m times, since none arrives an (m + 1)-th time before it has
// waited for nwg * m); a swept job of the batched kernel uses its members'
// epoch flags (n = group size, target the boundary's epoch; flags only grow).
// The words are read once before the tile load is issued and checked after it
// (the loads hide the round trip); only a word that is short is polled again
// (bounded, as in grid_barrier).
__device__ __forceinline__ void tile_arrive(uint32_t* bar)
{
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(bar + (size_t)kTileCountSlot * kFlagStride, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// GATE 1: one word (the sweep's counter), read by thread 0; GATE 2: the n
// words words[i * kFlagStride] (a batched job's member flags), thread i
// reading word i, so n must not exceed the workgroup size (a batched job has
// at most one member per compute unit, 256, against 512 threads).  Threads
// without a word see the target.
template <int GATE>
__device__ __forceinline__ uint32_t gate_peek(const uint32_t* words, uint32_t target, int n)
{
    const int nw = GATE == 1 ? 1 : n;
    return (int)threadIdx.x < nw ? __hip_atomic_load(words + (size_t)threadIdx.x * kFlagStride, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                                 : target;
}

template <int GATE>
__device__ __forceinline__ void gate_wait(uint32_t* words, uint32_t target, int n, uint32_t seen, int* err,
                                          uint32_t spin_limit)
{
    const int nw = GATE == 1 ? 1 : n;
    if ((int)threadIdx.x < nw && !reached(seen, target))
        spin_until(words + (size_t)threadIdx.x * kFlagStride, target, err, GATE == 1 ? 2 : 4, spin_limit);
    __syncthreads();
}

// The synchronisation at an exchange point: by default each workgroup waits
// for the workgroups whose cells it reads (neighbour epoch flags); with
// P.grid_sync every workgroup waits for all of them at a device-wide barrier
// (the bulk-synchronous grid barrier of Section 3.2, kept to measure what the
// neighbour-wise form is worth).  `epoch` counts this run's exchange points
// from 1, which is also the barrier's number (its counters are reset before
// every launch).
__device__ __forceinline__ void sync_point(const ProbDesc& P, uint32_t* flags, int me, const WgDesc& d, uint32_t base,
                                           uint32_t epoch, int* err, uint32_t spin_limit)
{
    if (P.grid_sync) grid_barrier(P.bar, epoch, err, spin_limit);
    else exchange_point(flags, me, d, base + epoch, err, spin_limit);
}

// All time steps of one tile, the halo addends either fixed (HALO_ROWS =
// false) or read per row.  The state is in register set a at every epoch
// boundary: steps go in pairs a -> b -> a (LDS edge parity 0 then 1); an odd
// tail step is copied back.  A run of k steps is followed by an exchange
// point (a workgroup barrier), so an odd k never lets two consecutive steps
// share a parity.
template <bool HALO_ROWS, bool STAGED, typename Tl>
__device__ __forceinline__ void run_epochs(Tl& t, const ProbDesc& P, const WgDesc& d, int64_t steps, int me,
                                           uint32_t* flags, uint32_t base, uint32_t& epoch, int* err,
                                           uint32_t spin_limit)
{
    using T = typename std::remove_reference<decltype(t.a[0][0])>::type;
    constexpr int R = sizeof(t.a) / sizeof(t.a[0]);
    constexpr int C = sizeof(t.a[0]) / sizeof(t.a[0][0]);
    const int rows = P.rows, kk = P.k;
    const int64_t pitch = P.pitch;
    int64_t done = 0;
    bool exchanged = false;
    const bool poison = (P.debug & 2) != 0;
    if (poison) t.poison(t.a, d, kk, rows, P.cols);
    // Exchanges go through the LDS staging area unless the ring is deeper than it holds.
    using Tile_ = typename std::remove_reference<Tl>::type;
    constexpr bool kStagedHere = STAGED && Tile_::G::kStaged;
    const bool staged = kStagedHere && !P.direct_xchg && kk <= Tile_::G::kStageK;
    // DTB_DEBUG_TIMING: phase clocks of thread 0 (uniform branch, off by default).
    const bool timing = P.timing != nullptr;
    uint64_t tm[kEpochTimingSlots] = {};  // the slots below kTimeLoad (the others are added directly)
    uint64_t t0 = timing ? __builtin_amdgcn_s_memrealtime() : 0, t_start = t0;
    while (done < steps) {
        const int64_t left = steps - done;
        const int nsteps = (int)(left < kk ? left : kk);
        for (int s = 0; s + 1 < nsteps; s += 2) {
            t.template step<HALO_ROWS>(t.a, t.b, 0, rows);
            t.template step<HALO_ROWS>(t.b, t.a, 1, rows);
        }
        if (nsteps & 1) {
            t.template step<HALO_ROWS>(t.a, t.b, 0, rows);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < C; ++c) t.a[r][c] = t.b[r][c];
        }
        done += nsteps;
        if (done < steps) {
            T* xb = (T*)P.xbuf[epoch & 1];
            if (timing) {
                __syncthreads();
                const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
                tm[kTimeSteps] += t1 - t0;
                t0 = t1;
            }
            // An opaque copy of k keeps the maps from being hoisted out of the loop.
            int kx = kk;
            asm volatile("" : "+s"(kx));
            if constexpr (kStagedHere) {
                if (staged) {
                    const StageMap m = rim_map(d, kx);
                    t.template stage_cells<false>(t.a, m);
                    __syncthreads();
                    if (timing) {
                        const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
                        tm[kTimeStageOut] += t1 - t0;
                        t0 = t1;
                    }
                    t.template stage_copy<true>(xb, pitch, m);
                } else {
                    t.publish(t.a, xb, pitch, d, kk);
                }
            } else {
                t.publish(t.a, xb, pitch, d, kk);
            }
            if (timing) {
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
                const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
                tm[kTimePublish] += t1 - t0;
                t0 = t1;
            }
            ++epoch;
            sync_point(P, flags, me, d, base, epoch, err, spin_limit);
            if (timing) {
                const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
                tm[kTimeWait] += t1 - t0;
                t0 = t1;
            }
            exchanged = true;
            asm volatile("" : "+s"(kx));
            if constexpr (kStagedHere) {
                if (staged) {
                    const StageMap m = ring_map(d, kx);
                    t.template stage_copy<false>(xb, pitch, m);
                    __syncthreads();
                    if (timing) {
                        const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
                        tm[kTimeStageIn] += t1 - t0;
                        t0 = t1;
                    }
                    t.template stage_cells<true>(t.a, m);
                } else {
                    t.load_ghost(t.a, xb, pitch, d, kk);
                }
            } else {
                t.load_ghost(t.a, xb, pitch, d, kk);
            }
            // Set b = a.  Only cells a step never writes (outside the grid,
            // for COLMASK / ROWCHECK tiles) keep their value in b, and there
            // a and b agree; so b is dead from the last step of a segment to
            // here, which leaves its registers free for the staged exchange.
            // A tile whose steps write every cell needs no copy at all.
            if constexpr (kStagedHere && Tile_::kKeepsCells) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int c = 0; c < C; ++c) t.b[r][c] = t.a[r][c];
            }
            if (timing) {
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
                const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
                tm[kTimeGhost] += t1 - t0;
                tm[kTimeExchanges] += 1;
                t0 = t1;
            }
            if (poison) t.poison(t.a, d, kk, rows, P.cols);
        }
    }
    if (timing) {
        __syncthreads();
        const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
        tm[kTimeSteps] += t1 - t0;
        tm[kTimeTotal] += t1 - t_start;
        if (threadIdx.x == 0) {
            uint64_t* out = P.timing + (size_t)me * kTimingSlots;
            for (int i = 0; i < kEpochTimingSlots; ++i) atomicAdd((unsigned long long*)(out + i), (unsigned long long)tm[i]);
        }
    }
    // Neighbours read their initial ghost ring from the source grid; when the
    // result goes back in place, make sure they all have before it is written.
    if (!exchanged) {
        ++epoch;
        sync_point(P, flags, me, d, base, epoch, err, spin_limit);
    }
}

// DTB_DEBUG_TIMING: wait for this workgroup's memory accesses, then add the
// ticks since t0 to its clock `slot`.
__device__ __forceinline__ void add_clock(const ProbDesc& P, int me, int slot, uint64_t t0)
{
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __syncthreads();
    const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0)
        atomicAdd((unsigned long long*)(P.timing + (size_t)me * kTimingSlots + slot), (unsigned long long)(t1 - t0));
}

// Load a workgroup's extended tile from src into both register sets, the
// rows just above and below it into the LDS edge slots and the west/east halo
// products into LDS, and set up the tile's per-lane constants.  SC1: src is
// read with device-scope loads (other XCDs wrote it inside the same launch).
template <bool SC1, typename Tl, typename T>
__device__ __forceinline__ void load_tile(Tl& t, const ProbDesc& P, const WgDesc& d, const T* src, char* lds)
{
    using G = typename Tl::G;
    constexpr int C = G::EC / kWaveSize;
    constexpr int R = G::ER / (Tl::kWaves);
    constexpr int WAVES = Tl::kWaves;
    constexpr bool COLMASK = Tl::kColmask;
    const T* grid = src;
    const int64_t pitch = P.pitch;
    const int rows = P.rows, cols = P.cols;
    t.edge = (T*)lds;
    t.stage = (T*)lds + G::kEdgeElems + G::kHaloElems;
    T* hx = (T*)lds + G::kEdgeElems;  // [0, ER): w*hW, [ER, 2ER): e*hE, [2ER, 3ER): 0
    t.wave = uniform(threadIdx.x >> 6);
    t.lane = threadIdx.x & 63;
    t.g0 = d.ext_r0 + t.wave * R;
    t.col0 = d.ext_c0 + t.lane * C;
    if constexpr (Tl::kPts == 9) t.k = load_coef9<T>(P.coeffs);
    else t.k = load_coef<T>(P.coeffs);
#pragma unroll
    for (int c = 0; c < C; ++c) t.colact[c] = (t.col0 + c) <= cols;

    // ---- the extended tile (both register sets)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int g = t.g0 + r;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int col = t.col0 + c;
            T v = T(0);
            if (g <= rows + 1 && col <= cols + 1) {
                if constexpr (SC1)
                    v = __hip_atomic_load(grid + (int64_t)g * pitch + col, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else
                    v = grid[(int64_t)g * pitch + col];
            }
            t.a[r][c] = v;
            t.b[r][c] = v;
        }
    }
    // Rows just above and below the extended tile (the halo rows for edge
    // tiles, stale ghost values otherwise), both parities.
    const int gt = d.ext_r0 - 1;
    const int gb = d.ext_r0 + G::ER;
    for (int idx = threadIdx.x; idx < G::EC; idx += WAVES * kWaveSize) {
        const int col = d.ext_c0 + idx;
        const T vt = (col <= cols + 1) ? grid[(int64_t)gt * pitch + col] : T(0);
        const T vb = (gb <= rows + 1 && col <= cols + 1) ? grid[(int64_t)gb * pitch + col] : T(0);
        const int pos = Tl::edge_pos(idx / C, idx % C);
        for (int p = 0; p < 2; ++p) {
            t.edge_row(p, 0, 1)[pos] = vt;
            t.edge_row(p, WAVES + 1, 0)[pos] = vb;
        }
    }
    // West/east halo products for the rows of an edge tile (zero elsewhere:
    // the outermost ghost columns of an interior tile are expendable).
    const bool west_edge = d.ext_c0 == 1;
    const bool east_edge = !COLMASK && d.ext_c0 + G::EC - 1 == cols;
    const T zero = T(0);
    if constexpr (Tl::kPts == 9) {
        // Box: the halo values themselves, of the storage rows ext_r0 - 1 ..
        // ext_r0 + ER (the rows the tile's diagonal neighbours reach, corner
        // cells included): [0, ER+2) west, [ER+2, 2ER+4) east, then zeros.
        constexpr int H = G::ER + 2;
        for (int idx = threadIdx.x; idx < H; idx += WAVES * kWaveSize) {
            const int g = d.ext_r0 - 1 + idx;
            const bool grow = g >= 0 && g <= rows + 1;
            hx[idx] = (west_edge && grow) ? grid[(int64_t)g * pitch] : T(0);
            hx[H + idx] = (east_edge && grow) ? grid[(int64_t)g * pitch + cols + 1] : T(0);
            hx[2 * H + idx] = T(0);
        }
        __syncthreads();
        t.bw = t.lane == 0 ? hx[1] : zero;
        t.be = t.lane == 63 ? hx[H + 1] : zero;
        t.bwe = zero;
        t.hbw = hx + (t.lane == 0 ? 0 : 2 * H);
        t.hbe = hx + (t.lane == 63 ? H : 2 * H);
        t.hbwe = hx + 2 * H;
    } else {
        for (int idx = threadIdx.x; idx < G::ER; idx += WAVES * kWaveSize) {
            const int g = d.ext_r0 + idx;
            const bool grow = g >= 1 && g <= rows;
            hx[idx] = (west_edge && grow) ? t.k.w * grid[(int64_t)g * pitch] : T(0);
            hx[G::ER + idx] = (east_edge && grow) ? t.k.e * grid[(int64_t)g * pitch + cols + 1] : T(0);
            hx[2 * G::ER + idx] = T(0);
        }
        __syncthreads();

        // With HALO_ROWS == false the products are the same on every row (checked
        // by the caller) and live in registers.
        t.bw = t.lane == 0 ? hx[0] : zero;
        t.be = t.lane == 63 ? hx[G::ER] : zero;
        t.bwe = t.lane == 0 ? hx[0] : (t.lane == 63 ? hx[G::ER] : zero);
        t.hbw = hx + (t.lane == 0 ? 0 : 2 * G::ER);
        t.hbe = hx + (t.lane == 63 ? G::ER : 2 * G::ER);
        t.hbwe = hx + (t.lane == 0 ? 0 : (t.lane == 63 ? G::ER : 2 * G::ER));
    }
}

// One segment of work for one workgroup: load its extended tile from src,
// advance it `steps` steps (exchanging every k), store its owned cells inside
// the stored region to dst.  SWEEP: src/dst are the sweep's HBM buffers, read
// and written with device-scope accesses (other XCDs wrote / will read them
// inside the same launch).
template <typename T, int C, int R, int WAVES, bool FMA, bool COLMASK, bool ROWCHECK, bool HALO_ROWS, bool SWEEP,
          bool STAGED = true, int PTS = 5, int GATE = 0>
__device__ __forceinline__ void run_segment(const ProbDesc& P, const WgDesc& d, const T* src, T* dst, int64_t steps,
                                            int me, uint32_t* flags, uint32_t base, uint32_t& epoch, int* err,
                                            uint32_t spin_limit, char* lds, uint32_t* gate_words = nullptr,
                                            uint32_t gate_target = 0, int gate_n = 0)
{
    using Tl = Tile<T, C, R, WAVES, FMA, COLMASK, ROWCHECK, PTS>;
    Tl t;
    const bool timing = P.timing != nullptr;  // DTB_DEBUG_TIMING (uniform branch)
    uint64_t t0 = timing ? __builtin_amdgcn_s_memrealtime() : 0;
    // gate_words != null (GATE 1 or 2): the split-phase barrier between big
    // tiles must have been passed before this segment's first strip store.
    const bool gated = GATE != 0 && gate_words != nullptr;
    const uint32_t seen = gated ? gate_peek<GATE>(gate_words, gate_target, gate_n) : 0u;
    load_tile<SWEEP>(t, P, d, src, lds);
    if (timing) add_clock(P, me, kTimeLoad, t0);
    if (gated) {
        if (timing) t0 = __builtin_amdgcn_s_memrealtime();
        gate_wait<GATE>(gate_words, gate_target, gate_n, seen, err, spin_limit);
        if (timing) add_clock(P, me, kTimeBarrier, t0);
    }
    run_epochs<HALO_ROWS, STAGED>(t, P, d, steps, me, flags, base, epoch, err, spin_limit);
    if (timing) t0 = __builtin_amdgcn_s_memrealtime();
    t.store_owned(t.a, dst, P.pitch, d);
    if (timing) add_clock(P, me, kTimeStore, t0);
}

// Overlapped (trapezoidal) temporal blocking of one workgroup, with no
// synchronisation between workgroups at all: its extended tile is loaded from
// src with a ring as deep as the number of steps, advanced `steps` steps
// (after which the owned cells are exact: stale values from the tile's open
// edges move one cell per step), and its owned cells are stored to dst.
template <typename T, int C, int R, int WAVES, bool FMA, bool COLMASK, bool ROWCHECK, bool HALO_ROWS>
__device__ __forceinline__ void run_overlapped(const ProbDesc& P, const WgDesc& d, const T* src, T* dst, int steps,
                                               char* lds)
{
    using Tl = Tile<T, C, R, WAVES, FMA, COLMASK, ROWCHECK>;
    Tl t;
    load_tile<false>(t, P, d, src, lds);
    const int rows = P.rows;
    for (int s = 0; s + 1 < steps; s += 2) {
        t.template step<HALO_ROWS>(t.a, t.b, 0, rows);
        t.template step<HALO_ROWS>(t.b, t.a, 1, rows);
    }
    if (steps & 1) {
        t.template step<HALO_ROWS>(t.a, t.b, 0, rows);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c) t.a[r][c] = t.b[r][c];
    }
    t.store_owned(t.a, dst, P.pitch, d);
}

// Does the west or east halo of this tile's rows change from row to row?
// (Only edge tiles look: an interior tile never reads the halo.)  The box
// stencil also reads the halo of the rows just above and below the tile
// (corner cells included).
template <typename T, int C, int R, int WAVES, bool COLMASK, int PTS = 5>
__device__ __forceinline__ bool halo_varies(const ProbDesc& P, const WgDesc& d)
{
    using G = Geo<T, C, R, WAVES>;
    const T* grid = (const T*)P.grid;
    const int rows = P.rows, cols = P.cols;
    const bool west_edge = d.ext_c0 == 1;
    const bool east_edge = !COLMASK && d.ext_c0 + G::EC - 1 == cols;
    bool mine = false;
    if (west_edge || east_edge) {
        const int r0 = PTS == 9 ? max(d.ext_r0 - 1, 0) : max(d.ext_r0, 1);
        const int r1 = PTS == 9 ? min(d.ext_r0 + G::ER, rows + 1) : min(d.ext_r0 + G::ER - 1, rows);
        const T w0 = grid[(int64_t)r0 * P.pitch], e0 = grid[(int64_t)r0 * P.pitch + cols + 1];
        for (int g = r0 + (int)threadIdx.x; g <= r1; g += WAVES * kWaveSize) {
            if (west_edge && grid[(int64_t)g * P.pitch] != w0) mine = true;
            if (east_edge && grid[(int64_t)g * P.pitch + cols + 1] != e0) mine = true;
        }
    }
    return __syncthreads_or(mine);
}

// LDS for the largest instance a kernel can run.
template <typename T, int C, int R, int WAVES>
__device__ __forceinline__ char* dtb_lds()
{
    __shared__ __attribute__((aligned(16))) char lds[Geo<T, C, R, WAVES>::kLdsBytes];
    return lds;
}

template <typename T, int C, int R, int WAVES, bool FMA, bool COLMASK, bool ROWCHECK, int PTS = 5>
__global__ __launch_bounds__(WAVES * 64, 2) void k_dtb(ProbDesc P, const WgDesc* __restrict__ wgs,
                                                    uint32_t* flags, int* err, uint32_t spin_limit)
{
    const int me = blockIdx.x;
    const WgDesc& d = wgs[me];
    char* lds = dtb_lds<T, C, R, WAVES>();
    const uint32_t base = __hip_atomic_load(flags + (size_t)me * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t epoch = 0;
    T* grid = (T*)P.grid;
    if (halo_varies<T, C, R, WAVES, COLMASK, PTS>(P, d))
        run_segment<T, C, R, WAVES, FMA, COLMASK, ROWCHECK, true, false, true, PTS>(P, d, grid, grid, P.T, me, flags,
                                                                                    base, epoch, err, spin_limit, lds);
    else
        run_segment<T, C, R, WAVES, FMA, COLMASK, ROWCHECK, false, false, true, PTS>(P, d, grid, grid, P.T, me, flags,
                                                                                     base, epoch, err, spin_limit, lds);
}

// Overlapped per-workgroup temporal blocking (the "overlapped tiling within
// thread blocks" that Section 2 sets the grid-barrier design against): one
// launch per round of `steps` steps, any number of workgroups, each reading
// its extended tile from src and writing its owned cells to dst, with no
// synchronisation between workgroups.
template <typename T, int C, int R, int WAVES, bool FMA, bool COLMASK, bool ROWCHECK>
__global__ __launch_bounds__(WAVES * 64, 2) void k_ovl(ProbDesc P, const WgDesc* __restrict__ wgs, const T* src,
                                                    T* dst, int steps)
{
    const WgDesc& d = wgs[blockIdx.x];
    char* lds = dtb_lds<T, C, R, WAVES>();
    if (halo_varies<T, C, R, WAVES, COLMASK>(P, d))
        run_overlapped<T, C, R, WAVES, FMA, COLMASK, ROWCHECK, true>(P, d, src, dst, steps, lds);
    else
        run_overlapped<T, C, R, WAVES, FMA, COLMASK, ROWCHECK, false>(P, d, src, dst, steps, lds);
}

// The tile-serial sweep (Sections 1, 3.1, 3.3, Figure 1): rounds of D steps;
// in every round the big tiles run one after another on the whole chip, each
// reading its computed region (valid part + D ring) from buffer A and writing
// its valid part to buffer B; a split-phase barrier separates the big tiles
// of a round, a device-wide barrier the rounds.  Round r reads bufs[r & 1]
// and writes bufs[(r + 1) & 1]; bufs[0] is the grid.
template <typename T, int C, int R, int WAVES, bool FMA, bool COLMASK, bool ROWCHECK, int PTS = 5>
__global__ __launch_bounds__(WAVES * 64, 2) void k_dtb_sweep(ProbDesc P, SweepArgs S, const WgDesc* __restrict__ table,
                                                          uint32_t* flags, int* err, uint32_t spin_limit)
{
    const int me = blockIdx.x;
    char* lds = dtb_lds<T, C, R, WAVES>();
    const uint32_t base = __hip_atomic_load(flags + (size_t)me * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t epoch = 0;
    uint32_t nbar = 0;
    int64_t done = 0;
    // Within a round the big tiles are independent (each reads A and writes its
    // own valid part of B), so the barrier between two of them only keeps the
    // next tile's exchanges from overwriting strips of this one that a slower
    // workgroup may still read: a split-phase barrier (tile_arrive, then
    // gate_wait after the next tile's load) that does not wait for this
    // tile's stores to B, which drain while the next tile loads.  B is read in
    // the next round only: the round's last barrier waits for the stores,
    // makes them visible to every XCD (agent-scope release) and, past the
    // barrier, drops whatever this XCD's caches hold of them (agent-scope
    // acquire), so that the next round loads A with plain (wide) loads.
    uint32_t nbound = 0;  // tile boundaries inside rounds so far (split-phase barrier)
    for (int round = 0; round < S.nrounds; ++round) {
        const T* A = (const T*)S.bufs[round & 1];
        T* B = (T*)S.bufs[(round + 1) & 1];
        const int64_t left = P.T - done;
        const int64_t steps = left < S.D ? left : S.D;
        for (int tile = 0; tile < S.ntiles; ++tile) {
            const WgDesc& d = table[(size_t)tile * S.nwg + me];
            // Past the first big tile of a round, wait for every workgroup to
            // be done with the previous one before storing strips.
            uint32_t* const gw = tile > 0 ? S.bar + (size_t)kTileCountSlot * kFlagStride : nullptr;
            const uint32_t target = nbound * gridDim.x;
            if (d.own_r0 == d.own_r1) {
                // Idle for this tile: keep the epoch count in step with the others.
                const int64_t per = (steps + P.k - 1) / P.k - 1;
                epoch += per > 0 ? (uint32_t)per : 1u;
                if (gw != nullptr) gate_wait<1>(gw, target, 1, gate_peek<1>(gw, target, 1), err, spin_limit);
            } else if (halo_varies<T, C, R, WAVES, COLMASK, PTS>(P, d)) {
                run_segment<T, C, R, WAVES, FMA, COLMASK, ROWCHECK, true, false, true, PTS, 1>(
                    P, d, A, B, steps, me, flags, base, epoch, err, spin_limit, lds, gw, target);
            } else {
                run_segment<T, C, R, WAVES, FMA, COLMASK, ROWCHECK, false, false, true, PTS, 1>(
                    P, d, A, B, steps, me, flags, base, epoch, err, spin_limit, lds, gw, target);
            }
            if (tile + 1 < S.ntiles) {
                ++nbound;
                tile_arrive(S.bar);
            } else {
                // The round's end: a full barrier that also makes B visible to
                // every XCD (see above).
                ++nbar;
                const uint64_t tb = P.timing ? __builtin_amdgcn_s_memrealtime() : 0;
                grid_barrier(S.bar, nbar, err, spin_limit, true, true, true);
                if (P.timing) add_clock(P, me, kTimeBarrier, tb);
            }
        }
        done += steps;
    }
    // A workgroup idle in the last tiles has not published its final epoch;
    // every flag must end the run at the same value, since the next run
    // starts counting from it.
    if (threadIdx.x == 0) __hip_atomic_store(flags + (size_t)me * kFlagStride, base + epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


constexpr int kDtbWaves = 8;

// ============================================================================ batched launch

// Group-wide synchronisation point of a batched job: raise this member's
// flag, wait (bounded) until every member's flag reached `target`.
__device__ __forceinline__ void group_point(uint32_t* flags, int flag_base, int g, int local, uint32_t target,
                                            int* err, uint32_t spin_limit, bool release = false)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0 && release) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // as in grid_barrier
    if (threadIdx.x == 0)
        __hip_atomic_store(flags + (size_t)(flag_base + local) * kFlagStride, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int i = threadIdx.x; i < g; i += blockDim.x) {
        uint32_t spins = 0;
        while (!reached(__hip_atomic_load(flags + (size_t)(flag_base + i) * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                        target)) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > spin_limit) {
                __hip_atomic_fetch_or(err, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            if ((spins & 1023) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}

// One job for one member of its group.  A grid held on chip runs in place
// (one segment of T steps); a larger one is swept through big tiles, with
// the halo ring first copied into the second buffer and, after an odd number
// of rounds, the interior copied back -- both split over the group.
template <typename T, int C, int R, int WAVES, bool FMA, bool COLMASK>
__device__ __forceinline__ void run_job(const ProbDesc& P, const JobDesc& J, const WgDesc* __restrict__ table,
                                        int local, uint32_t* flags, int* err, uint32_t spin_limit, char* lds)
{
    const int me = J.flag_base + local;
    const uint32_t base = __hip_atomic_load(flags + (size_t)me * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t epoch = 0;
    T* grid = (T*)P.grid;
    if (!J.sweep) {
        const WgDesc& d = table[J.table_off + local];
        // Batched jobs use the staging area too: the batched kernel, which holds every variant in
        // one function, then spills a few words, but measured 7 % faster on a 64-grid batch.
        if (halo_varies<T, C, R, WAVES, COLMASK>(P, d))
            run_segment<T, C, R, WAVES, FMA, COLMASK, true, true, false, true>(P, d, grid, grid, P.T, me, flags, base,
                                                                          epoch, err, spin_limit, lds);
        else
            run_segment<T, C, R, WAVES, FMA, COLMASK, true, false, false, true>(P, d, grid, grid, P.T, me, flags, base,
                                                                           epoch, err, spin_limit, lds);
        return;
    }
    T* ws = (T*)J.ws;
    const int rows = P.rows, cols = P.cols;
    const int64_t pitch = P.pitch;
    const int nthr = J.g * WAVES * kWaveSize;
    const int tid = local * WAVES * kWaveSize + threadIdx.x;
    // Halo ring of the grid into the second buffer.
    for (int idx = tid; idx < 2 * (cols + 2) + 2 * rows; idx += nthr) {
        int64_t off;
        if (idx < cols + 2) off = idx;
        else if (idx < 2 * (cols + 2)) off = (int64_t)(rows + 1) * pitch + (idx - (cols + 2));
        else {
            const int j = idx - 2 * (cols + 2);
            off = (int64_t)(1 + (j >> 1)) * pitch + ((j & 1) ? cols + 1 : 0);
        }
        __hip_atomic_store(ws + off, grid[off], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    ++epoch;
    group_point(flags, J.flag_base, J.g, local, base + epoch, err, spin_limit);
    int64_t done = 0;
    // As in the tile-serial sweep: the big tiles of a round are separated by a
    // split-phase barrier on the members' epoch flags (a member raises its flag
    // when done with a tile, and waits for everyone's before its first strip
    // store in the next one); the round's end is a full group barrier that
    // releases the plain stores of B and, past it, acquires them, so that A is
    // read with plain loads.
    for (int round = 0; round < J.nrounds; ++round) {
        const T* A = (round & 1) ? ws : grid;
        T* B = (round & 1) ? grid : ws;
        const int64_t left = P.T - done;
        const int64_t steps = left < J.D ? left : J.D;
        for (int tile = 0; tile < J.ntiles; ++tile) {
            const WgDesc& d = table[J.table_off + (size_t)tile * J.g + local];
            uint32_t* const gw = tile > 0 ? flags + (size_t)J.flag_base * kFlagStride : nullptr;
            const uint32_t target = base + epoch;  // the epoch every member raised at the end of the last tile
            if (d.own_r0 == d.own_r1) {
                const int64_t per = (steps + P.k - 1) / P.k - 1;
                epoch += per > 0 ? (uint32_t)per : 1u;
                if (gw != nullptr) gate_wait<2>(gw, target, J.g, gate_peek<2>(gw, target, J.g), err, spin_limit);
            } else if (halo_varies<T, C, R, WAVES, COLMASK>(P, d)) {
                run_segment<T, C, R, WAVES, FMA, COLMASK, true, true, false, true, 5, 2>(
                    P, d, A, B, steps, me, flags, base, epoch, err, spin_limit, lds, gw, target, J.g);
            } else {
                run_segment<T, C, R, WAVES, FMA, COLMASK, true, false, false, true, 5, 2>(
                    P, d, A, B, steps, me, flags, base, epoch, err, spin_limit, lds, gw, target, J.g);
            }
            ++epoch;
            if (tile + 1 < J.ntiles) {
                // Arrive: this member is done with the tile (its ring loads have returned).
                if (threadIdx.x == 0)
                    __hip_atomic_store(flags + (size_t)me * kFlagStride, base + epoch, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            } else {
                group_point(flags, J.flag_base, J.g, local, base + epoch, err, spin_limit, true);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        }
        done += steps;
    }
    // Members idle in the last tiles have not published their final epoch;
    // every member's flag must end at the same value (the next run counts from it).
    if (threadIdx.x == 0) __hip_atomic_store(flags + (size_t)me * kFlagStride, base + epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (J.nrounds & 1) {
        // The result is in the second buffer: copy the interior back.
        const int64_t n = (int64_t)rows * cols;
        for (int64_t idx = tid; idx < n; idx += nthr) {
            const int64_t i = 1 + idx / cols, j = 1 + idx % cols;
            grid[i * pitch + j] = __hip_atomic_load(ws + i * pitch + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// The register-tile instances of the batched kernel: two shapes per
// precision (a taller and a wider one) with the same cells per lane.
constexpr int kBatchR64a = 16, kBatchC64a = 2;  // FP64 128 x 128
constexpr int kBatchR64b = 8, kBatchC64b = 4;   // FP64 64 x 256
constexpr int kBatchR32a = 16, kBatchC32a = 4;  // FP32 128 x 256
constexpr int kBatchR32b = 8, kBatchC32b = 4;   // FP32 64 x 256

constexpr size_t max_sz(size_t a, size_t b) { return a > b ? a : b; }

// One job with the instance the planner chose for it.
template <typename T, int C, int R, bool FMA>
__device__ __forceinline__ void run_job_any(const ProbDesc& P, const JobDesc& J, const WgDesc* __restrict__ table,
                                            int local, uint32_t* flags, int* err, uint32_t spin_limit, char* lds)
{
    if (P.narrow_cols) run_job<T, C, R, kDtbWaves, FMA, true>(P, J, table, local, flags, err, spin_limit, lds);
    else run_job<T, C, R, kDtbWaves, FMA, false>(P, J, table, local, flags, err, spin_limit, lds);
}

// Many grids of uneven sizes, step counts and precisions in one persistent
// launch.  Launch slot b works through its list of (job, member) items in the
// global job order the planner chose (so no two jobs can wait on each other).
// Each job runs with the register-tile instance the planner chose for it;
// rows are always checked against the grid (small grids leave rows idle).
template <bool FMA>
__global__ __launch_bounds__(kDtbWaves * 64) void k_dtb_batched(const ProbDesc* __restrict__ probs,
                                                                const JobDesc* __restrict__ jobs,
                                                                const WgDesc* __restrict__ table,
                                                                const int* __restrict__ wl_off,
                                                                const WorkItem* __restrict__ wl, uint32_t* flags,
                                                                int* err, uint32_t spin_limit)
{
    constexpr size_t kLds = max_sz(max_sz(Geo<double, kBatchC64a, kBatchR64a, kDtbWaves>::kLdsBytes,
                                          Geo<double, kBatchC64b, kBatchR64b, kDtbWaves>::kLdsBytes),
                                   max_sz(Geo<float, kBatchC32a, kBatchR32a, kDtbWaves>::kLdsBytes,
                                          Geo<float, kBatchC32b, kBatchR32b, kDtbWaves>::kLdsBytes));
    __shared__ __attribute__((aligned(16))) char lds[kLds];
    const int slot = blockIdx.x;
    for (int i = wl_off[slot]; i < wl_off[slot + 1]; ++i) {
        const WorkItem w = wl[i];
        const JobDesc& J = jobs[w.job];
        const ProbDesc& P = probs[J.prob];
        if (P.dtype == 0) {
            if (J.C == kBatchC64b && J.R == kBatchR64b)
                run_job_any<double, kBatchC64b, kBatchR64b, FMA>(P, J, table, w.local, flags, err, spin_limit, lds);
            else
                run_job_any<double, kBatchC64a, kBatchR64a, FMA>(P, J, table, w.local, flags, err, spin_limit, lds);
        } else {
            if (J.C == kBatchC32b && J.R == kBatchR32b)
                run_job_any<float, kBatchC32b, kBatchR32b, FMA>(P, J, table, w.local, flags, err, spin_limit, lds);
            else
                run_job_any<float, kBatchC32a, kBatchR32a, FMA>(P, J, table, w.local, flags, err, spin_limit, lds);
        }
        __syncthreads();
    }
}

// The kernels of one (precision, columns per lane, rows per lane, waves,
// stencil) instance: kind 0 resident (k_dtb), 1 tile-serial sweep
// (k_dtb_sweep), 2 overlapped per-workgroup blocking (k_ovl, only where OVL is
// set), each in 8 variants (fma, colmask, rowcheck); nullptr where there is none.
template <typename T, int C, int R, int WAVES, bool OVL, bool F, bool M, bool W, int PTS>
const void* kernel_of(int kind)
{
    if (kind == 0) return (const void*)&k_dtb<T, C, R, WAVES, F, M, W, PTS>;
    if (kind == 1) return (const void*)&k_dtb_sweep<T, C, R, WAVES, F, M, W, PTS>;
    if constexpr (OVL) {
        if (kind == 2) return (const void*)&k_ovl<T, C, R, WAVES, F, M, W>;
    }
    return nullptr;
}

template <typename T, int C, int R, int WAVES = kDtbWaves, bool OVL = false, int PTS = 5>
const void* pick_instance(int kind, bool fma, bool colmask, bool rowcheck)
{
    switch ((fma ? 4 : 0) | (colmask ? 2 : 0) | (rowcheck ? 1 : 0)) {
    case 0: return kernel_of<T, C, R, WAVES, OVL, false, false, false, PTS>(kind);
    case 1: return kernel_of<T, C, R, WAVES, OVL, false, false, true, PTS>(kind);
    case 2: return kernel_of<T, C, R, WAVES, OVL, false, true, false, PTS>(kind);
    case 3: return kernel_of<T, C, R, WAVES, OVL, false, true, true, PTS>(kind);
    case 4: return kernel_of<T, C, R, WAVES, OVL, true, false, false, PTS>(kind);
    case 5: return kernel_of<T, C, R, WAVES, OVL, true, false, true, PTS>(kind);
    case 6: return kernel_of<T, C, R, WAVES, OVL, true, true, false, PTS>(kind);
    default: return kernel_of<T, C, R, WAVES, OVL, true, true, true, PTS>(kind);
    }
}

}  // namespace dtb
