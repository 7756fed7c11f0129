// dtb_api.cpp -- the libdtb C ABI: argument checks, plans, plan cache, launches.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dtb.h"
#include "../../include/dtb_testing.h"
#include "dtb_internal.h"
#include "dtb_launch.h"
#include "dtb_plan.h"

using namespace dtb;

namespace {

constexpr uint32_t kSpinLimit = 1u << 22;  // bounded wait: a few seconds of polling
constexpr size_t kBarrierWords = kBarrierSlots * (size_t)kFlagStride;  // device-wide barrier counters, one slot each
constexpr int kNumXcd = 8;                 // MI355X: 8 XCDs, workgroups dealt round-robin
// Instantiated rows per lane: FP64 8, 16, 24 (2 columns per lane) and 12 (4 columns); FP32 8, 16, 24, 28.
constexpr int kDtbRowsPerLane[] = {8, 12, 16, 24, 28};

struct DeviceInfo {
    int device = -1;
    int n_cu = 0;
};

bool device_info(DeviceInfo* di)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    di->device = dev;
    di->n_cu = ncu;
    return true;
}

}  // namespace

struct dtb_plan_s {
    int device = -1;
    int64_t rows = 0, cols = 0, pitch = 0;
    int dtype = 0;
    int pts = 5;  // stencil: 5 (j2d5pt) or 9 (the 3 x 3 box)
    int path = DTB_PATH_STEP;
    bool fma = true;
    // one-step path
    void* ws = nullptr;
    // resident path
    Layout layout;
    const void* kfunc = nullptr;
    bool colmask = false, rowcheck = false;
    WgDesc* d_wgs = nullptr;
    uint32_t* d_flags = nullptr;
    int* d_err = nullptr;
    void* xbuf[2] = {nullptr, nullptr};
    // tile-serial sweep (uses ws as its second buffer)
    SweepPlan sweep;
    // overlapped per-workgroup blocking (layout with k = D, ws as its second buffer)
    int ovl_D = 0;
    // j3d7pt (dtb_plan3d): 2.5D streaming, K steps per launch over ntiles3 (x, y) tiles x nzb z-blocks
    bool is3d = false;
    int64_t depth = 0, plane_pitch = 0;
    int K3 = 0, zb = 0, nzb = 0, ntiles3 = 0, ty3 = 0, tx3 = 0, R3 = 0, C3 = 0;
    Tile3Desc* d_tiles3 = nullptr;
    bool grid_sync = false;  // resident path: device-wide barrier at every exchange
    uint32_t* d_bar = nullptr;
    int nwg_launch = 0;
    int debug = 0;
    uint64_t* d_timing = nullptr;  // DTB_DEBUG_TIMING
    // The workspace serves one run at a time: the last run's stream and an
    // event recorded after it, which a run on another stream waits for.
    hipEvent_t done = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_run = false;

    uint32_t spin_limit() const { return (debug & DTB_DEBUG_TINY_SPIN) ? 4u : kSpinLimit; }

    ~dtb_plan_s()
    {
        if (done) (void)hipEventDestroy(done);
        if (ws) (void)hipFree(ws);
        if (d_bar) (void)hipFree(d_bar);
        if (d_timing) (void)hipFree(d_timing);
        if (d_wgs) (void)hipFree(d_wgs);
        if (d_flags) (void)hipFree(d_flags);
        if (d_err) (void)hipFree(d_err);
        if (d_tiles3) (void)hipFree(d_tiles3);
        for (void* p : xbuf)
            if (p) (void)hipFree(p);
    }
};

namespace {

size_t elem_size(int dtype) { return dtype == DTB_F64 ? 8 : 4; }

dtb_status check_shape(int64_t rows, int64_t cols, int64_t pitch, int dtype)
{
    if (rows < 1 || cols < 1 || pitch < cols + 2) return DTB_ERR_INVALID_ARG;
    if (dtype != DTB_F64 && dtype != DTB_F32) return DTB_ERR_INVALID_ARG;
    // Descriptors and kernel index math are 32-bit in rows/cols.
    if (rows > (1 << 30) || cols > (1 << 30)) return DTB_ERR_UNSUPPORTED;
    return DTB_OK;
}

dtb_status check_opts(const dtb_plan_opts* o)
{
    if (!o) return DTB_OK;
    if (o->path < DTB_PATH_AUTO || o->path > DTB_PATH_STREAM3D) return DTB_ERR_INVALID_ARG;
    if (o->sync != 0 && o->sync != 1) return DTB_ERR_INVALID_ARG;
    if (o->stencil != 0 && o->stencil != 5 && o->stencil != 7 && o->stencil != 9) return DTB_ERR_INVALID_ARG;
    if (o->ghost_k < 0 || o->depth_D < 0 || o->rows_per_lane < 0 || o->max_wg < 0 || o->cols_per_lane < 0)
        return DTB_ERR_INVALID_ARG;
    if (o->waves != 0 && o->waves != 4 && o->waves != 8) return DTB_ERR_INVALID_ARG;
    if (o->exact != 0 && o->exact != 1) return DTB_ERR_INVALID_ARG;
    if ((o->debug_flags & ~(DTB_DEBUG_TINY_SPIN | DTB_DEBUG_POISON | DTB_DEBUG_TIMING | DTB_DEBUG_DIRECT_XCHG)) != 0 ||
        (o->tune != 0 && o->tune != 1))
        return DTB_ERR_INVALID_ARG;
    return DTB_OK;
}

int stencil_points(const dtb_plan_opts& o) { return o.stencil == 9 ? 9 : 5; }

// A requested tile instance must exist: FP64 8, 12, 16, 24 rows per lane and,
// with 4 waves per workgroup, 24 rows on the resident path only; FP32 8, 16,
// 24, 28 rows with 8 waves.  The box stencil: FP64 8 and FP32 16 rows, 8
// waves, resident and sweep paths, neighbour flags.  Checked before any HIP call.
dtb_status check_instance(const dtb_plan_opts& o, int dtype)
{
    if (o.stencil == 7 || o.path == DTB_PATH_STREAM3D) return DTB_ERR_UNSUPPORTED;  // 3-D: dtb_plan3d
    if (o.cols_per_lane != 0) return DTB_ERR_UNSUPPORTED;  // the 2-D instances are chosen by rows_per_lane
    const int pts = stencil_points(o);
    if (pts == 9 && (o.path == DTB_PATH_OVERLAPPED || o.waves == 4 || o.sync == 1)) return DTB_ERR_UNSUPPORTED;
    if (o.path == DTB_PATH_STEP) return DTB_OK;
    if (o.waves == 4 && (dtype != DTB_F64 || o.path == DTB_PATH_SWEEP || o.path == DTB_PATH_OVERLAPPED ||
                         (o.rows_per_lane != 0 && o.rows_per_lane != 24)))
        return DTB_ERR_UNSUPPORTED;
    // The device-wide barrier variant exists for the resident path only.
    if (o.sync == 1 && (o.path == DTB_PATH_SWEEP || o.path == DTB_PATH_OVERLAPPED || o.tune)) return DTB_ERR_UNSUPPORTED;
    if (o.rows_per_lane > 0) {
        int C = 0, waves = 0;
        const void* f = o.path == DTB_PATH_SWEEP ? dtb_sweep_kernel(dtype, o.rows_per_lane, true, false, false, &C, &waves, pts)
                      : o.path == DTB_PATH_OVERLAPPED ? dtb_ovl_kernel(dtype, o.rows_per_lane, true, false, false, &C, &waves)
                      : dtb_kernel(dtype, o.rows_per_lane, true, false, false, &C, &waves, o.waves, pts);
        if (!f) return DTB_ERR_UNSUPPORTED;
    }
    return DTB_OK;
}

// A kernel instance whose registers spill to scratch is never chosen.
// Scratch bytes per lane of a kernel (registers spilled), or -1 if unknown.
int64_t spill_bytes(const void* f)
{
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, f) != hipSuccess) return -1;
    return (int64_t)a.localSizeBytes;
}

bool spills(const void* f) { return spill_bytes(f) != 0; }

// The sweep may take a kernel that spills a few words (in the sweep kernels
// these are tile-loop values, reloaded once per big tile), priced like any
// other: measured at 16384^2 FP32, 24 rows per lane with 16 bytes of spill
// beat the 16-row tile by 6 %, and at 3072^2 FP64 24 rows per lane (12 bytes)
// beat the 16-row tile by 13 % (1572 against 1385 GCells/s), an order that a
// 10 % penalty on spilling kernels used to reverse.
constexpr int64_t kSweepSpillSlack = 32;

// Choose (rows per lane, k) for the resident path by the static cost model.
bool choose_resident(int64_t rows, int64_t cols, int dtype, const dtb_plan_opts& o, int n_cu, bool fma,
                     Layout* best_layout, const void** best_func, bool* colmask, bool* rowcheck)
{
    const int pts = stencil_points(o);
    double best = 1e300;
    bool found = false;
    // Every ring depth from 2 to 24: with all tiles running side by side, the
    // deepest ring whose tiles still fit on the chip usually wins (2048^2 FP64:
    // k = 11 fits 252 tiles of 96 x 256, k = 12 would need 261).
    std::vector<int> ks;
    if (o.ghost_k > 0) ks.push_back(o.ghost_k);
    else
        for (int k = 2; k <= 24; ++k) ks.push_back(k);
    for (int R : kDtbRowsPerLane) {
        if (o.rows_per_lane > 0 && o.rows_per_lane != R) continue;
        // Half-height workgroups only on request: measured slower than full
        // height at 2048^2 (2.62 vs 2.35 us per step).
        for (int want_waves : {8, 4})
        for (int k : ks) {
            if (o.waves != want_waves && !(o.waves == 0 && want_waves == 8)) continue;
            int C = 0, waves = 0;
            const void* f0 = dtb_kernel(dtype, R, fma, false, false, &C, &waves, want_waves, pts);
            if (!f0) continue;
            Layout L;
            // No more tiles than can be co-resident (at most two workgroups per compute unit): larger
            // layouts are not even built (at 16384^2 they run to 10^5 tiles).
            if (!build_layout(rows, cols, interior(rows, cols), interior(rows, cols), R, C, waves, k, kNumXcd, 0, 0, &L,
                              true, 2 * n_cu))
                continue;
            const bool cm = L.cols.narrow, rc = L.rows.narrow;
            const void* f = dtb_kernel(dtype, R, fma, cm, rc, &C, &waves, want_waves, pts);
            if (spills(f)) continue;
            int occ = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, waves * kWaveSize, 0) != hipSuccess) continue;
            int cap = occ * n_cu;
            if (o.max_wg > 0) cap = std::min(cap, o.max_wg);
            if (L.nwg > cap) continue;
            const double cost = layout_cost(L, occ, n_cu, dtype == DTB_F64 ? 8 : 4, pts);
            if (cost < best) {
                best = cost;
                *best_layout = L;
                *best_func = f;
                *colmask = cm;
                *rowcheck = rc;
                found = true;
            }
        }
    }
    return found;
}

// Model of one time step of the sweep, in microseconds: every big tile runs
// D steps on the whole chip (VALU time of one register tile per step), one
// exchange every k steps, a fixed cost per big tile (the tile load's latency
// and the synchronisation between big tiles), and its HBM traffic (load of
// the computed region, store of the valid part) once per D steps.
double sweep_step_us(const SweepPlan& sp, int dtype, int pts)
{
    const int eb = dtype == DTB_F64 ? 8 : 4;
    const double t_step = tile_step_time_us(sp.ER, sp.EC, eb, pts);
    const double t_exch = exchange_time_us(sp.ER, sp.EC, sp.R, sp.C, eb, exchange_staged(sp.R, sp.C, eb, sp.k));
    const double t_bar = 10.0;  // per big tile: the tile load's latency and the barrier between big tiles
    const double hbm_bytes_per_us = 4.0e6;
    const double b = dtype == DTB_F64 ? 8.0 : 4.0;
    double total = 0;
    for (const Layout& L : sp.tiles) {
        const double cr = (double)(L.rows.bounds.back() - L.rows.bounds.front()) *
                          (L.cols.bounds.back() - L.cols.bounds.front());
        const double io = (cr * b + cr * b) / hbm_bytes_per_us;  // upper bound: store <= load
        total += sp.D * t_step + ((double)sp.D / sp.k) * t_exch + t_bar + io;
    }
    return total / sp.D;
}

// Overlapped per-workgroup blocking: every workgroup runs D steps on its own
// tile and moves the tile through HBM once per D steps.  Model per time step:
// the workgroups run in ceil(nwg / slots) waves; each workgroup spends D
// register-tile steps plus its tile's load and store at its share of HBM
// bandwidth (4 TB/s over the slots) -- a load cannot overlap the tile's own
// steps.
double overlapped_step_us(const Layout& L, int slots, int elem_bytes)
{
    const double waves = std::ceil((double)L.nwg / std::max(slots, 1));
    const double t_step = tile_step_time_us(L.ER, L.EC, elem_bytes);
    const double io = (double)L.ER * L.EC * elem_bytes * 2.0 / (4.0e6 / std::max(slots, 1)) + 2.0;
    return waves * (L.k * t_step + io) / L.k;
}

bool choose_overlapped(int64_t rows, int64_t cols, int dtype, const dtb_plan_opts& o, int n_cu, bool fma,
                       Layout* best_layout, const void** best_func, bool* colmask, bool* rowcheck)
{
    double best = 1e300;
    bool found = false;
    std::vector<int> Ds;
    if (o.depth_D > 0) Ds.push_back(o.depth_D);
    else
        for (int D = 2; D <= 32; ++D) Ds.push_back(D);
    for (int R : kDtbRowsPerLane) {
        if (o.rows_per_lane > 0 && o.rows_per_lane != R) continue;
        int C = 0, waves = 0;
        if (!dtb_ovl_kernel(dtype, R, fma, false, false, &C, &waves)) continue;
        for (int D : Ds) {
            Layout L;
            if (!build_layout(rows, cols, interior(rows, cols), interior(rows, cols), R, C, waves, D, kNumXcd, 0, 0, &L,
                              false))
                continue;
            const bool cm = L.cols.narrow, rc = L.rows.narrow;
            const void* f = dtb_ovl_kernel(dtype, R, fma, cm, rc, &C, &waves);
            if (!f || spills(f)) continue;
            int occ = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, waves * kWaveSize, 0) != hipSuccess || occ < 1)
                continue;
            int slots = occ * n_cu;
            if (o.max_wg > 0) slots = std::min(slots, o.max_wg);
            const double cost = overlapped_step_us(L, slots, dtype == DTB_F64 ? 8 : 4);
            if (cost < best) {
                best = cost;
                *best_layout = std::move(L);
                *best_func = f;
                *colmask = cm;
                *rowcheck = rc;
                found = true;
            }
        }
    }
    return found;
}

bool choose_sweep(int64_t rows, int64_t cols, int dtype, const dtb_plan_opts& o, int n_cu, bool fma, SweepPlan* best,
                  const void** best_func, bool* colmask, bool* rowcheck, int* nwg_cap)
{
    const int pts = stencil_points(o);
    double best_t = 1e300;
    bool found = false;
    std::vector<int> ks, Ds;
    if (o.ghost_k > 0) ks.push_back(o.ghost_k);
    else ks = {4, 6, 8, 10, 12};
    if (o.depth_D > 0) Ds.push_back(o.depth_D);
    else Ds = {8, 16, 24, 32, 48, 64, 96, 128, 192};
    for (int R : kDtbRowsPerLane) {
        if (o.rows_per_lane > 0 && o.rows_per_lane != R) continue;
        int C = 0, waves = 0;
        if (!dtb_sweep_kernel(dtype, R, fma, false, false, &C, &waves, pts)) continue;
        const bool cm = cols < kWaveSize * C, rc = rows < waves * R;
        const void* f = dtb_sweep_kernel(dtype, R, fma, cm, rc, &C, &waves, pts);
        const int64_t sb = spill_bytes(f);
        if (sb < 0 || sb > kSweepSpillSlack) continue;
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, waves * kWaveSize, 0) != hipSuccess) continue;
        int cap = std::min(occ, 1) * n_cu;  // one tile per compute unit: the tiles of a big tile run side by side
        if (o.max_wg > 0) cap = std::min(cap, o.max_wg);
        if (cap < 1) continue;
        for (int k : ks) {
            for (int D : Ds) {
                SweepPlan sp;
                if (!plan_sweep(rows, cols, R, C, waves, k, D, cap, kNumXcd, &sp)) continue;
                const double t = sweep_step_us(sp, dtype, pts);
                if (t < best_t) {
                    best_t = t;
                    *best = std::move(sp);
                    *best_func = f;
                    *colmask = cm;
                    *rowcheck = rc;
                    *nwg_cap = cap;
                    found = true;
                }
            }
        }
    }
    return found;
}

dtb_status plan_impl(dtb_plan_t* out, int64_t rows, int64_t cols, int64_t pitch, int dtype, int64_t T_hint,
                     const dtb_plan_opts* opts);
dtb_status run_plan_impl(dtb_plan_t p, const dtb_grid* g, const double* coeffs, int64_t T, void* stream);

// ---- autotuner: timed trials of the model's best candidates

struct TuneChoice {
    int path = 0, R = 0, k = 0, D = 0;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune;
bool g_tune_loaded = false;

std::string tune_key(int64_t rows, int64_t cols, int64_t pitch, int dtype, int pts, int exact, int64_t T_hint,
                     int max_wg)
{
    hipDeviceProp_t prop{};
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    // Step counts in power-of-two buckets: the best exchange/round depth changes slowly with T.
    int tb = 0;
    while ((int64_t(1) << tb) < T_hint && tb < 62) ++tb;
    char buf[256];
    snprintf(buf, sizeof(buf), "%lld,%lld,%lld,%d,%d,%d,%d,%d,%s,%d", (long long)rows, (long long)cols,
             (long long)pitch, dtype, pts, exact, tb, max_wg, prop.gcnArchName, prop.multiProcessorCount);
    return buf;
}

void tune_cache_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("DTB_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
        // key<TAB>path R k D
        char* tab = strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        TuneChoice c;
        if (sscanf(tab + 1, "%d %d %d %d", &c.path, &c.R, &c.k, &c.D) == 4) g_tune[line] = c;
    }
    fclose(f);
}

void tune_cache_store(const std::string& key, const TuneChoice& c)
{
    g_tune[key] = c;
    const char* path = getenv("DTB_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s\t%d %d %d %d\n", key.c_str(), c.path, c.R, c.k, c.D);
    fclose(f);
}

// Candidates ranked by the static model, best first.
std::vector<std::pair<double, TuneChoice>> tune_candidates(int64_t rows, int64_t cols, int dtype,
                                                           const dtb_plan_opts& o, int n_cu)
{
    std::vector<std::pair<double, TuneChoice>> out;
    const bool fma = o.exact == 0;
    const int pts = stencil_points(o);
    for (int R : kDtbRowsPerLane) {
        if (o.rows_per_lane > 0 && o.rows_per_lane != R) continue;
        int C = 0, waves = 0;
        if (!dtb_kernel(dtype, R, fma, false, false, &C, &waves, 0, pts)) continue;
        for (int k : {2, 4, 6, 8, 10, 12, 16, 20, 24}) {
            if (o.ghost_k > 0 && o.ghost_k != k) continue;
            if (o.path == DTB_PATH_AUTO || o.path == DTB_PATH_RESIDENT) {
                Layout L;
                if (build_layout(rows, cols, interior(rows, cols), interior(rows, cols), R, C, waves, k, kNumXcd, 0,
                                 0, &L, true, 2 * n_cu)) {
                    const void* f = dtb_kernel(dtype, R, fma, L.cols.narrow, L.rows.narrow, &C, &waves, 0, pts);
                    int occ = 0;
                    if (f && !spills(f) &&
                        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, waves * kWaveSize, 0) == hipSuccess) {
                        int cap = occ * n_cu;
                        if (o.max_wg > 0) cap = std::min(cap, o.max_wg);
                        if (L.nwg <= cap)
                            out.push_back({layout_cost(L, occ, n_cu, dtype == DTB_F64 ? 8 : 4, pts),
                                           TuneChoice{DTB_PATH_RESIDENT, R, k, 0}});
                    }
                }
            }
            if (o.path == DTB_PATH_SWEEP || (o.path == DTB_PATH_AUTO && out.empty())) {
                const bool cm = cols < kWaveSize * C, rc = rows < waves * R;
                const void* f = dtb_sweep_kernel(dtype, R, fma, cm, rc, &C, &waves, pts);
                if (!f || spills(f)) continue;
                const int cap = o.max_wg > 0 ? std::min(n_cu, o.max_wg) : n_cu;
                for (int D : {16, 32, 48, 64, 96, 128, 192}) {
                    if (o.depth_D > 0 && o.depth_D != D) continue;
                    SweepPlan sp;
                    if (!plan_sweep(rows, cols, R, C, waves, k, D, cap, kNumXcd, &sp)) continue;
                    out.push_back({sweep_step_us(sp, dtype, pts), TuneChoice{DTB_PATH_SWEEP, R, k, D}});
                }
            }
        }
    }
    std::stable_sort(out.begin(), out.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    return out;
}

// Time a plan built with `c` on a zero-filled scratch grid: best of two runs of `steps` steps.
double time_candidate(int64_t rows, int64_t cols, int64_t pitch, int dtype, const dtb_plan_opts& base,
                      const TuneChoice& c, void* scratch, int64_t steps)
{
    dtb_plan_opts o = base;
    o.tune = 0;
    o.path = c.path;
    o.rows_per_lane = c.R;
    o.ghost_k = c.k;
    o.depth_D = c.D;
    dtb_plan_t p = nullptr;
    if (plan_impl(&p, rows, cols, pitch, dtype, steps, &o) != DTB_OK) return 1e300;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best = 1e300;
    double coeffs[9];
    for (double& c : coeffs) c = 1.0 / stencil_points(o);  // weights summing to 1: the zero grid stays zero
    const dtb_grid g{scratch, rows, cols, pitch};
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess) {
        if (run_plan_impl(p, &g, coeffs, steps, st) == DTB_OK && hipStreamSynchronize(st) == hipSuccess) {
            for (int rep = 0; rep < 2; ++rep) {
                (void)hipEventRecord(e0, st);
                if (run_plan_impl(p, &g, coeffs, steps, st) != DTB_OK) break;
                (void)hipEventRecord(e1, st);
                if (hipEventSynchronize(e1) != hipSuccess) break;
                float ms = 0;
                if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = std::min(best, (double)ms);
            }
        }
        int e = 0;
        if (p->d_err && hipMemcpy(&e, p->d_err, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess && e) best = 1e300;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    dtb_plan_destroy(p);
    return best / steps;
}

dtb_status tune_plan(dtb_plan_t* out, int64_t rows, int64_t cols, int64_t pitch, int dtype, int64_t T_hint,
                     const dtb_plan_opts& o)
{
    DeviceInfo di;
    if (!device_info(&di)) return DTB_ERR_HIP;
    const std::string key = tune_key(rows, cols, pitch, dtype, stencil_points(o), o.exact, T_hint, o.max_wg);
    TuneChoice choice;
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_load();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            choice = it->second;
            have = true;
        }
    }
    if (!have) {
        auto cands = tune_candidates(rows, cols, dtype, o, di.n_cu);
        if (cands.empty()) return DTB_ERR_NOT_CORESIDENT;
        if (cands.size() > 6) cands.resize(6);
        void* scratch = nullptr;
        const size_t bytes = (size_t)(rows + 2) * (size_t)pitch * elem_size(dtype);
        if (hipMalloc(&scratch, bytes) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMemset(scratch, 0, bytes) != hipSuccess) {
            (void)hipFree(scratch);
            return DTB_ERR_HIP;
        }
        double best = 1e300;
        for (auto& c : cands) {
            int64_t steps = c.second.path == DTB_PATH_SWEEP ? 2 * (int64_t)c.second.D : 8 * (int64_t)c.second.k;
            if (T_hint > 0) steps = std::min<int64_t>(steps, std::max<int64_t>(T_hint, 1));
            const double t = time_candidate(rows, cols, pitch, dtype, o, c.second, scratch, std::max<int64_t>(steps, 2));
            if (t < best) {
                best = t;
                choice = c.second;
                have = true;
            }
        }
        (void)hipFree(scratch);
        if (!have || best >= 1e299) return DTB_ERR_HIP;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_store(key, choice);
    }
    dtb_plan_opts fixed = o;
    fixed.tune = 0;
    fixed.path = choice.path;
    fixed.rows_per_lane = choice.R;
    fixed.ghost_k = choice.k;
    fixed.depth_D = choice.D;
    return plan_impl(out, rows, cols, pitch, dtype, T_hint, &fixed);
}

dtb_status plan_impl(dtb_plan_t* out, int64_t rows, int64_t cols, int64_t pitch, int dtype, int64_t T_hint,
                     const dtb_plan_opts* opts)
{
    if (!out) return DTB_ERR_INVALID_ARG;
    *out = nullptr;
    dtb_status st = check_shape(rows, cols, pitch, dtype);
    if (st != DTB_OK) return st;
    st = check_opts(opts);
    if (st != DTB_OK) return st;
    dtb_plan_opts o{};
    if (opts) o = *opts;
    st = check_instance(o, dtype);
    if (st != DTB_OK) return st;
    if (o.tune && o.path != DTB_PATH_STEP && o.path != DTB_PATH_OVERLAPPED)
        return tune_plan(out, rows, cols, pitch, dtype, T_hint, o);

    DeviceInfo di;
    if (!device_info(&di)) return DTB_ERR_HIP;
    std::unique_ptr<dtb_plan_s> p(new dtb_plan_s());
    p->device = di.device;
    p->rows = rows;
    p->cols = cols;
    p->pitch = pitch;
    p->dtype = dtype;
    p->fma = o.exact == 0;
    p->pts = stencil_points(o);
    p->debug = o.debug_flags;
    const size_t bytes = (size_t)(rows + 2) * (size_t)pitch * elem_size(dtype);

    int path = o.path;
    if (path == DTB_PATH_OVERLAPPED) {
        Layout L;
        const void* f = nullptr;
        bool cm = false, rc = false;
        if (!choose_overlapped(rows, cols, dtype, o, di.n_cu, p->fma, &L, &f, &cm, &rc)) return DTB_ERR_UNSUPPORTED;
        p->ovl_D = L.k;
        p->layout = std::move(L);
        p->kfunc = f;
        p->colmask = cm;
        p->rowcheck = rc;
    }
    if (path == DTB_PATH_AUTO || path == DTB_PATH_RESIDENT) {
        Layout L;
        const void* f = nullptr;
        bool cm = false, rc = false;
        if (choose_resident(rows, cols, dtype, o, di.n_cu, p->fma, &L, &f, &cm, &rc)) {
            path = DTB_PATH_RESIDENT;
            p->layout = std::move(L);
            p->kfunc = f;
            p->colmask = cm;
            p->rowcheck = rc;
        } else if (path == DTB_PATH_RESIDENT) {
            return DTB_ERR_NOT_CORESIDENT;
        } else {
            path = DTB_PATH_SWEEP;  // larger than the chip: big tiles one after another
        }
    }
    if (o.sync == 1) {
        if (path != DTB_PATH_RESIDENT) return DTB_ERR_UNSUPPORTED;
        p->grid_sync = true;
    }
    if (path == DTB_PATH_SWEEP) {
        const void* f = nullptr;
        bool cm = false, rc = false;
        int cap = 0;
        if (!choose_sweep(rows, cols, dtype, o, di.n_cu, p->fma, &p->sweep, &f, &cm, &rc, &cap))
            return DTB_ERR_NOT_CORESIDENT;
        p->kfunc = f;
        p->colmask = cm;
        p->rowcheck = rc;
        p->nwg_launch = p->sweep.nwg;
        p->layout = p->sweep.tiles.front();  // for describe()
    }
    p->path = path;

    if (path == DTB_PATH_STEP) {
        if (hipMalloc(&p->ws, bytes) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
    } else if (path == DTB_PATH_OVERLAPPED) {
        const size_t nwg = p->layout.wgs.size();
        if (hipMalloc(&p->ws, bytes) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&p->d_wgs, nwg * sizeof(WgDesc)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMemcpy(p->d_wgs, p->layout.wgs.data(), nwg * sizeof(WgDesc), hipMemcpyHostToDevice) != hipSuccess)
            return DTB_ERR_HIP;
    } else if (path == DTB_PATH_SWEEP) {
        const size_t n = p->sweep.table.size();
        const size_t nwg = (size_t)p->nwg_launch;
        if (hipMalloc(&p->ws, bytes) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&p->d_wgs, n * sizeof(WgDesc)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&p->d_flags, nwg * kFlagStride * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&p->d_err, sizeof(int)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&p->d_bar, kBarrierWords * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        for (int i = 0; i < 2; ++i)
            if (hipMalloc(&p->xbuf[i], bytes) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMemcpy(p->d_wgs, p->sweep.table.data(), n * sizeof(WgDesc), hipMemcpyHostToDevice) != hipSuccess)
            return DTB_ERR_HIP;
        if (hipMemset(p->d_flags, 0, nwg * kFlagStride * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_HIP;
        if (hipMemset(p->d_err, 0, sizeof(int)) != hipSuccess) return DTB_ERR_HIP;
        if (hipMemset(p->d_bar, 0, kBarrierWords * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_HIP;
    } else {
        const size_t nwg = p->layout.wgs.size();
        if (hipMalloc(&p->d_wgs, nwg * sizeof(WgDesc)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&p->d_flags, nwg * kFlagStride * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&p->d_err, sizeof(int)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        for (int i = 0; i < 2; ++i)
            if (hipMalloc(&p->xbuf[i], bytes) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMemcpy(p->d_wgs, p->layout.wgs.data(), nwg * sizeof(WgDesc), hipMemcpyHostToDevice) != hipSuccess)
            return DTB_ERR_HIP;
        if (hipMemset(p->d_flags, 0, nwg * kFlagStride * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_HIP;
        if (hipMemset(p->d_err, 0, sizeof(int)) != hipSuccess) return DTB_ERR_HIP;
        if (p->grid_sync) {
            if (hipMalloc(&p->d_bar, kBarrierWords * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
            if (hipMemset(p->d_bar, 0, kBarrierWords * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_HIP;
        }
    }
    if (hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) return DTB_ERR_HIP;
    if ((p->debug & DTB_DEBUG_TIMING) && path != DTB_PATH_STEP && path != DTB_PATH_OVERLAPPED) {
        const size_t n = (size_t)std::max<int>(p->nwg_launch, p->layout.nwg) * kTimingSlots;
        if (hipMalloc(&p->d_timing, n * sizeof(uint64_t)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMemset(p->d_timing, 0, n * sizeof(uint64_t)) != hipSuccess) return DTB_ERR_HIP;
    }
    *out = p.release();
    return DTB_OK;
}

dtb_status run_step(dtb_plan_t p, void* data, const double* coeffs, int64_t T, hipStream_t st)
{
    const int rows = (int)p->rows, cols = (int)p->cols;
    if (launch_copy_halo(p->dtype, data, p->ws, p->pitch, rows, cols, st) != hipSuccess) return DTB_ERR_HIP;
    void* in = data;
    void* out = p->ws;
    for (int64_t t = 0; t < T; ++t) {
        if (launch_step(p->dtype, p->fma, in, out, p->pitch, rows, cols, coeffs, st, p->pts) != hipSuccess)
            return DTB_ERR_HIP;
        std::swap(in, out);
    }
    if (in != data) {
        if (launch_copy_interior(p->dtype, in, data, p->pitch, rows, cols, st) != hipSuccess) return DTB_ERR_HIP;
    }
    return DTB_OK;
}

// Debug: fill the exchange buffers with NaN before a run, so a ghost cell
// that was never published in this run shows up in the result.
dtb_status poison_xbufs(dtb_plan_t p, hipStream_t st)
{
    if (!(p->debug & DTB_DEBUG_POISON)) return DTB_OK;
    // A debug aid for direct launches only: memset nodes recorded into a
    // captured graph are not replayed reliably.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return DTB_ERR_HIP;
    if (cs != hipStreamCaptureStatusNone) return DTB_ERR_UNSUPPORTED;
    const size_t bytes = (size_t)(p->rows + 2) * (size_t)p->pitch * elem_size(p->dtype);
    for (void* x : p->xbuf)
        if (x && hipMemsetAsync(x, 0xFF, bytes, st) != hipSuccess) return DTB_ERR_HIP;
    return DTB_OK;
}

dtb_status run_resident(dtb_plan_t p, void* data, const double* coeffs, int64_t T, hipStream_t st)
{
    if (dtb_status rc = poison_xbufs(p, st); rc != DTB_OK) return rc;
    ProbDesc P{};
    P.grid = data;
    P.xbuf[0] = p->xbuf[0];
    P.xbuf[1] = p->xbuf[1];
    P.pitch = p->pitch;
    P.T = T;
    P.rows = (int)p->rows;
    P.cols = (int)p->cols;
    P.k = p->layout.k;
    P.wg0 = 0;
    P.nwg = p->layout.nwg;
    P.dtype = p->dtype;
    P.fma = p->fma ? 1 : 0;
    P.narrow_cols = p->colmask ? 1 : 0;
    P.narrow_rows = p->rowcheck ? 1 : 0;
    P.debug = p->debug;
    P.timing = p->d_timing;
    P.direct_xchg = (p->debug & DTB_DEBUG_DIRECT_XCHG) ? 1 : 0;
    P.grid_sync = p->grid_sync ? 1 : 0;
    P.bar = p->d_bar;
    if (p->grid_sync && launch_reset_counter(p->d_bar, st) != hipSuccess) return DTB_ERR_HIP;
    for (int i = 0; i < p->pts; ++i) P.coeffs[i] = coeffs[i];
    const WgDesc* wgs = p->d_wgs;
    uint32_t* flags = p->d_flags;
    int* err = p->d_err;
    uint32_t spin = p->spin_limit();
    void* args[] = {&P, (void*)&wgs, (void*)&flags, (void*)&err, &spin};
    const dim3 grid(p->layout.nwg), block(p->layout.waves * kWaveSize);
    if (hipLaunchCooperativeKernel(p->kfunc, grid, block, args, 0, st) != hipSuccess) return DTB_ERR_HIP;
    return DTB_OK;
}

// Overlapped per-workgroup blocking: rounds of D steps, one launch each,
// between the grid and the workspace (whose halo ring is copied first); after
// an odd number of rounds the interior is copied back.
dtb_status run_overlapped_path(dtb_plan_t p, void* data, const double* coeffs, int64_t T, hipStream_t st)
{
    const int rows = (int)p->rows, cols = (int)p->cols;
    const int D = p->ovl_D;
    if (launch_copy_halo(p->dtype, data, p->ws, p->pitch, rows, cols, st) != hipSuccess) return DTB_ERR_HIP;
    ProbDesc P{};
    P.grid = data;
    P.pitch = p->pitch;
    P.T = T;
    P.rows = rows;
    P.cols = cols;
    P.k = D;
    P.nwg = p->layout.nwg;
    P.dtype = p->dtype;
    P.fma = p->fma ? 1 : 0;
    P.narrow_cols = p->colmask ? 1 : 0;
    P.narrow_rows = p->rowcheck ? 1 : 0;
    for (int i = 0; i < p->pts; ++i) P.coeffs[i] = coeffs[i];
    const WgDesc* wgs = p->d_wgs;
    void* bufs[2] = {data, p->ws};
    const dim3 grid(p->layout.nwg), block(p->layout.waves * kWaveSize);
    int64_t done = 0, round = 0;
    while (done < T) {
        int steps = (int)std::min<int64_t>(D, T - done);
        void* src = bufs[round & 1];
        void* dst = bufs[(round + 1) & 1];
        void* args[] = {&P, (void*)&wgs, &src, &dst, &steps};
        if (hipLaunchKernel(p->kfunc, grid, block, args, 0, st) != hipSuccess) return DTB_ERR_HIP;
        done += steps;
        ++round;
    }
    if (round & 1) {
        if (launch_copy_interior(p->dtype, p->ws, data, p->pitch, rows, cols, st) != hipSuccess) return DTB_ERR_HIP;
    }
    return DTB_OK;
}

dtb_status run_sweep(dtb_plan_t p, void* data, const double* coeffs, int64_t T, hipStream_t st)
{
    if (dtb_status rc = poison_xbufs(p, st); rc != DTB_OK) return rc;
    const int rows = (int)p->rows, cols = (int)p->cols;
    const SweepPlan& sp = p->sweep;
    // The second buffer needs the grid's halo: the kernel reads it from whichever buffer is current.
    if (launch_copy_halo(p->dtype, data, p->ws, p->pitch, rows, cols, st) != hipSuccess) return DTB_ERR_HIP;
    if (launch_reset_counter(p->d_bar, st) != hipSuccess) return DTB_ERR_HIP;
    ProbDesc P{};
    P.grid = data;
    P.xbuf[0] = p->xbuf[0];
    P.xbuf[1] = p->xbuf[1];
    P.pitch = p->pitch;
    P.T = T;
    P.rows = rows;
    P.cols = cols;
    P.k = sp.k;
    P.wg0 = 0;
    P.nwg = p->nwg_launch;
    P.dtype = p->dtype;
    P.fma = p->fma ? 1 : 0;
    P.narrow_cols = p->colmask ? 1 : 0;
    P.narrow_rows = p->rowcheck ? 1 : 0;
    P.debug = p->debug;
    P.timing = p->d_timing;
    P.direct_xchg = (p->debug & DTB_DEBUG_DIRECT_XCHG) ? 1 : 0;
    for (int i = 0; i < p->pts; ++i) P.coeffs[i] = coeffs[i];
    SweepArgs S{};
    S.bufs[0] = data;
    S.bufs[1] = p->ws;
    S.ntiles = (int)sp.tiles.size();
    S.nwg = p->nwg_launch;
    S.D = sp.D;
    const int64_t nrounds = (T + sp.D - 1) / sp.D;
    if (nrounds > (1 << 30)) return DTB_ERR_UNSUPPORTED;
    S.nrounds = (int)nrounds;
    S.bar = p->d_bar;
    const WgDesc* table = p->d_wgs;
    uint32_t* flags = p->d_flags;
    int* err = p->d_err;
    uint32_t spin = p->spin_limit();
    void* args[] = {&P, &S, (void*)&table, (void*)&flags, (void*)&err, &spin};
    const dim3 grid(p->nwg_launch), block(sp.waves * kWaveSize);
    if (hipLaunchCooperativeKernel(p->kfunc, grid, block, args, 0, st) != hipSuccess) return DTB_ERR_HIP;
    if (nrounds & 1) {
        if (launch_copy_interior(p->dtype, p->ws, data, p->pitch, rows, cols, st) != hipSuccess) return DTB_ERR_HIP;
    }
    return DTB_OK;
}

// A run on a stream other than the previous run's waits for the previous run
// (its workspace -- exchange buffers, flags, sweep buffer, descriptor table --
// is shared).  Inside a stream capture the wait is left out: an event recorded
// outside the capture cannot be waited on there, and runs captured on one
// stream are ordered by that stream.
dtb_status order_after_last_run(hipEvent_t done, bool has_run, hipStream_t last, hipStream_t st)
{
    if (!has_run || last == st) return DTB_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return DTB_ERR_HIP;
    if (cs != hipStreamCaptureStatusNone) return DTB_OK;
    return hipStreamWaitEvent(st, done, 0) == hipSuccess ? DTB_OK : DTB_ERR_HIP;
}

dtb_status run_plan_impl(dtb_plan_t p, const dtb_grid* g, const double* coeffs, int64_t T, void* stream)
{
    if (!p || !g || !coeffs || !g->data) return DTB_ERR_INVALID_ARG;
    if (T < 0) return DTB_ERR_INVALID_ARG;
    if (p->is3d || g->rows != p->rows || g->cols != p->cols || g->pitch != p->pitch) return DTB_ERR_MISMATCH;
    if (T == 0) return DTB_OK;
    hipStream_t st = (hipStream_t)stream;
    if (dtb_status rc = order_after_last_run(p->done, p->has_run, p->last_stream, st); rc != DTB_OK) return rc;
    dtb_status rc = DTB_ERR_UNSUPPORTED;
    if (p->path == DTB_PATH_STEP) rc = run_step(p, g->data, coeffs, T, st);
    else if (p->path == DTB_PATH_RESIDENT) rc = run_resident(p, g->data, coeffs, T, st);
    else if (p->path == DTB_PATH_SWEEP) rc = run_sweep(p, g->data, coeffs, T, st);
    else if (p->path == DTB_PATH_OVERLAPPED) rc = run_overlapped_path(p, g->data, coeffs, T, st);
    if (rc != DTB_OK) return rc;
    if (hipEventRecord(p->done, st) != hipSuccess) return DTB_ERR_HIP;
    p->last_stream = st;
    p->has_run = true;
    return DTB_OK;
}

// ---- dtb_run's plan cache
struct CacheKey {
    int64_t rows, cols, pitch;
    int dtype, device;
    bool operator<(const CacheKey& o) const
    {
        return std::tie(rows, cols, pitch, dtype, device) < std::tie(o.rows, o.cols, o.pitch, o.dtype, o.device);
    }
};
std::mutex g_cache_mu;
std::map<CacheKey, dtb_plan_t> g_cache;

// ---- dtb_run_batched: planned, allocated and turned into a one-node HIP graph
// on the first call for a set of shapes/precisions/step counts, replayed after.
struct BatchEntry {
    int device = -1;
    BatchPlan plan;
    TileInst insts[kMaxBatchInsts];
    int ninst = 0;
    std::vector<ProbDesc> probs;  // templates: everything but grid pointer and coefficients
    ProbDesc* d_probs = nullptr;
    JobDesc* d_jobs = nullptr;
    WgDesc* d_table = nullptr;
    int* d_wl_off = nullptr;
    WorkItem* d_wl = nullptr;
    uint32_t* d_flags = nullptr;
    int* d_err = nullptr;
    std::vector<void*> bufs;          // exchange buffers and sweep buffers
    ProbDesc* h_stage[2] = {nullptr, nullptr};  // pinned staging for the per-call descriptors
    hipEvent_t ev[2] = {nullptr, nullptr};
    int stage = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool cooperative = false;
    uint32_t spin = kSpinLimit;       // bounded waits of this batch (see batch_spin_limit)
    hipEvent_t done = nullptr;        // recorded after every replay
    hipStream_t last_stream = nullptr;
    bool has_run = false;

    ~BatchEntry()
    {
        if (done) (void)hipEventDestroy(done);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (int i = 0; i < 2; ++i) {
            if (ev[i]) (void)hipEventDestroy(ev[i]);
            if (h_stage[i]) (void)hipHostFree(h_stage[i]);
        }
        for (void* b : bufs) (void)hipFree(b);
        void* ds[] = {d_probs, d_jobs, d_table, d_wl_off, d_wl, d_flags, d_err};
        for (void* d : ds)
            if (d) (void)hipFree(d);
    }
};

std::mutex g_batch_mu;
std::map<std::vector<int64_t>, BatchEntry*> g_batch_cache;

dtb_status make_batch(const dtb_problem* problems, int32_t count, int device, BatchEntry** out)
{
    DeviceInfo di;
    if (!device_info(&di)) return DTB_ERR_HIP;
    std::unique_ptr<BatchEntry> b(new BatchEntry());
    b->device = device;
    const void* kfn = batched_kernel(b->insts, &b->ninst);
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kfn, 8 * kWaveSize, 0) != hipSuccess) return DTB_ERR_HIP;
    // One slot per compute unit; at most one per thread of a workgroup, since a swept job's members wait for
    // each other with one thread per member flag.
    const int nslots = std::min(std::min(occ, 1) * di.n_cu, 8 * kWaveSize);
    if (nslots < 1) return DTB_ERR_NOT_CORESIDENT;
    std::vector<BatchSpec> specs(count);
    for (int i = 0; i < count; ++i) {
        specs[i].rows = problems[i].grid.rows;
        specs[i].cols = problems[i].grid.cols;
        specs[i].pitch = problems[i].grid.pitch;
        specs[i].T = problems[i].T;
        specs[i].dtype = problems[i].dtype;
    }
    if (!plan_batch(specs, std::vector<TileInst>(b->insts, b->insts + b->ninst), 8, nslots, &b->plan))
        return DTB_ERR_UNSUPPORTED;
    const BatchPlan& bp = b->plan;

    // Per problem: two exchange buffers; per sweep job: the second grid buffer.
    b->probs.assign(count, ProbDesc{});
    std::vector<JobDesc> jobs(bp.jobs.size());
    for (size_t j = 0; j < bp.jobs.size(); ++j) {
        const BatchJob& J = bp.jobs[j];
        const dtb_problem& q = problems[J.prob];
        const size_t bytes = (size_t)(q.grid.rows + 2) * (size_t)q.grid.pitch * elem_size(q.dtype);
        ProbDesc& P = b->probs[J.prob];
        for (int i = 0; i < 2; ++i) {
            void* x = nullptr;
            if (hipMalloc(&x, bytes) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
            b->bufs.push_back(x);
            P.xbuf[i] = x;
        }
        P.pitch = q.grid.pitch;
        P.T = q.T;
        P.rows = (int)q.grid.rows;
        P.cols = (int)q.grid.cols;
        P.k = J.k;
        P.wg0 = J.flag_base;
        P.nwg = J.g;
        P.dtype = q.dtype;
        P.fma = 1;
        P.narrow_cols = J.narrow_cols ? 1 : 0;
        P.narrow_rows = J.narrow_rows ? 1 : 0;
        JobDesc& D = jobs[j];
        D.prob = J.prob;
        D.g = J.g;
        D.flag_base = J.flag_base;
        D.table_off = J.table_off;
        D.ntiles = J.ntiles;
        D.D = J.D;
        D.nrounds = J.nrounds;
        D.sweep = J.sweep ? 1 : 0;
        D.R = J.R;
        D.C = J.C;
        D.ws = nullptr;
        if (J.sweep) {
            if (hipMalloc(&D.ws, bytes) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
            b->bufs.push_back(D.ws);
        }
    }
    std::vector<WorkItem> wl(bp.wl_job.size());
    for (size_t i = 0; i < wl.size(); ++i) wl[i] = WorkItem{bp.wl_job[i], bp.wl_local[i]};
    auto up = [](void** dst, const void* src, size_t bytes) -> dtb_status {
        if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return DTB_ERR_HIP;
        return DTB_OK;
    };
    dtb_status st;
    if ((st = up((void**)&b->d_probs, b->probs.data(), count * sizeof(ProbDesc))) != DTB_OK) return st;
    if ((st = up((void**)&b->d_jobs, jobs.data(), jobs.size() * sizeof(JobDesc))) != DTB_OK) return st;
    if ((st = up((void**)&b->d_table, bp.table.data(), bp.table.size() * sizeof(WgDesc))) != DTB_OK) return st;
    if ((st = up((void**)&b->d_wl_off, bp.wl_off.data(), bp.wl_off.size() * sizeof(int))) != DTB_OK) return st;
    if ((st = up((void**)&b->d_wl, wl.data(), wl.size() * sizeof(WorkItem))) != DTB_OK) return st;
    if (hipMalloc(&b->d_flags, (size_t)std::max(bp.nflags, 1) * kFlagStride * sizeof(uint32_t)) != hipSuccess)
        return DTB_ERR_OUT_OF_MEMORY;
    if (hipMemset(b->d_flags, 0, (size_t)std::max(bp.nflags, 1) * kFlagStride * sizeof(uint32_t)) != hipSuccess)
        return DTB_ERR_HIP;
    if (hipMalloc(&b->d_err, sizeof(int)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
    if (hipMemset(b->d_err, 0, sizeof(int)) != hipSuccess) return DTB_ERR_HIP;
    for (int i = 0; i < 2; ++i) {
        if (hipHostMalloc((void**)&b->h_stage[i], count * sizeof(ProbDesc), hipHostMallocDefault) != hipSuccess)
            return DTB_ERR_OUT_OF_MEMORY;
        if (hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming) != hipSuccess) return DTB_ERR_HIP;
    }

    // One kernel node: the persistent batched kernel over every slot.
    if (hipGraphCreate(&b->graph, 0) != hipSuccess) return DTB_ERR_HIP;
    if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) return DTB_ERR_HIP;
    b->spin = batch_spin_limit(bp.makespan, kSpinLimit);
    void* args[] = {(void*)&b->d_probs, (void*)&b->d_jobs, (void*)&b->d_table, (void*)&b->d_wl_off,
                    (void*)&b->d_wl, (void*)&b->d_flags, (void*)&b->d_err, (void*)&b->spin};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(kfn);
    kp.gridDim = dim3(nslots);
    kp.blockDim = dim3(8 * kWaveSize);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    if (hipGraphAddKernelNode(&node, b->graph, nullptr, 0, &kp) != hipSuccess) return DTB_ERR_HIP;
    // Every wait in the batched kernel relies on all slots being resident at
    // once: without the cooperative attribute there is no such guarantee, so
    // refuse rather than replay an ordinary launch.
    hipKernelNodeAttrValue v{};
    v.cooperative = 1;
    if (hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &v) != hipSuccess) {
        (void)hipGetLastError();
        return DTB_ERR_UNSUPPORTED;
    }
    b->cooperative = true;
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return DTB_ERR_HIP;
    *out = b.release();
    return DTB_OK;
}

dtb_status run_batched_impl(const dtb_problem* problems, int32_t count, hipStream_t st)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DTB_ERR_HIP;
    std::vector<int64_t> key{dev, count};
    for (int32_t i = 0; i < count; ++i) {
        const dtb_problem& q = problems[i];
        key.insert(key.end(), {q.grid.rows, q.grid.cols, q.grid.pitch, q.dtype, q.T});
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchEntry* b = nullptr;
    auto it = g_batch_cache.find(key);
    if (it != g_batch_cache.end()) {
        b = it->second;
    } else {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess) return DTB_ERR_HIP;
        if (cs != hipStreamCaptureStatusNone) return DTB_ERR_NOT_PLANNED;
        dtb_status rc = make_batch(problems, count, dev, &b);
        if (rc != DTB_OK) return rc;
        g_batch_cache[key] = b;
    }
    // The descriptor table and the flags serve one replay at a time.
    if (dtb_status rc = order_after_last_run(b->done, b->has_run, b->last_stream, st); rc != DTB_OK) return rc;
    // This call's grid pointers and coefficients into the descriptor table.
    const int s = b->stage;
    b->stage ^= 1;
    if (hipEventSynchronize(b->ev[s]) != hipSuccess) return DTB_ERR_HIP;
    ProbDesc* h = b->h_stage[s];
    for (int32_t i = 0; i < count; ++i) {
        h[i] = b->probs[i];
        h[i].grid = problems[i].grid.data;
        for (int c = 0; c < 5; ++c) h[i].coeffs[c] = problems[i].coeffs[c];
    }
    if (hipMemcpyAsync(b->d_probs, h, count * sizeof(ProbDesc), hipMemcpyHostToDevice, st) != hipSuccess)
        return DTB_ERR_HIP;
    if (hipEventRecord(b->ev[s], st) != hipSuccess) return DTB_ERR_HIP;
    if (hipGraphLaunch(b->exec, st) != hipSuccess) return DTB_ERR_HIP;
    if (hipEventRecord(b->done, st) != hipSuccess) return DTB_ERR_HIP;
    b->last_stream = st;
    b->has_run = true;
    return DTB_OK;
}

// ---- j3d7pt: 2.5D streaming

dtb_status check_shape3(int64_t depth, int64_t rows, int64_t cols, int64_t pitch, int64_t plane_pitch, int dtype)
{
    if (depth < 1 || rows < 1 || cols < 1 || pitch < cols + 2 || plane_pitch < (rows + 2) * pitch)
        return DTB_ERR_INVALID_ARG;
    if (dtype != DTB_F64 && dtype != DTB_F32) return DTB_ERR_INVALID_ARG;
    if (depth > (1 << 30) || rows > (1 << 30) || cols > (1 << 30)) return DTB_ERR_UNSUPPORTED;
    return DTB_OK;
}

// Columns per lane of the streaming instance for a grid `cols` wide: the one whose overlapping column tiles
// (split_axis3) compute the fewest columns, the wider on a tie.  FP64 has one instance.
int stream3_cols_per_lane(int dtype, int64_t cols, int K)
{
    if (dtype != DTB_F32) return 2;
    int best = 4;
    int64_t best_cols = INT64_MAX;
    for (int c : {4, 3}) {
        std::vector<Span3> xs;
        if (!split_axis3(cols, kWaveSize * c, K, &xs)) continue;
        const int64_t computed = (int64_t)xs.size() * kWaveSize * c;
        if (computed < best_cols) {
            best_cols = computed;
            best = c;
        }
    }
    return best;
}

dtb_status plan3d_impl(dtb_plan_t* out, int64_t depth, int64_t rows, int64_t cols, int64_t pitch,
                       int64_t plane_pitch, int dtype, const dtb_plan_opts* opts)
{
    if (!out) return DTB_ERR_INVALID_ARG;
    *out = nullptr;
    dtb_status st = check_shape3(depth, rows, cols, pitch, plane_pitch, dtype);
    if (st != DTB_OK) return st;
    st = check_opts(opts);
    if (st != DTB_OK) return st;
    dtb_plan_opts o{};
    if (opts) o = *opts;
    if (o.stencil != 0 && o.stencil != 7) return DTB_ERR_INVALID_ARG;
    // The streaming path: K = 1 .. 3 steps per launch, 8 waves, neighbour-free (overlapped) tiles.
    if (o.path != DTB_PATH_AUTO && o.path != DTB_PATH_STEP && o.path != DTB_PATH_STREAM3D) return DTB_ERR_UNSUPPORTED;
    if (o.ghost_k > 3 || o.sync != 0 || o.tune != 0 || (o.waves != 0 && o.waves != 8) ||
        (o.debug_flags & ~DTB_DEBUG_TINY_SPIN) != 0)
        return DTB_ERR_UNSUPPORTED;
    const bool fma = o.exact == 0;
    const int path = o.path == DTB_PATH_STEP ? DTB_PATH_STEP : DTB_PATH_STREAM3D;
    int C = 0, R = 0;
    const int K = o.ghost_k > 0 ? o.ghost_k : 3;
    if (path == DTB_PATH_STREAM3D) {
        const int want = o.cols_per_lane > 0 ? o.cols_per_lane : stream3_cols_per_lane(dtype, cols, K);
        if (!dtb_stream3d_kernel(dtype, K, fma, want, &C, &R)) return DTB_ERR_UNSUPPORTED;
        if (o.rows_per_lane != 0 && o.rows_per_lane != R) return DTB_ERR_UNSUPPORTED;
    } else if (o.cols_per_lane != 0) {
        return DTB_ERR_UNSUPPORTED;
    }
    DeviceInfo di;
    if (!device_info(&di)) return DTB_ERR_HIP;
    std::unique_ptr<dtb_plan_s> p(new dtb_plan_s());
    p->device = di.device;
    p->is3d = true;
    p->depth = depth;
    p->rows = rows;
    p->cols = cols;
    p->pitch = pitch;
    p->plane_pitch = plane_pitch;
    p->dtype = dtype;
    p->pts = 7;
    p->fma = fma;
    p->path = path;
    p->debug = o.debug_flags;
    const size_t bytes = (size_t)(depth + 2) * (size_t)plane_pitch * elem_size(dtype);
    if (path == DTB_PATH_STREAM3D) {
        std::vector<Span3> ys, xs;
        const int ER = kStreamWaves * R, EC = kWaveSize * C;
        if (!split_axis3(rows, ER, K, &ys) || !split_axis3(cols, EC, K, &xs)) return DTB_ERR_UNSUPPORTED;
        std::vector<Tile3Desc> tiles;
        for (const Span3& y : ys)
            for (const Span3& x : xs) {
                Tile3Desc t{};
                t.ext_r0 = y.e0;
                t.ext_c0 = x.e0;
                t.own_r0 = y.own0;
                t.own_r1 = y.own1;
                t.own_c0 = x.own0;
                t.own_c1 = x.own1;
                t.edge = (y.e0 < 1 || y.e0 + ER - 1 > rows || x.e0 < 1 || x.e0 + EC - 1 > cols) ? 1 : 0;
                tiles.push_back(t);
            }
        const int ntiles = (int)tiles.size();
        int zb = 0;
        if (o.depth_D > 0) {
            zb = (int)std::min<int64_t>(o.depth_D, depth);
        } else {
            const int cap = o.max_wg > 0 ? std::min(o.max_wg, di.n_cu) : di.n_cu;
            zb = choose_zblock(ntiles, ER, EC, K, (int)elem_size(dtype), depth, depth * rows * cols, cap);
        }
        const int64_t nzb = (depth + zb - 1) / zb;
        if ((int64_t)ntiles * nzb > INT32_MAX / 2) return DTB_ERR_UNSUPPORTED;
        p->K3 = K;
        p->zb = zb;
        p->nzb = (int)nzb;
        p->ntiles3 = ntiles;
        p->ty3 = (int)ys.size();
        p->tx3 = (int)xs.size();
        p->R3 = R;
        p->C3 = C;
        if (hipMalloc(&p->d_tiles3, tiles.size() * sizeof(Tile3Desc)) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
        if (hipMemcpy(p->d_tiles3, tiles.data(), tiles.size() * sizeof(Tile3Desc), hipMemcpyHostToDevice) != hipSuccess)
            return DTB_ERR_HIP;
    }
    if (hipMalloc(&p->ws, bytes) != hipSuccess) return DTB_ERR_OUT_OF_MEMORY;
    if (hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) return DTB_ERR_HIP;
    *out = p.release();
    return DTB_OK;
}

dtb_status run3d_impl(dtb_plan_t p, const dtb_grid3d* g, const double* coeffs, int64_t T, void* stream)
{
    if (!p || !g || !coeffs || !g->data || T < 0) return DTB_ERR_INVALID_ARG;
    if (!p->is3d || g->depth != p->depth || g->rows != p->rows || g->cols != p->cols || g->pitch != p->pitch ||
        g->plane_pitch != p->plane_pitch)
        return DTB_ERR_MISMATCH;
    if (T == 0) return DTB_OK;
    hipStream_t st = (hipStream_t)stream;
    if (dtb_status rc = order_after_last_run(p->done, p->has_run, p->last_stream, st); rc != DTB_OK) return rc;
    const int depth = (int)p->depth, rows = (int)p->rows, cols = (int)p->cols;
    if (launch_copy_shell3d(p->dtype, g->data, p->ws, p->pitch, p->plane_pitch, depth, rows, cols, st) != hipSuccess)
        return DTB_ERR_HIP;
    void* bufs[2] = {g->data, p->ws};
    int64_t done = 0, rounds = 0;
    if (p->path == DTB_PATH_STEP) {
        for (; done < T; ++done, ++rounds)
            if (launch_step3d(p->dtype, p->fma, bufs[rounds & 1], bufs[(rounds + 1) & 1], p->pitch, p->plane_pitch,
                              depth, rows, cols, coeffs, st) != hipSuccess)
                return DTB_ERR_HIP;
    } else {
        Stream3Args A{};
        A.pitch = p->pitch;
        A.plane_pitch = p->plane_pitch;
        A.depth = depth;
        A.rows = rows;
        A.cols = cols;
        A.zb = p->zb;
        A.nzb = p->nzb;
        A.ntiles = p->ntiles3;
        for (int i = 0; i < 7; ++i) A.coeffs[i] = coeffs[i];
        const Tile3Desc* tiles = p->d_tiles3;
        const dim3 grid((unsigned)((int64_t)p->ntiles3 * p->nzb)), block(kStreamWaves * kWaveSize);
        for (; done < T; ++rounds) {
            // The last launch may take fewer steps: the K-step layout serves it (a deeper ring than needed).
            const int k = (int)std::min<int64_t>(p->K3, T - done);
            int C = 0, R = 0;
            const void* f = dtb_stream3d_kernel(p->dtype, k, p->fma, p->C3, &C, &R);
            if (!f) return DTB_ERR_UNSUPPORTED;
            A.src = bufs[rounds & 1];
            A.dst = bufs[(rounds + 1) & 1];
            void* args[] = {&A, (void*)&tiles};
            if (hipLaunchKernel(f, grid, block, args, 0, st) != hipSuccess) return DTB_ERR_HIP;
            done += k;
        }
    }
    if (rounds & 1) {
        if (launch_copy_interior3d(p->dtype, p->ws, g->data, p->pitch, p->plane_pitch, depth, rows, cols, st) !=
            hipSuccess)
            return DTB_ERR_HIP;
    }
    if (hipEventRecord(p->done, st) != hipSuccess) return DTB_ERR_HIP;
    p->last_stream = st;
    p->has_run = true;
    return DTB_OK;
}

}  // namespace

extern "C" {

dtb_status dtb_plan3d(dtb_plan_t* out, int64_t depth, int64_t rows, int64_t cols, int64_t pitch, int64_t plane_pitch,
                      dtb_dtype dtype, const dtb_plan_opts* opts)
{
    return plan3d_impl(out, depth, rows, cols, pitch, plane_pitch, (int)dtype, opts);
}

dtb_status dtb_run3d_plan(dtb_plan_t plan, const dtb_grid3d* grid, const double* coeffs, int64_t T, void* stream)
{
    return run3d_impl(plan, grid, coeffs, T, stream);
}

dtb_status dtb_plan(dtb_plan_t* out, int64_t rows, int64_t cols, int64_t pitch, dtb_dtype dtype, int64_t T_hint,
                    const dtb_plan_opts* opts)
{
    return plan_impl(out, rows, cols, pitch, (int)dtype, T_hint, opts);
}

dtb_status dtb_run_plan(dtb_plan_t plan, const dtb_grid* grid, const double* coeffs, int64_t T, void* stream)
{
    return run_plan_impl(plan, grid, coeffs, T, stream);
}

dtb_status dtb_run(const dtb_grid* grid, const double coeffs[5], int64_t T, dtb_dtype dtype, void* stream)
{
    if (!grid || !coeffs || !grid->data || T < 0) return DTB_ERR_INVALID_ARG;
    dtb_status st = check_shape(grid->rows, grid->cols, grid->pitch, (int)dtype);
    if (st != DTB_OK) return st;
    if (T == 0) return DTB_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DTB_ERR_HIP;
    const CacheKey key{grid->rows, grid->cols, grid->pitch, (int)dtype, dev};
    dtb_plan_t p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) p = it->second;
    }
    if (!p) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess) return DTB_ERR_HIP;
        if (cs != hipStreamCaptureStatusNone) return DTB_ERR_NOT_PLANNED;
        st = plan_impl(&p, grid->rows, grid->cols, grid->pitch, (int)dtype, T, nullptr);
        if (st != DTB_OK) return st;
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            delete p;
            p = it->second;
        } else {
            g_cache[key] = p;
        }
    }
    return run_plan_impl(p, grid, coeffs, T, stream);
}

dtb_status dtb_run_batched(const dtb_problem* problems, int32_t count, void* stream)
{
    if (count < 0 || (count > 0 && !problems)) return DTB_ERR_INVALID_ARG;
    for (int32_t i = 0; i < count; ++i) {
        const dtb_problem& q = problems[i];
        if (!q.grid.data || q.T < 0) return DTB_ERR_INVALID_ARG;
        dtb_status st = check_shape(q.grid.rows, q.grid.cols, q.grid.pitch, q.dtype);
        if (st != DTB_OK) return st;
    }
    if (count == 0) return DTB_OK;
    return run_batched_impl(problems, count, (hipStream_t)stream);
}

dtb_status dtb_batch_check(void* stream)
{
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return DTB_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    dtb_status rc = DTB_OK;
    for (auto& kv : g_batch_cache) {
        BatchEntry* b = kv.second;
        int e = 0;
        if (hipMemcpy(&e, b->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return DTB_ERR_HIP;
        if (e != 0) {
            rc = DTB_ERR_TIMEOUT;
            if (hipMemset(b->d_err, 0, sizeof(int)) != hipSuccess) return DTB_ERR_HIP;
            if (hipMemset(b->d_flags, 0, (size_t)b->plan.nflags * kFlagStride * sizeof(uint32_t)) != hipSuccess)
                return DTB_ERR_HIP;
        }
    }
    return rc;
}

dtb_status dtb_plan_check(dtb_plan_t p, void* stream)
{
    if (!p) return DTB_ERR_INVALID_ARG;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return DTB_ERR_HIP;
    if (!p->d_err) return DTB_OK;
    int e = 0;
    if (hipMemcpy(&e, p->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return DTB_ERR_HIP;
    if (e == 0) return DTB_OK;
    // A timed-out run leaves the epoch counters out of step: reset them.
    if (hipMemset(p->d_err, 0, sizeof(int)) != hipSuccess) return DTB_ERR_HIP;
    const size_t nflags = p->path == DTB_PATH_SWEEP ? (size_t)p->nwg_launch : p->layout.wgs.size();
    if (hipMemset(p->d_flags, 0, nflags * kFlagStride * sizeof(uint32_t)) != hipSuccess) return DTB_ERR_HIP;
    return DTB_ERR_TIMEOUT;
}

dtb_status dtb_plan_timing(dtb_plan_t p, uint64_t* out, int32_t n, void* stream)
{
    if (!p || n < 0 || (n > 0 && !out)) return DTB_ERR_INVALID_ARG;
    if (!p->d_timing) return DTB_ERR_NOT_PLANNED;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return DTB_ERR_HIP;
    const int nwg = std::max<int>(p->nwg_launch, p->layout.nwg);
    const size_t m = std::min<size_t>((size_t)n, (size_t)nwg * kTimingSlots);
    if (m && hipMemcpy(out, p->d_timing, m * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return DTB_ERR_HIP;
    if (hipMemset(p->d_timing, 0, (size_t)nwg * kTimingSlots * sizeof(uint64_t)) != hipSuccess) return DTB_ERR_HIP;
    return DTB_OK;
}

dtb_status dtb_plan_describe(dtb_plan_t p, int64_t* v, int32_t n)
{
    if (!p || (n > 0 && !v) || n < 0) return DTB_ERR_INVALID_ARG;
    if (p->is3d) {
        const bool sm = p->path == DTB_PATH_STREAM3D;
        const int64_t all[] = {p->path, sm ? (int64_t)p->ntiles3 * p->nzb : 0, p->K3, p->zb,
                               sm ? kStreamWaves * p->R3 : 0, sm ? kWaveSize * p->C3 : 0, p->ty3, p->tx3, p->R3, p->C3,
                               p->nzb, p->fma ? 0 : 1, sm ? kStreamWaves : 0, 0, p->pts};
        for (int32_t i = 0; i < n && i < (int32_t)(sizeof(all) / sizeof(all[0])); ++i) v[i] = all[i];
        return DTB_OK;
    }
    const Layout& L = p->layout;
    const bool sw = p->path == DTB_PATH_SWEEP, ov = p->path == DTB_PATH_OVERLAPPED;
    const int64_t all[] = {p->path, sw ? p->nwg_launch : L.nwg, ov ? 0 : L.k, sw ? p->sweep.D : (ov ? p->ovl_D : 0), L.ER, L.EC,
                           L.rows.parts, L.cols.parts, L.R, L.C, sw ? (int64_t)p->sweep.tiles.size() : 0,
                           p->fma ? 0 : 1, L.waves, p->grid_sync ? 1 : 0, p->pts};
    for (int32_t i = 0; i < n && i < (int32_t)(sizeof(all) / sizeof(all[0])); ++i) v[i] = all[i];
    return DTB_OK;
}

void dtb_plan_destroy(dtb_plan_t plan)
{
    if (!plan) return;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
            if (it->second == plan) {
                g_cache.erase(it);
                break;
            }
        }
    }
    delete plan;
}

void dtb_cache_clear(void)
{
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (auto& kv : g_cache) delete kv.second;
        g_cache.clear();
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (auto& kv : g_batch_cache) delete kv.second;
    g_batch_cache.clear();
}

const char* dtb_status_string(dtb_status s)
{
    switch (s) {
    case DTB_OK: return "DTB_OK";
    case DTB_ERR_INVALID_ARG: return "DTB_ERR_INVALID_ARG";
    case DTB_ERR_UNSUPPORTED: return "DTB_ERR_UNSUPPORTED";
    case DTB_ERR_NOT_CORESIDENT: return "DTB_ERR_NOT_CORESIDENT";
    case DTB_ERR_OUT_OF_MEMORY: return "DTB_ERR_OUT_OF_MEMORY";
    case DTB_ERR_HIP: return "DTB_ERR_HIP";
    case DTB_ERR_TIMEOUT: return "DTB_ERR_TIMEOUT";
    case DTB_ERR_NOT_PLANNED: return "DTB_ERR_NOT_PLANNED";
    case DTB_ERR_MISMATCH: return "DTB_ERR_MISMATCH";
    default: return "DTB_ERR_UNKNOWN";
    }
}

// ---- planner hooks for host-only tests (include/dtb_testing.h)

int32_t dtb_test_layout(int64_t rows, int64_t cols, int32_t rows_per_lane, int32_t cols_per_lane, int32_t waves,
                        int32_t k, int32_t n_xcd, int32_t* out, int32_t max_wg)
{
    Layout L;
    if (rows_per_lane < 1 || cols_per_lane < 1 || waves < 1 || k < 1 || max_wg < 0 || (max_wg > 0 && !out))
        return -1;
    if (!build_layout(rows, cols, interior(rows, cols), interior(rows, cols), rows_per_lane, cols_per_lane, waves, k,
                      n_xcd, 0, 0, &L))
        return -1;
    if (L.nwg > max_wg) return L.nwg;
    for (int i = 0; i < L.nwg; ++i) {
        const WgDesc& d = L.wgs[i];
        int32_t* o = out + (size_t)i * DTB_TEST_LAYOUT_STRIDE;
        o[0] = d.ext_r0;
        o[1] = d.ext_c0;
        o[2] = d.own_r0;
        o[3] = d.own_r1;
        o[4] = d.own_c0;
        o[5] = d.own_c1;
        o[6] = d.nnb;
        for (int j = 0; j < kMaxNeighbours; ++j) o[7 + j] = j < d.nnb ? d.nb[j] : -1;
        o[7 + kMaxNeighbours] = (L.rows.narrow ? 1 : 0) | (L.cols.narrow ? 2 : 0);
    }
    return L.nwg;
}

int32_t dtb_test_batch(int32_t count, const int64_t* rows, const int64_t* cols, const int32_t* dtype,
                       const int64_t* T, int32_t r64, int32_t r32, int32_t n_slots, int32_t* jobs,
                       int32_t* slot_lists, int32_t slot_lists_len, int64_t* info)
{
    if (count < 1 || !rows || !cols || !dtype || !T || r64 < 0 || r32 < 0 || n_slots < 1) return -1;
    std::vector<TileInst> insts;
    if (r64 == 0 && r32 == 0) {
        TileInst list[kMaxBatchInsts];
        int n = 0;
        (void)batched_kernel(list, &n);
        insts.assign(list, list + n);
    } else {
        if (r64 < 1 || r32 < 1) return -1;
        insts = {TileInst{0, r64, 2}, TileInst{1, r32, 4}};
    }
    std::vector<BatchSpec> specs(count);
    for (int i = 0; i < count; ++i) {
        if (rows[i] < 1 || cols[i] < 1 || T[i] < 0 || (dtype[i] != 0 && dtype[i] != 1)) return -1;
        specs[i].rows = rows[i];
        specs[i].cols = cols[i];
        specs[i].pitch = cols[i] + 2;
        specs[i].T = T[i];
        specs[i].dtype = dtype[i];
    }
    BatchPlan bp;
    if (!plan_batch(specs, insts, 8, n_slots, &bp)) return -1;
    if (info) {
        info[0] = (int64_t)bp.makespan;
        info[1] = batch_spin_limit(bp.makespan, kSpinLimit);
    }
    if (jobs) {
        for (size_t j = 0; j < bp.jobs.size(); ++j) {
            const BatchJob& J = bp.jobs[j];
            const int32_t v[DTB_TEST_BATCH_STRIDE] = {J.prob, J.g, J.sweep ? 1 : 0, J.ntiles, J.D, J.nrounds,
                                                      J.flag_base, J.table_off, (int32_t)J.start, (int32_t)J.dur,
                                                      J.k, J.R, J.C};
            for (int i = 0; i < DTB_TEST_BATCH_STRIDE; ++i) jobs[j * DTB_TEST_BATCH_STRIDE + i] = v[i];
        }
    }
    if (slot_lists) {
        const int64_t need = (int64_t)n_slots + 1 + 2 * (int64_t)bp.wl_job.size();
        if (need > slot_lists_len) return -1;
        for (int i = 0; i <= n_slots; ++i) slot_lists[i] = bp.wl_off[i];
        for (size_t i = 0; i < bp.wl_job.size(); ++i) {
            slot_lists[n_slots + 1 + 2 * i] = bp.wl_job[i];
            slot_lists[n_slots + 1 + 2 * i + 1] = bp.wl_local[i];
        }
    }
    return (int32_t)bp.jobs.size();
}

int32_t dtb_test_sweep(int64_t rows, int64_t cols, int32_t rows_per_lane, int32_t cols_per_lane, int32_t waves,
                       int32_t k, int32_t D, int32_t max_wg, int32_t n_xcd, int32_t* out, int32_t max_records)
{
    if (rows < 1 || cols < 1 || rows_per_lane < 1 || cols_per_lane < 1 || waves < 1 || k < 1 || D < 1 ||
        max_wg < 1 || max_records < 0 || (max_records > 0 && !out))
        return -1;
    SweepPlan sp;
    if (!plan_sweep(rows, cols, rows_per_lane, cols_per_lane, waves, k, D, max_wg, n_xcd, &sp)) return -1;
    const int nt = (int)sp.tiles.size();
    const int64_t nrec = (int64_t)nt * sp.nwg;
    if (nrec > max_records) return (int32_t)std::min<int64_t>(nrec, INT32_MAX);
    for (int t = 0; t < nt; ++t) {
        for (int b = 0; b < sp.nwg; ++b) {
            const WgDesc& d = sp.table[(size_t)t * sp.nwg + b];
            int32_t* o = out + ((size_t)t * sp.nwg + b) * DTB_TEST_SWEEP_STRIDE;
            const int32_t v[] = {t, sp.nwg, d.ext_r0, d.ext_c0, d.own_r0, d.own_r1, d.own_c0, d.own_c1,
                                 d.cr_r0, d.cr_r1, d.cr_c0, d.cr_c1, d.st_r0, d.st_r1, d.st_c0, d.st_c1, d.nnb};
            for (int i = 0; i < 17; ++i) o[i] = v[i];
            for (int j = 0; j < kMaxNeighbours; ++j) o[17 + j] = j < d.nnb ? d.nb[j] : -1;
        }
    }
    return (int32_t)nrec;
}

int32_t dtb_test_split3(int64_t n, int32_t E, int32_t K, int32_t* out, int32_t max_spans)
{
    if (max_spans < 0 || (max_spans > 0 && !out)) return -1;
    std::vector<Span3> spans;
    if (!split_axis3(n, E, K, &spans)) return -1;
    const int32_t ns = (int32_t)spans.size();
    if (ns > max_spans) return ns;
    for (int32_t i = 0; i < ns; ++i) {
        out[3 * i] = spans[i].e0;
        out[3 * i + 1] = spans[i].own0;
        out[3 * i + 2] = spans[i].own1;
    }
    return ns;
}

int32_t dtb_test_zblock(int64_t ntiles, int32_t ext_rows, int32_t ext_cols, int32_t K, int32_t elem_bytes,
                        int64_t depth, int64_t interior_cells, int32_t n_cu)
{
    if (ntiles < 1 || ext_rows < 1 || ext_cols < 1 || K < 1 || (elem_bytes != 4 && elem_bytes != 8) || depth < 1 ||
        interior_cells < 1 || n_cu < 1)
        return -1;
    return choose_zblock(ntiles, ext_rows, ext_cols, K, elem_bytes, depth, interior_cells, n_cu);
}

int32_t dtb_test_cols3(int32_t dtype, int64_t cols, int32_t K)
{
    if ((dtype != DTB_F64 && dtype != DTB_F32) || cols < 1 || K < 1 || K > 3) return -1;
    return stream3_cols_per_lane(dtype, cols, K);
}

}  // extern "C"
