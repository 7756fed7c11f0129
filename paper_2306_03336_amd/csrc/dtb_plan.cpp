// dtb_plan.cpp -- tile planner (host C++, no HIP calls).
#include "dtb_plan.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <functional>
#include <queue>

namespace dtb {

int64_t axis_capacity(int ext, int k, int parts)
{
    if (parts < 1) return 0;
    if (parts == 1) return ext;
    const int64_t inner = ext - 2 * k, edge = ext - k;
    if (edge < 1) return 0;
    if (parts > 2 && inner < 1) return 0;
    return 2 * edge + (int64_t)(parts - 2) * std::max<int64_t>(inner, 0);
}

bool split_axis_core(int64_t lo, int64_t hi, int64_t dom, int ext, int k, int parts, int* bounds, int* ext0,
                     bool* narrow)
{
    const int64_t len = hi - lo;
    if (len < 1 || lo < 1 || hi > dom + 1 || ext < 1 || k < 1 || parts < 1 || parts > len) return false;
    *narrow = dom < ext;
    if (*narrow) {
        // The whole interior fits in one extended tile placed at its start.
        if (parts != 1 || lo != 1 || hi != dom + 1) return false;
        bounds[0] = 1;
        bounds[1] = (int)dom + 1;
        ext0[0] = 1;
        return true;
    }
    // Capacities: an end tile of the range needs a ghost ring on one side only.
    auto cap = [&](int i) -> int64_t {
        const int sides = (parts == 1) ? 0 : ((i == 0 || i == parts - 1) ? 1 : 2);
        return ext - (int64_t)sides * k;
    };
    for (int i = 0; i < parts; ++i)
        if (cap(i) < 1) return false;
    // Even split, then hand the remainder to tiles with room, ends first
    // (order 0, parts - 1, 1, 2, ...).  The widths are kept in ext0 until the
    // bounds are known.
    int* w = ext0;
    const int64_t q = len / parts;
    int64_t left = len;
    for (int i = 0; i < parts; ++i) {
        w[i] = (int)std::min<int64_t>(q, cap(i));
        left -= w[i];
    }
    auto order = [&](int j) { return j == 0 ? 0 : (j == 1 ? parts - 1 : j - 1); };
    while (left > 0) {
        bool moved = false;
        for (int j = 0; j < parts && left > 0; ++j) {
            const int i = order(j);
            if (w[i] < cap(i)) {
                ++w[i];
                --left;
                moved = true;
            }
        }
        if (!moved) return false;
    }
    bounds[0] = (int)lo;
    for (int i = 0; i < parts; ++i) {
        if (w[i] < 1) return false;
        bounds[i + 1] = bounds[i] + w[i];
    }
    for (int i = 0; i < parts; ++i) {
        const int64_t o0 = bounds[i], o1 = bounds[i + 1];
        const int64_t f0 = std::max<int64_t>(o0 - k, lo), f1 = std::min<int64_t>(o1 + k, hi);
        const int64_t e0 = std::min<int64_t>(std::max<int64_t>(f0, 1), dom - ext + 1);
        if (f0 < e0 || f1 > e0 + ext) return false;
        ext0[i] = (int)e0;
    }
    return true;
}

bool split_axis(int64_t lo, int64_t hi, int64_t dom, int ext, int k, int parts, AxisSplit* out)
{
    if (parts < 1 || parts > hi - lo) return false;
    AxisSplit s;
    s.parts = parts;
    s.bounds.assign(parts + 1, 0);
    s.ext0.assign(parts, 1);
    if (!split_axis_core(lo, hi, dom, ext, k, parts, s.bounds.data(), s.ext0.data(), &s.narrow)) return false;
    *out = std::move(s);
    return true;
}

int first_parts_guess(int64_t len, int ext, int k)
{
    const int64_t inner = ext - 2 * k, edge = ext - k;
    if (edge < 1) return 0;
    if (len <= ext) return 1;
    if (len <= 2 * edge) return 2;
    if (inner < 1) return 0;
    return (int)std::min<int64_t>(2 + (len - 2 * edge + inner - 1) / inner, INT_MAX);
}

int min_parts(int64_t lo, int64_t hi, int64_t dom, int ext, int k, int max_parts)
{
    const int64_t len = hi - lo;
    if (len < 1) return 0;
    AxisSplit s;
    if (len <= ext && split_axis(lo, hi, dom, ext, k, 1, &s)) return 1;
    int64_t p = std::max(first_parts_guess(len, ext, k), 2);
    if (first_parts_guess(len, ext, k) == 0) return 0;
    for (; p <= max_parts && p <= len; ++p) {
        if (split_axis(lo, hi, dom, ext, k, (int)p, &s)) return (int)p;
    }
    return 0;
}

void xcd_slot_order(int pr, int pc, const Region& cr, int n_xcd, int wg_base, int* slot_of_tile, int* scratch)
{
    const int n = pr * pc;
    int gy = 1, gx = 1;
    if (n_xcd > 1) {
        double best = 1e300;
        for (int a = 1; a <= n_xcd; ++a) {
            if (n_xcd % a) continue;
            const int b = n_xcd / a;
            if (a > pr || b > pc) continue;
            const double h = (double)(cr.r1 - cr.r0) / a, w = (double)(cr.c1 - cr.c0) / b;
            const double score = std::max(h / w, w / h);
            if (score < best) {
                best = score;
                gy = a;
                gx = b;
            }
        }
    }
    // scratch: the tiles (id tr * pc + tc) in XCD-block order.
    int m = 0;
    for (int by = 0; by < gy; ++by) {
        const int r0 = (int)((int64_t)pr * by / gy), r1 = (int)((int64_t)pr * (by + 1) / gy);
        for (int bx = 0; bx < gx; ++bx) {
            const int c0 = (int)((int64_t)pc * bx / gx), c1 = (int)((int64_t)pc * (bx + 1) / gx);
            for (int tr = r0; tr < r1; ++tr)
                for (int tc = c0; tc < c1; ++tc) scratch[m++] = tr * pc + tc;
        }
    }
    // Launch slots XCD by XCD (slot order kept within an XCD), matched to the tiles in that order.
    const int nx = std::max(n_xcd, 1);
    int i = 0;
    for (int x = 0; x < nx; ++x)
        for (int b = 0; b < n; ++b)
            if ((wg_base + b) % nx == x) slot_of_tile[scratch[i++]] = b;
}

bool build_layout(int64_t rows, int64_t cols, const Region& cr, const Region& st, int R, int C, int waves, int k,
                  int n_xcd, int wg_base, int prob, Layout* out, bool neighbours, int max_tiles)
{
    Layout L;
    L.R = R;
    L.C = C;
    L.waves = waves;
    L.ER = waves * R;
    L.EC = kWaveSize * C;
    L.k = k;
    const int pr = min_parts(cr.r0, cr.r1, rows, L.ER, k, 1 << 20);
    const int pc = min_parts(cr.c0, cr.c1, cols, L.EC, k, 1 << 20);
    if (pr < 1 || pc < 1) return false;
    if ((int64_t)pr * pc > max_tiles) return false;
    if (!split_axis(cr.r0, cr.r1, rows, L.ER, k, pr, &L.rows) ||
        !split_axis(cr.c0, cr.c1, cols, L.EC, k, pc, &L.cols))
        return false;
    const int n = pr * pc;
    L.nwg = n;

    std::vector<int> slot_of_tile(n), scratch(n);
    xcd_slot_order(pr, pc, cr, n_xcd, wg_base, slot_of_tile.data(), scratch.data());

    L.wgs.assign(n, WgDesc{});
    for (int tr = 0; tr < pr; ++tr) {
        for (int tc = 0; tc < pc; ++tc) {
            WgDesc& d = L.wgs[slot_of_tile[tr * pc + tc]];
            d.prob = prob;
            d.ext_r0 = L.rows.ext0[tr];
            d.ext_c0 = L.cols.ext0[tc];
            d.own_r0 = L.rows.bounds[tr];
            d.own_r1 = L.rows.bounds[tr + 1];
            d.own_c0 = L.cols.bounds[tc];
            d.own_c1 = L.cols.bounds[tc + 1];
            d.cr_r0 = cr.r0;
            d.cr_r1 = cr.r1;
            d.cr_c0 = cr.c0;
            d.cr_c1 = cr.c1;
            d.st_r0 = st.r0;
            d.st_r1 = st.r1;
            d.st_c0 = st.c0;
            d.st_c1 = st.c1;
            d.nnb = 0;
        }
    }
    // Neighbours: the tiles whose owned cells lie within k of a tile's owned
    // cells.  Owned ranges along an axis are consecutive, so they sit in a
    // contiguous run of tile rows and of tile columns around the tile's own;
    // listed in launch-slot order.
    if (neighbours) {
        std::vector<int> nbs;
        for (int tr = 0; tr < pr; ++tr) {
            int r_lo = tr, r_hi = tr;
            while (r_lo > 0 && L.rows.bounds[r_lo] > L.rows.bounds[tr] - k) --r_lo;        // bounds[r_lo] is tile r_lo's end
            while (r_hi + 1 < pr && L.rows.bounds[r_hi + 1] < L.rows.bounds[tr + 1] + k) ++r_hi;
            for (int tc = 0; tc < pc; ++tc) {
                int c_lo = tc, c_hi = tc;
                while (c_lo > 0 && L.cols.bounds[c_lo] > L.cols.bounds[tc] - k) --c_lo;
                while (c_hi + 1 < pc && L.cols.bounds[c_hi + 1] < L.cols.bounds[tc + 1] + k) ++c_hi;
                WgDesc& d = L.wgs[slot_of_tile[tr * pc + tc]];
                nbs.clear();
                for (int ur = r_lo; ur <= r_hi; ++ur)
                    for (int uc = c_lo; uc <= c_hi; ++uc)
                        if (ur != tr || uc != tc) nbs.push_back(wg_base + slot_of_tile[ur * pc + uc]);
                if ((int)nbs.size() > kMaxNeighbours) return false;
                std::sort(nbs.begin(), nbs.end());
                d.nnb = (int)nbs.size();
                for (int i = 0; i < d.nnb; ++i) d.nb[i] = nbs[i];
            }
        }
    }
    *out = std::move(L);
    return true;
}

// Fitted to per-workgroup phase clocks at 2048^2 (FP64) and 1536^2 / 3072^2
// (FP32): a step costs about 52 ps per FP64 cell with 4 columns per lane, 56 ps
// with 2 (two cross-lane moves per cell instead of one), and 39 ps per FP32
// cell (VALU-bound: wave64 FP64 and FP32 instructions at 16 and 32 lanes per
// clock per SIMD) plus the per-step barrier; an exchange costs a few
// microseconds of fixed latency (store completion, flag round trip, load
// latency) plus a part that grows with the number of border cells moved
// lane by lane.
double tile_step_time_us(int ER, int EC, int elem_bytes, int pts)
{
    double per_cell = elem_bytes == 8 ? (EC <= 2 * kWaveSize ? 56e-6 : 52e-6) : 39e-6;
    // The box: nine products instead of five and six lane shifts per row instead of two.
    if (pts == 9) per_cell *= 1.8;
    return (double)ER * EC * per_cell + 0.11;
}

double exchange_time_us(int ER, int EC, int R, int C, int elem_bytes, bool staged)
{
    (void)elem_bytes;
    if (staged) return 3.3 + 0.25e-3 * ER * EC * (elem_bytes == 8 ? 1.0 : 0.5);
    return 4.0 + 0.15 * R * C;
}

double layout_cost(const Layout& L, int slots_per_cu, int n_cu, int elem_bytes, int pts)
{
    return layout_cost_of(L.nwg, L.R, L.C, L.ER, L.EC, L.k, slots_per_cu, n_cu, elem_bytes, pts);
}

double layout_cost_of(int nwg, int R, int C, int ER, int EC, int k, int slots_per_cu, int n_cu, int elem_bytes,
                      int pts)
{
    const int slots = std::max(1, slots_per_cu) * std::max(1, n_cu);
    if (nwg > slots) return 1e300;
    const int per_cu = (nwg + n_cu - 1) / n_cu;
    const bool staged = exchange_staged(R, C, elem_bytes, k);
    const double step = tile_step_time_us(ER, EC, elem_bytes, pts);
    const double exch = exchange_time_us(ER, EC, R, C, elem_bytes, staged) / k;
    if (per_cu <= 1) return step + exch;
    // Several workgroups per compute unit: measured (2048^2 FP64, two
    // half-height workgroups per unit), their exchanges hardly overlap the
    // other workgroup's steps and each takes about 1.5x longer than alone.
    return per_cu * step + 1.5 * exch;
}

static int min_parts_fixed(int64_t lo, int64_t hi, int64_t dom, int ext, int k, int* bounds, int* ext0, bool* narrow)
{
    const int64_t len = hi - lo;
    if (len < 1) return 0;
    if (len <= ext && split_axis_core(lo, hi, dom, ext, k, 1, bounds, ext0, narrow)) return 1;
    const int guess = first_parts_guess(len, ext, k);
    if (guess == 0) return 0;
    for (int64_t p = std::max(guess, 2); p <= kFixedMaxParts && p <= len; ++p)
        if (split_axis_core(lo, hi, dom, ext, k, (int)p, bounds, ext0, narrow)) return (int)p;
    return 0;
}

bool build_fixed_layout(int64_t rows, int64_t cols, int R, int C, int waves, int k, int n_xcd, FixedLayout* out)
{
    FixedLayout& L = *out;
    L.R = R;
    L.C = C;
    L.waves = waves;
    L.ER = waves * R;
    L.EC = kWaveSize * C;
    L.k = k;
    if (k < 1 || rows < 1 || cols < 1) return false;
    L.pr = min_parts_fixed(1, rows + 1, rows, L.ER, k, L.rb, L.re0, &L.narrow_rows);
    L.pc = min_parts_fixed(1, cols + 1, cols, L.EC, k, L.cb, L.ce0, &L.narrow_cols);
    if (L.pr < 1 || L.pc < 1 || L.pr * L.pc > kFixedMaxWg) return false;
    L.nwg = L.pr * L.pc;
    int scratch[kFixedMaxWg];
    xcd_slot_order(L.pr, L.pc, interior(rows, cols), n_xcd, 0, L.slot_of_tile, scratch);
    // Neighbours (tiles whose owned cells lie within k of a tile's) must fit a descriptor.
    for (int a = 0; a < L.nwg; ++a) {
        const int ar = a / L.pc, ac = a % L.pc;
        int nnb = 0;
        for (int b = 0; b < L.nwg; ++b) {
            if (b == a) continue;
            const int br = b / L.pc, bc = b % L.pc;
            const bool meet = L.rb[br] < L.rb[ar + 1] + k && L.rb[br + 1] > L.rb[ar] - k &&
                              L.cb[bc] < L.cb[ac + 1] + k && L.cb[bc + 1] > L.cb[ac] - k;
            if (meet) ++nnb;
        }
        if (nnb > kMaxNeighbours) return false;
    }
    return true;
}

// Even split of [1, len + 1) into n ranges.
static std::vector<int> even_bounds(int64_t len, int n)
{
    std::vector<int> b(n + 1);
    for (int i = 0; i <= n; ++i) b[i] = 1 + (int)(len * i / n);
    return b;
}

bool plan_sweep(int64_t rows, int64_t cols, int R, int C, int waves, int k, int D, int max_wg, int n_xcd,
                SweepPlan* out)
{
    if (D < 1 || k < 1 || max_wg < 1) return false;
    const int ER = waves * R, EC = kWaveSize * C;
    // Pick the workgroup grid pr x pc (pr * pc <= max_wg) whose big tiles
    // (capacity minus a D ring on each side) need the fewest tiles.
    int best_nt = 0;
    double best_score = 1e300;
    std::vector<int> best_vr, best_vc;
    for (int pr = 1; pr <= max_wg; ++pr) {
        const int pc = max_wg / pr;
        if (pc < 1) break;
        const int64_t cap_r = axis_capacity(ER, k, pr), cap_c = axis_capacity(EC, k, pc);
        // An interior big tile has a D ring on both sides.
        const int64_t lr = std::min<int64_t>(cap_r - 2 * (int64_t)D, rows);
        const int64_t lc = std::min<int64_t>(cap_c - 2 * (int64_t)D, cols);
        if (lr < 1 || lc < 1) continue;
        const int nr = (int)((rows + lr - 1) / lr), nc = (int)((cols + lc - 1) / lc);
        const double nt = (double)nr * nc;
        // Tiles processed one after another: time ~ number of tiles; break
        // ties toward less redundant ring.
        const double vr = (double)rows / nr, vc = (double)cols / nc;
        const double redundancy = (vr + 2.0 * D) * (vc + 2.0 * D) / (vr * vc);
        const double score = nt * 1000.0 + redundancy;
        if (score < best_score) {
            best_score = score;
            best_nt = (int)nt;
            best_vr = even_bounds(rows, nr);
            best_vc = even_bounds(cols, nc);
        }
    }
    if (best_nt < 1) return false;
    SweepPlan P;
    P.R = R;
    P.C = C;
    P.waves = waves;
    P.ER = ER;
    P.EC = EC;
    P.k = k;
    P.D = D;
    P.vr = best_vr;
    P.vc = best_vc;
    P.tiles_r = (int)best_vr.size() - 1;
    P.tiles_c = (int)best_vc.size() - 1;
    P.nwg = 0;
    for (int i = 0; i < P.tiles_r; ++i) {
        for (int j = 0; j < P.tiles_c; ++j) {
            Region st{P.vr[i], P.vr[i + 1], P.vc[j], P.vc[j + 1]};
            Region cr{std::max(st.r0 - D, 1), std::min<int>(st.r1 + D, (int)rows + 1), std::max(st.c0 - D, 1),
                      std::min<int>(st.c1 + D, (int)cols + 1)};
            Layout L;
            if (!build_layout(rows, cols, cr, st, R, C, waves, k, n_xcd, 0, 0, &L, true, max_wg)) return false;
            if (L.nwg > max_wg) return false;
            P.nwg = std::max(P.nwg, L.nwg);
            P.tiles.push_back(std::move(L));
        }
    }
    // Launch table: every big tile gets P.nwg descriptors; missing ones are idle.
    const int nt = (int)P.tiles.size();
    P.table.assign((size_t)nt * P.nwg, WgDesc{});
    for (int t = 0; t < nt; ++t) {
        const Layout& L = P.tiles[t];
        for (int b = 0; b < P.nwg; ++b) {
            WgDesc& d = P.table[(size_t)t * P.nwg + b];
            if (b < L.nwg) {
                d = L.wgs[b];
            } else {
                d = WgDesc{};
                d.ext_r0 = 1;
                d.ext_c0 = 1;
                d.own_r0 = d.own_r1 = 1;
                d.own_c0 = d.own_c1 = 1;
                d.nnb = 0;
            }
        }
    }
    // Cost per time step: every big tile runs on the whole chip one after another.
    const double ring = 1.0;  // placeholder weight for per-tile fixed costs
    P.est_cost = nt * ((double)ER * EC * (1.0 + 1.0 / k) + ring * ER * EC * 8.0 / D);
    *out = std::move(P);
    return true;
}

double tile_step_us(int ER, int EC, int elem_bytes, int active_rows)
{
    const int rows = std::min(ER, std::max(active_rows, 1));
    return tile_step_time_us(rows, EC, elem_bytes);
}

bool plan_batch(const std::vector<BatchSpec>& probs, const std::vector<TileInst>& insts, int waves, int nslots,
                BatchPlan* out)
{
    if (nslots < 1 || waves < 1) return false;
    BatchPlan bp;
    bp.nslots = nslots;
    const double t_bar = 5.0;  // device-wide barrier between sweep rounds
    // Every candidate of every problem: the job (without flags and table
    // offset) and its descriptor table (neighbours numbered from 0).
    struct Cand {
        BatchJob J;
        std::vector<WgDesc> tab;
    };
    std::vector<std::vector<Cand>> cands(probs.size());
    for (int p = 0; p < (int)probs.size(); ++p) {
        const BatchSpec& q = probs[p];
        const int eb = q.dtype == 0 ? 8 : 4;
        for (int ii = 0; ii < (int)insts.size(); ++ii) {
            const TileInst& ti = insts[ii];
            if (ti.dtype != q.dtype) continue;
            const int R = ti.R, C = ti.C, ER = waves * R, EC = kWaveSize * C;
            BatchJob base;
            base.prob = p;
            base.inst = ii;
            base.R = R;
            base.C = C;
            base.narrow_cols = q.cols < EC;
            base.narrow_rows = q.rows < ER;
            bool resident = false;
            for (int k = 1; k <= 16; ++k) {
                Layout L;
                if (!build_layout(q.rows, q.cols, interior(q.rows, q.cols), interior(q.rows, q.cols), R, C, waves, k, 1,
                                  0, p, &L, true, nslots))
                    continue;
                resident = true;
                Cand c{base, std::move(L.wgs)};
                c.J.sweep = false;
                c.J.g = L.nwg;
                c.J.k = k;
                c.J.D = (int)std::min<int64_t>(q.T, INT32_MAX);
                const int act = (int)std::min<int64_t>(q.rows, ER);
                const double t_exch = exchange_time_us(ER, EC, R, C, eb, exchange_staged(R, C, eb, k));
                const int64_t nexch = q.T > k ? (q.T + k - 1) / k - 1 : 1;
                c.J.dur = q.T * tile_step_us(ER, EC, eb, act) + (double)nexch * t_exch;
                cands[p].push_back(std::move(c));
            }
            if (resident) continue;
            for (int k : {4, 6, 8, 10, 12}) {
                for (int D : {16, 24, 32, 48, 64, 96, 128}) {
                    SweepPlan sp;
                    if (!plan_sweep(q.rows, q.cols, R, C, waves, k, D, nslots, 1, &sp)) continue;
                    const int64_t nrounds = (q.T + D - 1) / D;
                    if (nrounds > INT32_MAX) continue;
                    const double t_exch = exchange_time_us(ER, EC, R, C, eb, exchange_staged(R, C, eb, k));
                    const double per_tile = D * tile_step_us(ER, EC, eb, ER) + (double)D / k * t_exch + t_bar;
                    Cand c{base, std::move(sp.table)};
                    c.J.sweep = true;
                    c.J.g = sp.nwg;
                    c.J.k = k;
                    c.J.D = D;
                    c.J.ntiles = (int)sp.tiles.size();
                    c.J.nrounds = (int)nrounds;
                    c.J.dur = nrounds * per_tile * sp.tiles.size();
                    for (WgDesc& d : c.tab) d.prob = p;
                    cands[p].push_back(std::move(c));
                }
            }
        }
        if (cands[p].empty()) return false;
    }
    // The makespan cannot be shorter than the least total slot time spread
    // over every slot, nor than any job's least duration.
    double area = 0, longest = 0;
    for (const auto& cs : cands) {
        double a = 1e300, d = 1e300;
        for (const Cand& c : cs) {
            a = std::min(a, c.J.g * c.J.dur);
            d = std::min(d, c.J.dur);
        }
        area += a;
        longest = std::max(longest, d);
    }
    const double bound = std::max(area / nslots, longest);
    std::vector<BatchJob> jobs;
    std::vector<std::vector<WgDesc>> tables;
    int flag_base = 0;
    for (int p = 0; p < (int)probs.size(); ++p) {
        int best = -1;
        for (int i = 0; i < (int)cands[p].size(); ++i) {
            const BatchJob& J = cands[p][i].J;
            if (J.dur > bound * (1 + 1e-9)) continue;
            if (best < 0 || J.g * J.dur < cands[p][best].J.g * cands[p][best].J.dur) best = i;
        }
        if (best < 0)
            for (int i = 0; i < (int)cands[p].size(); ++i)
                if (best < 0 || cands[p][i].J.dur < cands[p][best].J.dur) best = i;
        Cand& c = cands[p][best];
        for (WgDesc& d : c.tab)
            for (int i = 0; i < d.nnb; ++i) d.nb[i] += flag_base;
        c.J.flag_base = flag_base;
        flag_base += c.J.g;
        jobs.push_back(std::move(c.J));
        tables.push_back(std::move(c.tab));
    }
    bp.nflags = flag_base;

    // Longest first onto the slots that free up earliest.
    std::vector<int> order(jobs.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return jobs[a].dur > jobs[b].dur; });
    std::vector<double> free_at(nslots, 0.0);
    for (int j : order) {
        BatchJob& J = jobs[j];
        std::vector<int> idx(nslots);
        for (int s = 0; s < nslots; ++s) idx[s] = s;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return free_at[a] < free_at[b]; });
        J.slots.assign(idx.begin(), idx.begin() + J.g);
        std::sort(J.slots.begin(), J.slots.end());
        double start = 0;
        for (int s : J.slots) start = std::max(start, free_at[s]);
        J.start = start;
        for (int s : J.slots) free_at[s] = start + J.dur;
        bp.makespan = std::max(bp.makespan, start + J.dur);
    }
    // Global order: by start time, ties by problem index.
    std::vector<int> glob(jobs.size());
    for (size_t i = 0; i < glob.size(); ++i) glob[i] = (int)i;
    std::stable_sort(glob.begin(), glob.end(), [&](int a, int b) {
        return jobs[a].start < jobs[b].start || (jobs[a].start == jobs[b].start && a < b);
    });
    for (int j : glob) {
        BatchJob J = jobs[j];
        J.table_off = (int)bp.table.size();
        bp.table.insert(bp.table.end(), tables[j].begin(), tables[j].end());
        bp.jobs.push_back(std::move(J));
    }
    // Work lists.
    std::vector<std::vector<std::pair<int, int>>> lists(nslots);
    for (int jj = 0; jj < (int)bp.jobs.size(); ++jj) {
        const BatchJob& J = bp.jobs[jj];
        for (int i = 0; i < J.g; ++i) lists[J.slots[i]].push_back({jj, i});
    }
    bp.wl_off.assign(nslots + 1, 0);
    for (int s = 0; s < nslots; ++s) {
        bp.wl_off[s + 1] = bp.wl_off[s] + (int)lists[s].size();
        for (auto& it : lists[s]) {
            bp.wl_job.push_back(it.first);
            bp.wl_local.push_back(it.second);
        }
    }
    *out = std::move(bp);
    return true;
}

// ---- 3-D streaming

bool split_axis3(int64_t n, int E, int K, std::vector<Span3>* out)
{
    out->clear();
    if (n < 1 || E < 2 * K + 1 || n > INT32_MAX / 2) return false;
    int64_t own0 = 1, e0 = 0;
    while (true) {
        if (e0 + E >= n + 2) {
            // The last range reaches the far halo (row n + 1): it owns everything up to it.  Moved back so
            // that it ends at the halo (a deeper near ring, never a shallower one), not before storage row 0.
            Span3 sp;
            sp.e0 = (int)std::max<int64_t>(0, n + 2 - E);
            sp.own0 = (int)own0;
            sp.own1 = (int)(n + 1);
            out->push_back(sp);
            return true;
        }
        Span3 sp;
        sp.e0 = (int)e0;
        sp.own0 = (int)own0;
        sp.own1 = (int)(e0 + E - K);
        out->push_back(sp);
        own0 = sp.own1;
        e0 = own0 - K;
    }
}

// Makespan, in plane iterations, of a streaming launch: its workgroups, dispatched in launch order (z-block by
// z-block, the tiles of a block in turn) onto n_cu compute units, one at a time on each, each taking one
// iteration per plane it streams (its z-block and the K-plane rings, clipped to the grid).  Past 32 waves of
// workgroups the order hardly matters and the even share is taken instead.
static double stream3_makespan(int64_t depth, int zb, int K, int64_t ntiles, int n_cu)
{
    const int64_t nz = (depth + zb - 1) / zb;
    auto iters = [&](int64_t b) {
        const int64_t z0 = 1 + b * zb, z1 = std::min<int64_t>(z0 + zb, depth + 1);
        return (double)(std::min<int64_t>(z1 + K, depth + 2) - std::max<int64_t>(z0 - K, 0));
    };
    if (ntiles * nz > 32 * (int64_t)n_cu) {
        double total = 0, longest = 0;
        for (int64_t b = 0; b < nz; ++b) {
            total += iters(b) * (double)ntiles;
            longest = std::max(longest, iters(b));
        }
        return total / n_cu + longest;
    }
    std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;  // per compute unit
    for (int i = 0; i < n_cu; ++i) free_at.push(0.0);
    double end = 0;
    for (int64_t b = 0; b < nz; ++b) {
        const double it = iters(b);
        for (int64_t t = 0; t < ntiles; ++t) {
            const double f = free_at.top() + it;
            free_at.pop();
            free_at.push(f);
            end = std::max(end, f);
        }
    }
    return end;
}

double stream3_launch_us(int nwg, int n_cu, int ER, int EC, int zb, int K, int elem_bytes, int64_t depth,
                         int64_t interior_cells, bool* bytes_bound)
{
    // Measured on MI355X (512^3, one workgroup per compute unit): a launch streams at about 4.3 TB/s (of the
    // bytes below) when every compute unit holds a workgroup, and each compute unit pulls its share, so
    // fewer workgroups than compute units leave bandwidth unused.  Bytes: every z-block loads its tile for
    // its planes and a K-deep ring below and above; the owned cells are stored once.  Compute: a workgroup
    // takes about 130 ps per cell and level for every plane it streams (its rings included), whatever the
    // precision (the FP64 and FP32 VALU rates are the same and the FP32 tile is twice as wide), one
    // workgroup per compute unit at a time, so the launch takes the makespan of its workgroups in launch
    // order (stream3_makespan).  That order decides the tail: the measured 512^3 launches rank as the
    // makespan does (FP32 with 4 columns per lane: one wave of 240 workgroups of 134 planes 905 GCells/s,
    // two of 70 planes 893, two of 108 756; with 3 columns per lane the same order, 1180, 1180 and 951-988;
    // FP64 with 11 z-blocks of 51 planes, the last one 2 planes short, 729 against 681 with 12 of 46).
    // FP64 (half the cells per plane) is bound by the bytes, FP32 by the compute.
    const double bw = 4.3e6;  // bytes per microsecond
    const int64_t nz = (depth + zb - 1) / zb;
    const int64_t tiles = nz > 0 ? nwg / nz : nwg;
    double planes = 0;
    for (int64_t b = 0; b < nz; ++b) {
        const int64_t z0 = 1 + b * zb, z1 = std::min<int64_t>(z0 + zb, depth + 1);
        planes += (double)(std::min<int64_t>(z1 + K, depth + 2) - std::max<int64_t>(z0 - K, 0));
    }
    const double bytes = planes * tiles * ER * EC * elem_bytes + (double)interior_cells * elem_bytes;
    const double w = (double)nwg / std::max(1, n_cu);
    const double mem = bytes / bw / std::min(w, 1.0);
    const double cell = 130e-6;  // microseconds per cell and level
    const double compute = stream3_makespan(depth, zb, K, tiles, n_cu) * ((double)ER * EC * cell * K + 0.3);
    if (bytes_bound) *bytes_bound = mem >= compute;
    return std::max(mem, compute);
}

int choose_zblock(int64_t ntiles, int ER, int EC, int K, int elem_bytes, int64_t depth, int64_t interior_cells,
                  int n_cu)
{
    // The block height with the least modelled launch time: taller blocks amortise the K-deep z ring, more
    // blocks fill the compute units.  Measured at 512^3: a launch bound by its memory traffic (FP64) streams
    // best with several waves of workgroups queued per compute unit (41-51 planes per block, 1100-1300
    // workgroups, beat 64-128 planes by 1.1x), so for such launches blocks that leave fewer than four
    // workgroups per compute unit are taken only when the grid is too shallow for more (among those, 51
    // planes per block, 729 GCells/s, beat 46, 681: stream3_launch_us); a compute-bound one (FP32) is best
    // with the fewest ring planes in whole waves of workgroups (128 planes per block, one wave, 905
    // GCells/s; 64, two waves, 893; 18, seven, 801; with 3 columns per lane 128 and 64 both 1180).  FP64
    // blocks of 103 planes (two waves of 500 workgroups) measured 1-3 % above 51 on three boxes; the
    // bytes model does not see the difference, and the rule above keeps 51.
    double best = 1e300;
    int zb = 1;
    const int64_t want = 4 * (int64_t)n_cu;
    const bool deep_enough = ntiles * ((depth + 4 * K - 1) / (4 * K)) >= want;
    for (int z = 1; z <= depth; z = z < 16 ? z + 1 : z + z / 8) {
        const int64_t nz = (depth + z - 1) / z;
        const int64_t nwg = ntiles * nz;
        if (nwg > INT32_MAX / 2) continue;
        bool bytes_bound = false;
        const double t = stream3_launch_us((int)nwg, n_cu, ER, EC, z, K, elem_bytes, depth, interior_cells,
                                           &bytes_bound);
        if (bytes_bound && deep_enough && (nwg < want || z < 4 * K)) continue;
        if (t < best) {
            best = t;
            zb = z;
        }
    }
    return zb;
}

}  // namespace dtb
