// dtb_plan.cpp -- tile planner (host C++, no HIP calls).
#include "dtb_plan.h"

#include <algorithm>
#include <cmath>

namespace dtb {

bool split_axis(int64_t len, int ext, int k, int parts, AxisSplit* out)
{
    if (len < 1 || ext < 1 || k < 1 || parts < 1 || parts > len) return false;
    AxisSplit s;
    s.parts = parts;
    s.bounds.assign(parts + 1, 0);
    s.ext0.assign(parts, 1);
    if (parts == 1) {
        if (len > ext) return false;
        s.bounds[0] = 1;
        s.bounds[1] = (int)len + 1;
        s.ext0[0] = 1;
        s.narrow = len < ext;
        *out = s;
        return true;
    }
    if (len < ext) return false;  // several tiles need aligned extended tiles inside the axis
    // Capacities: an edge tile needs a ghost ring on one side only.
    std::vector<int64_t> cap(parts), w(parts, 0);
    for (int i = 0; i < parts; ++i) cap[i] = (i == 0 || i == parts - 1) ? ext - k : ext - 2 * k;
    for (int i = 0; i < parts; ++i)
        if (cap[i] < 1) return false;
    // Even split, then hand the remainder to tiles with room, edges first.
    const int64_t q = len / parts;
    int64_t left = len;
    for (int i = 0; i < parts; ++i) {
        w[i] = std::min<int64_t>(q, cap[i]);
        left -= w[i];
    }
    std::vector<int> order;
    order.push_back(0);
    order.push_back(parts - 1);
    for (int i = 1; i < parts - 1; ++i) order.push_back(i);
    while (left > 0) {
        bool moved = false;
        for (int i : order) {
            if (left == 0) break;
            if (w[i] < cap[i]) {
                ++w[i];
                --left;
                moved = true;
            }
        }
        if (!moved) return false;
    }
    s.bounds[0] = 1;
    for (int i = 0; i < parts; ++i) s.bounds[i + 1] = s.bounds[i] + (int)w[i];
    for (int i = 0; i < parts; ++i) {
        const int64_t o0 = s.bounds[i], o1 = s.bounds[i + 1];
        int64_t e0 = std::min<int64_t>(std::max<int64_t>(o0 - k, 1), len - ext + 1);
        const int64_t f0 = std::max<int64_t>(o0 - k, 1), f1 = std::min<int64_t>(o1 + k, len + 1);
        if (f0 < e0 || f1 > e0 + ext || w[i] < 1) return false;
        s.ext0[i] = (int)e0;
    }
    s.narrow = false;
    *out = s;
    return true;
}

int min_parts(int64_t len, int ext, int k, int max_parts)
{
    if (len <= ext) return 1;
    // Capacity grows linearly in parts: 2(ext-k) + (parts-2)(ext-2k).
    if (ext - 2 * k < 1) {
        AxisSplit s;
        return split_axis(len, ext, k, 2, &s) ? 2 : 0;
    }
    int64_t p = 2;
    if (len > 2 * (int64_t)(ext - k)) p = 2 + (len - 2 * (int64_t)(ext - k) + (ext - 2 * k) - 1) / (ext - 2 * k);
    for (; p <= max_parts && p <= len; ++p) {
        AxisSplit s;
        if (split_axis(len, ext, k, (int)p, &s)) return (int)p;
    }
    return 0;
}

bool build_layout(int64_t rows, int64_t cols, int R, int C, int waves, int k, int n_xcd, int wg_base,
                  int prob, Layout* out)
{
    Layout L;
    L.R = R;
    L.C = C;
    L.waves = waves;
    L.ER = waves * R;
    L.EC = kWaveSize * C;
    L.k = k;
    const int pr = min_parts(rows, L.ER, k, 1 << 20);
    const int pc = min_parts(cols, L.EC, k, 1 << 20);
    if (pr < 1 || pc < 1) return false;
    if (!split_axis(rows, L.ER, k, pr, &L.rows) || !split_axis(cols, L.EC, k, pc, &L.cols)) return false;
    const int n = pr * pc;
    L.nwg = n;

    // Spatial order: cut the pr x pc tile grid into gy x gx blocks (gy * gx =
    // n_xcd, blocks as square as possible in cells), list the tiles block by
    // block, row-major inside each block.
    int gy = 1, gx = 1;
    if (n_xcd > 1) {
        double best = 1e300;
        for (int a = 1; a <= n_xcd; ++a) {
            if (n_xcd % a) continue;
            const int b = n_xcd / a;
            if (a > pr || b > pc) continue;
            const double h = (double)rows / a, w = (double)cols / b;
            const double score = std::max(h / w, w / h);
            if (score < best) {
                best = score;
                gy = a;
                gx = b;
            }
        }
    }
    std::vector<int> spatial;  // tile id = tr * pc + tc, in XCD-block order
    spatial.reserve(n);
    for (int by = 0; by < gy; ++by) {
        const int r0 = (int)((int64_t)pr * by / gy), r1 = (int)((int64_t)pr * (by + 1) / gy);
        for (int bx = 0; bx < gx; ++bx) {
            const int c0 = (int)((int64_t)pc * bx / gx), c1 = (int)((int64_t)pc * (bx + 1) / gx);
            for (int tr = r0; tr < r1; ++tr)
                for (int tc = c0; tc < c1; ++tc) spatial.push_back(tr * pc + tc);
        }
    }
    // Workgroup b of the launch runs on XCD (wg_base + b) % n_xcd; list the
    // launch slots XCD by XCD and give them the tiles in spatial order.
    std::vector<int> slots(n);
    for (int b = 0; b < n; ++b) slots[b] = b;
    const int nx = std::max(n_xcd, 1);
    std::stable_sort(slots.begin(), slots.end(), [&](int x, int y) {
        const int ax = (wg_base + x) % nx, ay = (wg_base + y) % nx;
        return ax < ay;
    });
    std::vector<int> slot_of_tile(n);
    for (int i = 0; i < n; ++i) slot_of_tile[spatial[i]] = slots[i];

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
            d.nnb = 0;
        }
    }
    for (int a = 0; a < n; ++a) {
        WgDesc& d = L.wgs[a];
        const int f_r0 = d.own_r0 - k, f_r1 = d.own_r1 + k, f_c0 = d.own_c0 - k, f_c1 = d.own_c1 + k;
        for (int b = 0; b < n; ++b) {
            if (b == a) continue;
            const WgDesc& o = L.wgs[b];
            const bool meet = o.own_r0 < f_r1 && o.own_r1 > f_r0 && o.own_c0 < f_c1 && o.own_c1 > f_c0;
            if (!meet) continue;
            if (d.nnb >= kMaxNeighbours) return false;
            d.nb[d.nnb++] = wg_base + b;
        }
    }
    *out = std::move(L);
    return true;
}

double layout_cost(const Layout& L, int slots_per_cu, int n_cu, double sync_steps)
{
    const int slots = std::max(1, slots_per_cu) * std::max(1, n_cu);
    if (L.nwg > slots) return 1e300;
    const int per_cu = (L.nwg + n_cu - 1) / n_cu;
    const double cells = (double)per_cu * L.ER * L.EC;
    return cells * (1.0 + sync_steps / L.k);
}

}  // namespace dtb
