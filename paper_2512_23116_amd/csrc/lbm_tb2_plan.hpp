// lbm_tb2_plan.hpp — which (tile, z chunk) each workgroup of the two-step
// kernel takes, and the host's choice of that plan for a lattice shape.
// The item lookup is plain integer code shared by the kernel and the host test
// of the plan (built with address and undefined-behaviour sanitizers).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <functional>
#include <queue>
#include <vector>

namespace lbm {

// Extended tile of one workgroup: 64 x 16 columns, of which the inner 62 x 14
// are the tile and the rest its one-cell halo.
constexpr int TB_EX = 64, TB_TX = TB_EX - 2;
constexpr int kTbEY = 16, kTbTY = kTbEY - 2;
constexpr int TB_MAX_CHUNKS = 64;

// Work plan of a launch: the tiles are split into `groups` contiguous ranges
// cut[g] .. cut[g+1] (one per XCD; workgroup h runs on XCD h % 8), every tile
// into the same z chunks of zlen planes, the last one shorter: chunk k is planes
// k zlen .. min((k+1) zlen, nz) - 1.  Workgroup h takes item h / groups of its
// group, items ordered chunk-major: chunk k of every tile of the range, in tile
// order, then chunk k + 1.  Groups with fewer items pad with workgroups that
// exit at once.
struct Tb2Work {
    uint32_t groups, nchunk, zlen;
    uint32_t cut[9];
};

// Tile index, first plane and plane count of workgroup h of a lattice nz planes
// deep; false for padding.
__host__ __device__ inline bool tb2_item(const Tb2Work& W, uint32_t nz, uint32_t h,
                                         uint32_t& tile, uint32_t& z0, uint32_t& nzc) {
    const uint32_t grp = h % W.groups, item = h / W.groups;
    const uint32_t t0 = W.cut[grp], nt = W.cut[grp + 1] - t0;
    if (item >= nt * W.nchunk) return false;
    const uint32_t chunk = item / nt;
    tile = t0 + (item - chunk * nt);
    z0 = chunk * W.zlen;
    nzc = (nz - z0 < W.zlen) ? nz - z0 : W.zlen;
    return true;
}

struct Tb2Plan {
    Tb2Work w{};
    uint32_t per_group = 0;   // workgroups per group: the launch has groups * per_group
};

// Relative cost of one plane of a tile: phase 1 runs on all 64 x 16 columns,
// phase 2 on the interior only, about 35 % of a full tile's time (a tile with
// 2 of its 14 interior rows takes 0.70 of a full one at 800^3).
inline double tile_cost(uint32_t tile, uint32_t tiles_x, uint32_t nx, uint32_t ny) {
    const uint32_t x = tile % tiles_x, y = tile / tiles_x;
    const uint32_t w = std::min<uint32_t>(TB_TX, nx - x * TB_TX);
    const uint32_t h = std::min<uint32_t>(kTbTY, ny - y * kTbTY);
    return 0.65 + 0.35 * double(w * h) / double(TB_TX * kTbTY);
}

// Finishing time of the slowest group when each group's CUs take its items in
// order as they free up (list scheduling), an item costing its planes plus
// three: the two planes a chunk starts with and the workgroup's start-up (at
// 800^3 an item takes about 10 us plus 5.7 us per plane, and about 5 us pass
// between two items on a CU), times its tile's cost.
inline double plan_makespan(const Tb2Plan& P, uint32_t nz, const std::vector<double>& cost,
                            uint32_t cus_per_group) {
    double worst = 0.0;
    std::vector<double> cu;
    for (uint32_t g = 0; g < P.w.groups; ++g) {
        cu.assign(std::max<uint32_t>(1, cus_per_group), 0.0);
        std::priority_queue<double, std::vector<double>, std::greater<double>> q(cu.begin(),
                                                                               cu.end());
        for (uint32_t k = 0; k < P.w.nchunk; ++k) {
            const uint32_t z0 = k * P.w.zlen, n = std::min(P.w.zlen, nz - z0);
            const double planes = double(n + 3);
            for (uint32_t t = P.w.cut[g]; t < P.w.cut[g + 1]; ++t) {
                const double free_at = q.top();
                q.pop();
                q.push(free_at + planes * cost[t]);
            }
        }
        while (!q.empty()) {
            worst = std::max(worst, q.top());
            q.pop();
        }
    }
    return worst;
}

// The plan for a lattice shape: tiles cut into `groups` ranges of equal total
// cost, and of the chunk lengths tried (every length from 16 planes up to nz
// that changes the chunk count or the last chunk's length by a step) the one
// with the smallest estimated finishing time.
inline Tb2Plan make_plan(uint32_t nx, uint32_t ny, uint32_t nz, uint32_t tiles_x,
                         uint32_t tiles_y, uint32_t groups, uint32_t cus) {
    const uint32_t tiles = tiles_x * tiles_y;
    std::vector<double> cost(tiles), cum(tiles + 1, 0.0);
    for (uint32_t t = 0; t < tiles; ++t) {
        cost[t] = tile_cost(t, tiles_x, nx, ny);
        cum[t + 1] = cum[t] + cost[t];
    }
    Tb2Plan best;
    best.w.groups = groups;
    for (uint32_t g = 0; g <= groups; ++g) {
        const double target = cum[tiles] * g / groups;
        uint32_t t = 0;
        while (t < tiles && cum[t] < target) ++t;
        best.w.cut[g] = (g == groups) ? tiles : t;
    }
    const uint32_t cus_per_group = std::max<uint32_t>(1, cus / groups);
    // more than 64 items per CU gain nothing and cost planning time
    const uint64_t max_items = 64ull * std::max<uint32_t>(1, cus);
    double best_ms = -1.0;
    auto consider = [&](uint32_t zlen) {
        Tb2Plan P = best;
        P.w.zlen = zlen;
        P.w.nchunk = (nz + zlen - 1) / zlen;
        if (P.w.nchunk > (uint32_t)TB_MAX_CHUNKS) return;
        if (P.w.nchunk > 1 && (uint64_t)tiles * P.w.nchunk > max_items) return;
        const double ms = plan_makespan(P, nz, cost, cus_per_group);
        if (best_ms < 0.0 || ms < best_ms * (1.0 - 1e-9)) {
            best_ms = ms;
            best = P;
        }
    };
    consider(nz);                          // one chunk: always possible
    const uint32_t step = std::max<uint32_t>(1, nz / 256);
    for (uint32_t zlen = 16; zlen < nz; zlen += step) consider(zlen);
    for (uint32_t g = 0; g < groups; ++g) {
        const uint32_t items = (best.w.cut[g + 1] - best.w.cut[g]) * best.w.nchunk;
        best.per_group = std::max(best.per_group, items);
    }
    return best;
}

}  // namespace lbm
