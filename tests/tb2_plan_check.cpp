// tb2_plan_check.cpp — host test of the two-step kernel's work plan
// (paper_2512_23116_amd/csrc/lbm_tb2_plan.hpp), built with address and
// undefined-behaviour sanitizers by tests/test_index_cpu.py.
//
// For every lattice shape, grouping and CU count tried, the plan the library
// would launch must cover each (tile, plane) unit of the lattice exactly once:
// the workgroups 0 .. groups * per_group - 1 of the launch, each looked up with
// tb2_item as the kernel does, take chunks of one tile that lie inside the
// lattice, every workgroup of group g a tile of its range, and the chunks
// of zlen planes (the last one shorter) reach nz.
//
// Exit status 0 and a summary line (with the 800^3 plan) on success; a message
// and status 1 on the first failure.
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "lbm_tb2_plan.hpp"

using lbm::Tb2Plan;

static int fail(const char* what, uint32_t nx, uint32_t ny, uint32_t nz, uint64_t a) {
    fprintf(stderr, "FAIL %s: shape %u x %u x %u, %llu\n", what, nx, ny, nz,
            (unsigned long long)a);
    return 1;
}

static int check(uint32_t nx, uint32_t ny, uint32_t nz, uint32_t groups, uint32_t cus,
                 uint64_t* launched) {
    const uint32_t tx = (nx + lbm::TB_TX - 1) / lbm::TB_TX;
    const uint32_t ty = (ny + lbm::kTbTY - 1) / lbm::kTbTY;
    const uint32_t tiles = tx * ty;
    const Tb2Plan P = lbm::make_plan(nx, ny, nz, tx, ty, groups, cus);
    const lbm::Tb2Work& W = P.w;
    if (W.groups != groups) return fail("groups", nx, ny, nz, W.groups);
    if (W.nchunk < 1 || W.nchunk > (uint32_t)lbm::TB_MAX_CHUNKS)
        return fail("chunk count", nx, ny, nz, W.nchunk);
    if (W.zlen < 1 || (uint64_t)W.zlen * (W.nchunk - 1) >= nz ||
        (uint64_t)W.zlen * W.nchunk < nz)
        return fail("z chunks", nx, ny, nz, W.zlen);
    if (W.cut[0] != 0 || W.cut[groups] != tiles) return fail("tile bounds", nx, ny, nz, groups);
    uint32_t most = 0;
    for (uint32_t g = 0; g < groups; ++g) {
        if (W.cut[g + 1] < W.cut[g]) return fail("tile ranges", nx, ny, nz, g);
        const uint32_t items = (W.cut[g + 1] - W.cut[g]) * W.nchunk;
        most = items > most ? items : most;
    }
    if (P.per_group != most) return fail("workgroups per group", nx, ny, nz, P.per_group);
    std::vector<uint8_t> seen((size_t)tiles * nz, 0);
    uint64_t items = 0;
    const uint64_t G = (uint64_t)groups * P.per_group;
    for (uint64_t h = 0; h < G; ++h) {
        uint32_t tile = 0, z0 = 0, n = 0;
        if (!lbm::tb2_item(W, nz, (uint32_t)h, tile, z0, n)) continue;
        ++items;
        const uint32_t g = (uint32_t)(h % groups);
        if (tile < W.cut[g] || tile >= W.cut[g + 1]) return fail("tile outside its group", nx, ny,
                                                                 nz, h);
        if (n < 1 || z0 + n > nz) return fail("chunk outside the lattice", nx, ny, nz, h);
        for (uint32_t z = z0; z < z0 + n; ++z) {
            uint8_t& s = seen[(size_t)tile * nz + z];
            if (s) return fail("unit taken twice", nx, ny, nz, (uint64_t)tile * nz + z);
            s = 1;
        }
    }
    if (items != (uint64_t)tiles * W.nchunk) return fail("item count", nx, ny, nz, items);
    for (size_t u = 0; u < seen.size(); ++u)
        if (!seen[u]) return fail("unit never taken", nx, ny, nz, u);
    *launched += G;
    return 0;
}

int main() {
    const uint32_t small_xy[] = {1, 2, 13, 14, 15, 61, 62, 63, 64, 100, 125};
    const uint32_t zs[] = {1, 2, 3, 15, 16, 17, 31, 32, 33, 64, 67, 130, 400};
    uint64_t plans = 0, launched = 0;
    for (uint32_t nx : small_xy)
        for (uint32_t ny : small_xy)
            for (uint32_t nz : zs)
                for (uint32_t groups : {1u, 8u})
                    for (uint32_t cus : {1u, 80u, 256u}) {
                        if (check(nx, ny, nz, groups, cus, &launched)) return 1;
                        ++plans;
                    }
    const uint32_t large[][3] = {{800, 800, 800}, {1290, 1290, 1290}, {256, 256, 256},
                                 {512, 512, 512}, {800, 800, 1}, {1, 1, 1290},
                                 {62, 14, 800}, {600, 400, 1000}, {66, 64, 67}};
    for (const auto& s : large)
        for (uint32_t groups : {1u, 8u}) {
            if (check(s[0], s[1], s[2], groups, 256, &launched)) return 1;
            ++plans;
        }
    const Tb2Plan P = lbm::make_plan(800, 800, 800, 13, 58, 8, 256);
    printf("ok: %llu plans, %llu workgroups looked up; 800^3 on 8 x 32 CUs: %u workgroups, "
           "chunks", (unsigned long long)plans, (unsigned long long)launched,
           8 * P.per_group);
    for (uint32_t k = 0; k < P.w.nchunk; ++k)
        printf(" %u", (800 - k * P.w.zlen < P.w.zlen) ? 800 - k * P.w.zlen : P.w.zlen);
    printf("\n");
    return 0;
}
