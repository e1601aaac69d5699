// lbm_tb2.hip — two time steps per pass over HBM (A/B pull streaming).
//
// A single step moves 2 * 19 * b bytes per cell through HBM, and the
// single-step kernel runs at the ceiling of that access pattern.  This kernel
// keeps the intermediate time level on chip instead: a workgroup owns a
// 62 x 14 tile of (x, y) columns plus a one-cell halo (64 x 16 = 1024
// threads) and marches along z through a chunk of planes.  Which (tile,
// chunk) a workgroup takes is planned on the host once per lattice shape
// (lbm_tb2_plan.hpp): each XCD owns a contiguous range of tiles and runs
// their chunks in order, the long ones first and one short chunk per tile
// last, so that its CUs run out of work at nearly the same time.
//   phase 1  each of the 1024 columns pulls f(t) of plane z+1 from A
//            (eq. mrt_dns_guo, periodic) and collides; of the post-collision
//            values it keeps in LDS exactly what phase 2 will pull: the 5
//            populations with c_z = -1 (needed now), the 9 with c_z = 0
//            (needed one plane later, 2 slots) and the 5 with c_z = +1
//            (needed two planes later, 3 slots): 38 floats per column,
//            152 KB of the 160 KB LDS of a CDNA4 CU;
//   phase 2  each interior column pulls the step-(t+1) populations of plane z
//            from those buffers (planes z+1, z, z-1 and the neighbouring
//            columns), collides and writes B at its own cell.
// The loads of the next phase-1 plane are issued before phase 2 so that they
// overlap with its arithmetic.  HBM traffic per two cell updates: A is read
// once per extended column (1024 / 868 of the interior, plus 2 planes per
// chunk) and B is written once, instead of two full reads and writes.
// Per cell the arithmetic is the single-step collision, and for 16-bit
// storage the LDS buffers hold the intermediate level in the storage format:
// the result is that of two single steps up to the rounding of the FP32
// collision (the compiler may fuse the collision's multiply-adds differently
// in the two kernels).  It does not depend on the work plan.
#include <algorithm>
#include <array>
#include <atomic>
#include <map>
#include <mutex>

#include "lbm_device.hpp"
#include "lbm_tb2_plan.hpp"

namespace lbm {

// Position of direction i within its class of c_z (-1: 5, 0: 9, +1: 5).
__host__ __device__ constexpr int zclass_index(int i) {
    int n = 0;
    for (int k = 0; k < i; ++k) n += (cz_of(k) == cz_of(i)) ? 1 : 0;
    return n;
}

struct TB2Args {
    LatticeArgs L;
    uint32_t tiles_x, tiles_y;
    Tb2Work W;
};

__device__ __forceinline__ uint32_t wrap_add(uint32_t base, int d, uint32_t n) {
    // (base + d) mod n for base < n and -1 <= d <= 64 (n >= 1)
    int v = (int)base + d;
    if (v < 0) v += (int)n;
    return (uint32_t)v % n;
}

template <class Cd, int TB_EY>
__global__ __launch_bounds__(TB_EX * TB_EY) void k_step_tb2(TB2Args A) {
    constexpr int TB_TY = TB_EY - 2, TB_E = TB_EX * TB_EY;
    using T = typename Cd::T;
    using R = typename Cd::R;
    static_assert(std::is_same_v<R, float>, "the collision runs in FP32");
    // 16-bit storage: the intermediate level stays in LDS in the storage format
    // (the values a single step would store), at 2 B per value.  That leaves room
    // to rotate the buffers over more slots (down 2, mid 3, up 4: 57 values per
    // column, 117 KB) so that phase 1 of the next plane may overwrite no slot
    // phase 2 of this plane still reads: one barrier per plane.  FP32 storage
    // keeps FP32 values in the minimal 38 slots (152 KB) and two barriers.
    constexpr bool k16 = sizeof(T) == 2;
    using LT = std::conditional_t<k16, T, R>;
    constexpr int ND = k16 ? 2 : 1, NM = k16 ? 3 : 2, NU = k16 ? 4 : 3, NR = k16 ? 3 : 1;
    __shared__ LT down[ND][5][TB_E];   // c_z = -1 populations of plane z+1
    __shared__ LT mid[NM][9][TB_E];    // c_z =  0 populations, planes z+1, z (, z-1)
    __shared__ LT up[NU][5][TB_E];     // c_z = +1 populations, planes z+1, z, z-1 (, z-2)
    __shared__ R rowbuf[NR][TB_EY][16];  // force row coefficients of the phase-1 plane
    __shared__ R xbuf[TB_EX][4];         // x harmonics of the tile columns

    const LatticeArgs& L = A.L;
    uint32_t tile, Z0, nplanes;
    if (!tb2_item(A.W, L.nz, blockIdx.x, tile, Z0, nplanes)) return;   // padding: all leave
    const uint32_t tile_x = tile % A.tiles_x, tile_y = tile / A.tiles_x;
    const uint32_t X0 = tile_x * TB_TX, Y0 = tile_y * TB_TY;
    const int nzc = (int)nplanes;                                 // output planes of this chunk

    const int t = threadIdx.x;
    const int ex = t & (TB_EX - 1), ey = t / TB_EX;
    // phase-1 column: the extended tile, wrapped onto the lattice
    const uint32_t x1 = wrap_add(X0, ex - 1, L.nx), y1 = wrap_add(Y0, ey - 1, L.ny);
    // phase-2 column: interior only, never wrapped
    const uint32_t x2 = X0 + (uint32_t)ex - 1u, y2 = Y0 + (uint32_t)ey - 1u;
    const bool inner = ex >= 1 && ex <= TB_TX && ey >= 1 && ey <= TB_TY && x2 < L.nx && y2 < L.ny;

    // 16-bit storage: populations and force in units of 1/sigma (collide's
    // kScaled), so that every pass through the storage format is a conversion
    const R inv_s = inv_scale_of<R>(L), s_st = scale_of<R>(L);
    const R load_s = k16 ? R(1) : inv_s, store_s = k16 ? R(1) : s_st;
    const uint64_t pbytes = L.plane * (uint64_t)sizeof(T);
    const PlaneStride src{(char*)L.a, pbytes}, dst{(char*)L.b, pbytes};
    const CollideConst<R>& k = collide_const<R>(L);
    // 16-bit storage: the array bases are made opaque inside the loop, so the
    // compiler recomputes the 38 plane bases per use instead of keeping them
    // live across it and spilling scalar registers to VGPR lanes (at 800^3:
    // FP16 +1.4 %, BF16 +13 %; FP32 measured no gain and keeps hoisted bases)
    auto opaque_base = [&](char* p) -> char* {
        if constexpr (k16) asm volatile("" : "+s"(p));
        return p;
    };
    auto to_lds = [&](R v) -> LT {
        if constexpr (k16) return enc<Cd>(v, R(1));
        else return v;
    };
    auto from_lds = [&](LT v) -> R {
        if constexpr (k16) return dec<Cd>(v, R(1));
        else return v;
    };

    auto plane1 = [&](int j) {   // z of the phase-1 plane of iteration j: Z0 - 1 + j, wrapped
        int z = (int)Z0 - 1 + j;
        if (z < 0) z += (int)L.nz;
        if (z >= (int)L.nz) z -= (int)L.nz;
        return (uint32_t)z;
    };
    auto pull = [&](int j, R (&g)[19]) {
        CellPos p;
        p.x = x1;
        p.y = y1;
        p.z = plane1(j);
        p.row = y1 + L.ny * p.z;
        const Nbr nb = make_nbr(p, L);
        load_cell<Cd, PAT_AB>(PlaneStride{opaque_base(src.base), pbytes}, x1 + L.nx * p.row, nb,
                              g, load_s);
    };

    // Force (eq. forcing_pattern via the row / x-harmonic tables).  With 16-bit
    // storage the row coefficients of a phase-1 plane are fetched two iterations
    // ahead into LDS by the first 16 * TB_EY threads (one value each: tile row r,
    // coefficient e) and the x harmonics of the 64 columns sit in LDS, so phase 1
    // waits on no table load (+9 % at 800^3).  With FP32 storage that costs more
    // than it saves (-7 %): phase 1 reads the tables directly.
    const bool forced = L.rowc != nullptr;
    const R* rowc = (const R*)L.rowc;
    const int rr = t >> 4, re = t & 15;           // for t < 16 * TB_EY
    const bool row_loader = k16 && forced && t < 16 * TB_EY;
    const uint32_t ry = wrap_add(Y0, rr - 1, L.ny);
    auto row_coeff = [&](int j) { return rowc[(uint64_t)(ry + L.ny * plane1(j)) * 16 + re]; };
    const int niter = nzc + 2;
    if constexpr (k16) {
        if (forced && t < 4 * TB_EX)
            xbuf[t >> 2][t & 3] =
                ((const R*)L.xtab)[(uint64_t)wrap_add(X0, (t >> 2) - 1, L.nx) * 4 + (t & 3)];
        if (row_loader) {
            rowbuf[0][rr][re] = row_coeff(0);
            rowbuf[1][rr][re] = row_coeff(1);   // niter >= 3
        }
        __syncthreads();
    }

    // One iteration j: phase 1 on the prefetched pulls P of plane Z0 - 1 + j,
    // then the pulls of plane j + 2 are issued into P (two planes of prefetch
    // in flight), then phase 2 on plane Z0 + j - 2.
    // The phase-2 cell of iteration j is the phase-1 cell of iteration j - 1 (same
    // column, plane Z0 + j - 2): its force is carried over instead of recomputed.
    R Fpx = R(0), Fpy = R(0), Fpz = R(0);
    auto iteration = [&](int j, R (&P)[19]) {
        const uint32_t uj = (uint32_t)j;
        R Fx = R(0), Fy = R(0), Fz = R(0);
        {   // phase 1: step t at plane Z0 - 1 + j for every extended column
            R g[19];
#pragma unroll
            for (int i = 0; i < 19; ++i) g[i] = P[i];
            if constexpr (k16) {
                if (forced) {
                    const R* rc = rowbuf[uj % NR][ey];
                    const R s1 = xbuf[ex][0], c1 = xbuf[ex][1], s2 = xbuf[ex][2], c2 = xbuf[ex][3];
                    Fx = rc[0] + s1 * rc[3] + c1 * rc[6] + s2 * rc[9] + c2 * rc[12];
                    Fy = rc[1] + s1 * rc[4] + c1 * rc[7] + s2 * rc[10] + c2 * rc[13];
                    Fz = rc[2] + s1 * rc[5] + c1 * rc[8] + s2 * rc[11] + c2 * rc[14];
                    Fx *= s_st;
                    Fy *= s_st;
                    Fz *= s_st;
                }
            } else {
                CellPos p;
                p.x = x1;
                p.y = y1;
                p.z = plane1(j);
                p.row = y1 + L.ny * p.z;
                force_at<R>(L, p, Fx, Fy, Fz);
            }
            collide<R, true, k16>(g, Fx, Fy, Fz, k, inv_s);
            const uint32_t sd = uj % ND, sm = uj % NM, su = uj % NU;
            static_for<19>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int cz = cz_of(i), ii = zclass_index(i);
                const LT v = to_lds(g[i]);
                if constexpr (cz < 0) down[sd][ii][t] = v;
                else if constexpr (cz == 0) mid[sm][ii][t] = v;
                else up[su][ii][t] = v;
            });
        }
        __syncthreads();
        // (16-bit storage) the row coefficients of the phase-1 plane two iterations on
        R rnext = R(0);
        const bool fetch = row_loader && j + 2 < niter;
        if (fetch) rnext = row_coeff(j + 2);
        if (j + 2 < niter) pull(j + 2, P);
        if (j >= 2 && inner) {   // phase 2: step t+1 at plane Z0 + j - 2
            const uint32_t z2 = Z0 + (uint32_t)(j - 2);
            R g[19];
            // planes z2 + 1, z2 and z2 - 1: phase 1 of iterations j, j - 1, j - 2
            const uint32_t sd = uj % ND, sm = (uj - 1) % NM, su = (uj - 2) % NU;
            static_for<19>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i), ii = zclass_index(i);
                const int col = (ex - cx) + TB_EX * (ey - cy);
                if constexpr (cz < 0) g[i] = from_lds(down[sd][ii][col]);
                else if constexpr (cz == 0) g[i] = from_lds(mid[sm][ii][col]);
                else g[i] = from_lds(up[su][ii][col]);
            });
            collide<R, true, k16>(g, Fpx, Fpy, Fpz, k, inv_s);
            const uint32_t cell = x2 + L.nx * (y2 + L.ny * z2);
            const PlaneStride out{opaque_base(dst.base), pbytes};
            static_for<19>([&](auto I) {
                constexpr int i = decltype(I)::value;
                *elem_ptr<T>(out, i, cell) = enc<Cd>(g[i], store_s);
            });
        }
        // read by phase 1 two iterations on, after the next barrier; the slot was
        // last read by phase 1 of iteration j - 1, which every thread has passed
        if (fetch) rowbuf[(uj + 2) % NR][rr][re] = rnext;
        Fpx = Fx;
        Fpy = Fy;
        Fpz = Fz;
        // With the rotating 16-bit slots, phase 1 of iteration j + 1 writes no
        // slot that phase 2 of iteration j reads, and phase 1 of j + 2 waits at
        // the barrier of j + 1 for every phase 2 of j: no second barrier.
        if constexpr (!k16) __syncthreads();
    };

    R pa[19], pb[19];
    pull(0, pa);
    pull(1, pb);    // niter >= 3, so plane 1 always exists
    for (int j = 0; j < niter; j += 2) {   // unrolled by two: pa, pb stay in registers
        iteration(j, pa);
        if (j + 1 < niter) iteration(j + 1, pb);
    }
}

bool tb2_supported(int precision) { return precision != LBM_FP64; }

namespace {

// Compute units of the current device, asked once per device.
uint32_t compute_units() {
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return (uint32_t)n;
}

// Plans are made once per (shape, grouping, CU count) and kept.
const Tb2Plan& plan_for(uint32_t nx, uint32_t ny, uint32_t nz, uint32_t tiles_x,
                        uint32_t tiles_y, uint32_t groups) {
    static std::mutex mu;
    static std::map<std::array<uint32_t, 5>, Tb2Plan> plans;
    const uint32_t cus = compute_units();
    const std::array<uint32_t, 5> key{nx, ny, nz, groups, cus};
    std::lock_guard<std::mutex> lock(mu);
    auto it = plans.find(key);
    if (it == plans.end())
        it = plans.emplace(key, make_plan(nx, ny, nz, tiles_x, tiles_y, groups, cus)).first;
    return it->second;
}

}  // namespace

hipError_t launch_step_tb2(int precision, const LatticeArgs& L, hipStream_t s) {
    // 64 x 16 extended tiles: one 1024-thread workgroup and 117-155 KB of LDS per CU.
    // (64 x 8 tiles, two workgroups per CU, measured 25 % slower at 800^3.)
    constexpr int EY = kTbEY;
    TB2Args A;
    A.L = L;
    A.tiles_x = (L.nx + TB_TX - 1) / TB_TX;
    A.tiles_y = (L.ny + (EY - 2) - 1) / (EY - 2);
    // one tile range per XCD whenever a block order is asked for
    const uint32_t groups = L.xcd_remap ? 8u : 1u;
    const Tb2Plan& P = plan_for(L.nx, L.ny, L.nz, A.tiles_x, A.tiles_y, groups);
    A.W = P.w;
    const uint64_t nblocks = (uint64_t)P.w.groups * P.per_group;
    if (nblocks == 0 || nblocks > 0x7fffffffull) return hipErrorInvalidValue;
    const dim3 grid((uint32_t)nblocks), block(TB_EX * EY);
    switch (precision) {
        case LBM_FP32: hipLaunchKernelGGL((k_step_tb2<CdF32, EY>), grid, block, 0, s, A); break;
        case LBM_FP16_DEV: hipLaunchKernelGGL((k_step_tb2<CdF16, EY>), grid, block, 0, s, A); break;
        case LBM_BF16_DEV: hipLaunchKernelGGL((k_step_tb2<CdBF16, EY>), grid, block, 0, s, A); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
