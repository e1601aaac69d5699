// lbm_device.hpp — device-side building blocks shared by the single-lattice
// kernels (lbm_kernels.hip) and the batched serving kernel (lbm_batch.hip):
// storage codecs, index decode with periodic neighbours, the AA / A-B access
// patterns, and the per-cell body force.
#pragma once

#include <math.h>

#include <type_traits>
#include <utility>

#include "d3q19_mrt.hpp"
#include "lbm_internal.hpp"

namespace lbm {

// --------------------------------------------------------------- codecs ---
struct CdF64 { using T = double;   using R = double; };
struct CdF32 { using T = float;    using R = float;  };
struct CdF16 { using T = _Float16; using R = float;  };
struct CdBF16 { using T = uint16_t; using R = float; };

__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <class Cd>
__device__ __forceinline__ typename Cd::R dec(typename Cd::T v, typename Cd::R inv_s) {
    if constexpr (std::is_same_v<Cd, CdF16>) return (float)v * inv_s;
    else if constexpr (std::is_same_v<Cd, CdBF16>) return __uint_as_float((uint32_t)v << 16) * inv_s;
    else return v;
}
template <class Cd>
__device__ __forceinline__ typename Cd::T enc(typename Cd::R v, typename Cd::R s) {
    if constexpr (std::is_same_v<Cd, CdF16>) return (_Float16)(v * s);   // v_cvt_f16_f32: RNE
    else if constexpr (std::is_same_v<Cd, CdBF16>) return bf16_rne(v * s);
    else return v;
}

// ---------------------------------------------------------- small tools ---
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ uint32_t fast_div(uint32_t n, DivMagic d) {
    return (__umulhi(n, d.m) + n) >> d.s;
}

// Offsets (in cells) from x to x-1, x+1, y-1, ... with periodic wrap.
struct Nbr {
    int32_t xm, xp, ym, yp, zm, zp;
};

struct CellPos {
    uint32_t x, y, z, row;   // row = y + ny z
};

__device__ __forceinline__ CellPos decode(uint32_t cell, const LatticeArgs& L) {
    CellPos p;
    p.row = fast_div(cell, L.mx);
    p.x = cell - p.row * L.nx;
    p.z = fast_div(p.row, L.my);
    p.y = p.row - p.z * L.ny;
    return p;
}

__device__ __forceinline__ Nbr make_nbr(const CellPos& p, const LatticeArgs& L) {
    Nbr n;
    const int32_t nx = (int32_t)L.nx, sy = (int32_t)L.nx, sz = (int32_t)L.nxy;
    n.xm = (p.x == 0) ? nx - 1 : -1;
    n.xp = (p.x == L.nx - 1) ? 1 - nx : 1;
    n.ym = (p.y == 0) ? ((int32_t)L.ny - 1) * sy : -sy;
    n.yp = (p.y == L.ny - 1) ? (1 - (int32_t)L.ny) * sy : sy;
    n.zm = (p.z == 0) ? ((int32_t)L.nz - 1) * sz : -sz;
    n.zp = (p.z == L.nz - 1) ? (1 - (int32_t)L.nz) * sz : sz;
    return n;
}

// Offset of the cell x - c_I.
template <int I>
__device__ __forceinline__ int32_t off_minus(const Nbr& n) {
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
    int32_t o = 0;
    if constexpr (cx == 1) o += n.xm; else if constexpr (cx == -1) o += n.xp;
    if constexpr (cy == 1) o += n.ym; else if constexpr (cy == -1) o += n.yp;
    if constexpr (cz == 1) o += n.zm; else if constexpr (cz == -1) o += n.zp;
    return o;
}

// Runtime-direction variant (observation kernels only).
__device__ __forceinline__ int32_t off_minus_rt(int i, const Nbr& n) {
    const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
    int32_t o = 0;
    o += cx == 1 ? n.xm : (cx == -1 ? n.xp : 0);
    o += cy == 1 ? n.ym : (cy == -1 ? n.yp : 0);
    o += cz == 1 ? n.zm : (cz == -1 ? n.zp : 0);
    return o;
}

__device__ __forceinline__ uint32_t block_id(const LatticeArgs& L) {
    uint32_t b = blockIdx.x;
    if (L.xcd_remap) {
        // MI355X dispatches consecutive workgroups round-robin over its 8 XCDs;
        // give each XCD one contiguous range of blocks instead.
        const uint32_t G = gridDim.x, xcd = b & 7u, local = b >> 3;
        const uint32_t per = G >> 3, rem = G & 7u;
        b = xcd * per + (xcd < rem ? xcd : rem) + local;
    }
    return b;
}

// Location of the pre-collision f_i(x) for pattern PAT: slot and cell.
//   AA_EVEN: (i, x)   AA_ODD: (opp i, x - c_i)   AB: (i, x - c_i)
template <class Cd, int PAT>
__device__ __forceinline__ void load_cell(const typename Cd::T* base, uint64_t plane, uint32_t cell,
                                          const Nbr& nb, typename Cd::R (&g)[19],
                                          typename Cd::R inv_s) {
    static_for<19>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int slot = (PAT == PAT_AA_ODD) ? opp_of(i) : i;
        const uint32_t c = (PAT == PAT_AA_EVEN) ? cell : cell + (uint32_t)off_minus<i>(nb);
        g[i] = dec<Cd>(base[(uint64_t)slot * plane + c], inv_s);
    });
}

// Where the post-collision f*_i(x) goes for pattern PAT (the pattern the step
// reads with): AA_EVEN -> (opp i, x); AA_ODD -> (i, x + c_i); AB -> (i, x) of dst.
template <class Cd, int PAT>
__device__ __forceinline__ void store_cell(typename Cd::T* base, uint64_t plane, uint32_t cell,
                                           const Nbr& nb, const typename Cd::R (&g)[19],
                                           typename Cd::R s) {
    static_for<19>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int slot = (PAT == PAT_AA_EVEN) ? opp_of(i) : i;
        const uint32_t c = (PAT == PAT_AA_ODD) ? cell + (uint32_t)off_minus<opp_of(i)>(nb) : cell;
        base[(uint64_t)slot * plane + c] = enc<Cd>(g[i], s);
    });
}

template <typename R>
__device__ __forceinline__ CollideConst<R> collide_const(const LatticeArgs& L) {
    CollideConst<R> k;
    k.tau0 = (R)L.tau0; k.c3 = (R)L.c3; k.a_e = (R)L.a_e; k.b9 = (R)L.b9;
    k.s_e = (R)L.s_e; k.s_eps = (R)L.s_eps; k.s_q = (R)L.s_q; k.s_pi = (R)L.s_pi;
    k.s_m = (R)L.s_m; k.rho0 = (R)L.rho0;
    return k;
}

// Body force at (x, row) from the row coefficients and the x-harmonic table:
// F = c0 + A1 sin(2 pi x/nx) + B1 cos(2 pi x/nx) + A2 sin(4 pi x/nx) + B2 cos(4 pi x/nx).
template <typename R>
__device__ __forceinline__ void force_at(const LatticeArgs& L, const CellPos& p, R& Fx, R& Fy,
                                         R& Fz) {
    if (L.rowc == nullptr) {
        Fx = Fy = Fz = R(0);
        return;
    }
    const R* rc = (const R*)L.rowc + (uint64_t)p.row * 16;
    const R* xt = (const R*)L.xtab + (uint64_t)p.x * 4;
    const R s1 = xt[0], c1 = xt[1], s2 = xt[2], c2 = xt[3];
    Fx = rc[0] + s1 * rc[3] + c1 * rc[6] + s2 * rc[9] + c2 * rc[12];
    Fy = rc[1] + s1 * rc[4] + c1 * rc[7] + s2 * rc[10] + c2 * rc[13];
    Fz = rc[2] + s1 * rc[5] + c1 * rc[8] + s2 * rc[11] + c2 * rc[14];
}

// One cell of the fused stream-and-collide step (eq. mrt_les_guo): gather the
// 19 pre-collision populations of pattern PAT, collide, scatter.
template <class Cd, int PAT>
__device__ __forceinline__ void step_cell(const LatticeArgs& L, uint32_t cell) {
    using T = typename Cd::T;
    using R = typename Cd::R;
    const CellPos p = decode(cell, L);
    const Nbr nb = make_nbr(p, L);
    R g[19];
    load_cell<Cd, PAT>((const T*)L.a, L.plane, cell, nb, g, (R)L.inv_sigma);
    R Fx, Fy, Fz;
    force_at<R>(L, p, Fx, Fy, Fz);
    collide<R, true>(g, Fx, Fy, Fz, collide_const<R>(L));
    store_cell<Cd, PAT>((T*)(PAT == PAT_AB ? L.b : L.a), L.plane, cell, nb, g, (R)L.sigma);
}

}  // namespace lbm
