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

// float -> bf16 with round-to-nearest-even.  gfx950 has a conversion
// instruction for it (v_cvt_pk_bf16_f32, emitted for this cast): one
// instruction where the integer rounding took six, bit-identical to it for
// every finite input (NaN stays NaN).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    const __bf16 h = (__bf16)x;
    return __builtin_bit_cast(uint16_t, h);
}

// Whether the one-step kernel collides on the stored scale (collide's kScaled),
// so that the codec reduces to conversions: for BF16 (shift / convert plus a
// multiply each way otherwise).  FP16 keeps the unscaled form: its decode and
// encode already fold the scale into mixed-precision FMAs (v_fma_mix*), and
// the scaled form measured 5 VALU instructions more per cell.
template <class Cd>
constexpr bool kScaledCodec = std::is_same_v<Cd, CdBF16>;

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

// Element index (slot * plane + cell) of the canonical f_i(x) for a runtime
// direction and pattern (set-up and observation kernels).
__device__ __forceinline__ uint64_t canon_index(int pat, int i, uint32_t cell, const Nbr& nb,
                                                uint64_t plane) {
    const int slot = (pat == PAT_AA_ODD) ? opp_of(i) : i;
    const uint32_t c = (pat == PAT_AA_EVEN) ? cell : cell + (uint32_t)off_minus_rt(i, nb);
    return (uint64_t)slot * plane + c;
}

// Block of cells of this workgroup in the XCD-aware order of L.xcd_remap.
__device__ __forceinline__ uint32_t block_id(const LatticeArgs& L) {
    return block_order(blockIdx.x, gridDim.x, L.xcd_remap);
}

// Plane addressing.  The 64-bit base of plane `slot` is uniform (SGPRs) and
// the per-lane part is a 32-bit byte offset (plane bytes < 2^32 is enforced at
// create), which maps to global loads and stores with a scalar base.  Two ways
// to get the plane base:
//  * PlaneTable: the 19 bases precomputed on the host, read from the kernel
//    arguments (no scalar arithmetic; used where they need not stay live across
//    a loop);
//  * PlaneStride: array base + slot * plane bytes (a few scalar instructions,
//    no extra SGPRs held; used by the z-marching two-step kernel).
struct PlaneTable {
    char* const* p;
    __device__ __forceinline__ char* operator()(int slot) const { return p[slot]; }
};
struct PlaneStride {
    char* base;
    uint64_t bytes;
    __device__ __forceinline__ char* operator()(int slot) const {
        return base + (uint64_t)slot * bytes;
    }
};

template <typename T, class Planes>
__device__ __forceinline__ T* elem_ptr(const Planes& planes, int slot, uint32_t c) {
    return (T*)(planes(slot) + (uint32_t)(c * (uint32_t)sizeof(T)));
}

// Location of the pre-collision f_i(x) for pattern PAT: slot and cell.
//   AA_EVEN: (i, x)   AA_ODD: (opp i, x - c_i)   AB: (i, x - c_i)
template <class Cd, int PAT, bool kNT = false, class Planes>
__device__ __forceinline__ void load_cell(const Planes& planes, uint32_t cell,
                                          const Nbr& nb, typename Cd::R (&g)[19],
                                          typename Cd::R inv_s) {
    static_for<19>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int slot = (PAT == PAT_AA_ODD) ? opp_of(i) : i;
        const uint32_t c = (PAT == PAT_AA_EVEN) ? cell : cell + (uint32_t)off_minus<i>(nb);
        const typename Cd::T* p = elem_ptr<const typename Cd::T>(planes, slot, c);
        if constexpr (kNT) g[i] = dec<Cd>(__builtin_nontemporal_load(p), inv_s);
        else g[i] = dec<Cd>(*p, inv_s);
    });
}

// Where the post-collision f*_i(x) goes for pattern PAT (the pattern the step
// reads with): AA_EVEN -> (opp i, x); AA_ODD -> (i, x + c_i); AB -> (i, x) of dst.
template <class Cd, int PAT, bool kNT = false, class Planes>
__device__ __forceinline__ void store_cell(const Planes& planes, uint32_t cell,
                                           const Nbr& nb, const typename Cd::R (&g)[19],
                                           typename Cd::R s) {
    static_for<19>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int slot = (PAT == PAT_AA_EVEN) ? opp_of(i) : i;
        const uint32_t c = (PAT == PAT_AA_ODD) ? cell + (uint32_t)off_minus<opp_of(i)>(nb) : cell;
        typename Cd::T* p = elem_ptr<typename Cd::T>(planes, slot, c);
        if constexpr (kNT) __builtin_nontemporal_store(enc<Cd>(g[i], s), p);
        else *p = enc<Cd>(g[i], s);
    });
}

template <typename R>
__device__ __forceinline__ const CollideConst<R>& collide_const(const LatticeArgs& L) {
    if constexpr (std::is_same_v<R, double>) return L.kd;
    else return L.kf;
}
template <typename R>
__device__ __forceinline__ R scale_of(const LatticeArgs& L) {
    if constexpr (std::is_same_v<R, double>) return L.sigma;
    else return L.sigma_f;
}
template <typename R>
__device__ __forceinline__ R inv_scale_of(const LatticeArgs& L) {
    if constexpr (std::is_same_v<R, double>) return L.inv_sigma;
    else return L.inv_sigma_f;
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
// NT: bit 0 = non-temporal loads, bit 1 = non-temporal stores.
template <class Cd, int PAT, int NT = 0>
__device__ __forceinline__ void step_cell(const LatticeArgs& L, uint32_t cell) {
    using R = typename Cd::R;
    const CellPos p = decode(cell, L);
    const Nbr nb = make_nbr(p, L);
    constexpr bool kS = kScaledCodec<Cd>;
    R g[19];
    load_cell<Cd, PAT, (NT & 1) != 0>(PlaneTable{L.pa}, cell, nb, g,
                                      kS ? R(1) : inv_scale_of<R>(L));
    R Fx, Fy, Fz;
    force_at<R>(L, p, Fx, Fy, Fz);
    if constexpr (kS) {
        const R s = scale_of<R>(L);
        Fx *= s;
        Fy *= s;
        Fz *= s;
    }
    collide<R, true, kS>(g, Fx, Fy, Fz, collide_const<R>(L), inv_scale_of<R>(L));
    // Rebuild the store addresses from here: an empty register barrier on the
    // cell index keeps the compiler from holding 19 precomputed 64-bit store
    // addresses live across the collision (38 VGPRs), so stores use the same
    // scalar-base + 32-bit-offset form as the loads.
    uint32_t cs = cell;
    asm volatile("" : "+v"(cs));
    store_cell<Cd, PAT, (NT & 2) != 0>(PlaneTable{PAT == PAT_AB ? L.pb : L.pa}, cs, nb, g,
                                       kS ? R(1) : scale_of<R>(L));
}

}  // namespace lbm
