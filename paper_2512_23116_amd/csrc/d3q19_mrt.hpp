// d3q19_mrt.hpp — per-cell D3Q19 MRT-Smagorinsky-Guo collision for gfx950.
//
// One thread owns one cell.  The 19x19 moment transform of App. B
// (eq. moment-matrix) is unrolled in registers: each opposite pair (2k, 2k+1)
// contributes only its sum p_k to the even-parity rows (0, 1, 2, 9..15) and
// only its difference d_k to the odd-parity rows (3..8, 16..18), so the forward
// transform is ~95 additions and the inverse M^{-1} = M^T diag(1/n_r) mirrors
// it.  Populations are deviations g = f - w rho0, whose moments are
// M f - rho0 (1, -11, 3, 0, ..., 0); the equilibrium moments of eq. meq_fm are
// printed in exactly that deviation form (row 0 is delta rho).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Velocity set of App. B Fig. d3q19_table (0-based, rest = 18).
__host__ __device__ constexpr int cx_of(int i) {
    constexpr int v[19] = {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0};
    return v[i];
}
__host__ __device__ constexpr int cy_of(int i) {
    constexpr int v[19] = {0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, 0, 0, 0, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int cz_of(int i) {
    constexpr int v[19] = {0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 0};
    return v[i];
}
__host__ __device__ constexpr int opp_of(int i) { return i == 18 ? 18 : (i ^ 1); }
__host__ __device__ constexpr double w_of(int i) {
    return i < 6 ? 1.0 / 18.0 : (i < 18 ? 1.0 / 36.0 : 1.0 / 3.0);
}

// Reciprocal and square root: hardware v_rcp_f32 / v_sqrt_f32 (1 ulp) in FP32,
// IEEE operations in FP64.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }

// Constants of one lattice's collision, in the arithmetic type R.
template <typename R>
struct CollideConst {
    R tau0;      // bare relaxation time
    R c3;        // 3 C (linear form) or 3 C^2; tau_e = tau0 + c3 |S|
    R a_e;       // s_e / (38 rho0): coefficient of m1_neq in S_aa (eq. yu_strain);
                 // 0 in the self-consistent mode
    R b9;        // s_9 / (2 rho0): coefficient of m9_neq in S_xx; s_9 = 1/tau0
                 // (explicit mode) or 1 (self-consistent mode: |S| = |S_1| / tau_e)
    R s_e, s_eps, s_q, s_pi, s_m;
    R rho0;
    R tau0_sq;   // tau0^2
    int32_t self_consistent;   // 1: s_9 = 1/tau_e in eq. yu_strain, closed form
    int32_t pad;
};

// Result of the macroscopic / closure half of the collision.
template <typename R>
struct CellMacro {
    R drho;    // rho - rho0 (exact moment sum, kept for FP64 mass reductions)
    R rho, ux, uy, uz;
    R tau_t;   // tau_e - tau0 = 3 C Delta^2 |S| (or 3 C^2 Delta^2 |S|)
    R snorm2;  // |S|^2 = 2 S:S of the strain that sets tau_e (diagnostics only)
};

// Collide one cell in place.  g: deviation populations (pre-collision in,
// post-collision out).  F: body force at the cell.  kFull = false computes
// only the macroscopic quantities and tau_e (diagnostics) and leaves g as is.
//
// kScaled: g and F come in units of 1/sigma (sigma g, sigma F, with sigma = 1/is
// a power of two: the 16-bit storage scale) and g leaves in the same units, so
// the storage codec needs no multiplications.  Every moment, equilibrium and
// relaxed moment is then exactly sigma times its unscaled value (power-of-two
// scaling commutes with rounding); the four places that need unscaled values
// (rho, 1/rho, |S| -> tau_e, the diagnostics' |S|^2 and delta rho) apply is, so
// the result equals sigma times the unscaled collision's, bit for bit.  The
// returned CellMacro is unscaled either way.
template <typename R, bool kFull, bool kScaled = false>
__device__ __forceinline__ CellMacro<R> collide(R (&g)[19], R Fx, R Fy, R Fz,
                                                const CollideConst<R>& k, R is = R(1)) {
    const R h = R(0.5);
    // pair sums (even rows) and differences (odd rows)
    const R p0 = g[0] + g[1], d0 = g[0] - g[1];
    const R p1 = g[2] + g[3], d1 = g[2] - g[3];
    const R p2 = g[4] + g[5], d2 = g[4] - g[5];
    const R p3 = g[6] + g[7], d3 = g[6] - g[7];
    const R p4 = g[8] + g[9], d4 = g[8] - g[9];
    const R p5 = g[10] + g[11], d5 = g[10] - g[11];
    const R p6 = g[12] + g[13], d6 = g[12] - g[13];
    const R p7 = g[14] + g[15], d7 = g[14] - g[15];
    const R p8 = g[16] + g[17], d8 = g[16] - g[17];
    const R r = g[18];

    // m = M g (eq. moment-matrix), deviation form
    const R sa = p0 + p1 + p2;                 // axis pairs
    const R sd = (p3 + p4) + (p5 + p6) + (p7 + p8);  // diagonal pairs
    const R m0 = sa + sd + r;                  // delta rho
    const R m1 = R(-11) * sa + R(8) * sd - R(30) * r;
    const R m2 = R(-4) * sa + sd + R(12) * r;
    const R jx = d0 + d3 + d4 + d7 + d8;
    const R jy = d1 + d3 - d4 + d5 + d6;
    const R jz = d2 + d5 - d6 + d7 - d8;
    const R m4 = jx - R(5) * d0;
    const R m6 = jy - R(5) * d1;
    const R m8 = jz - R(5) * d2;
    const R v9 = (p3 + p4) + (p7 + p8) - R(2) * (p5 + p6);
    const R m9 = R(2) * p0 - p1 - p2 + v9;
    const R m10 = R(-4) * p0 + R(2) * (p1 + p2) + v9;
    const R v11 = (p3 + p4) - (p7 + p8);
    const R m11 = p1 - p2 + v11;
    const R m12 = R(2) * (p2 - p1) + v11;
    const R m13 = p3 - p4;
    const R m14 = p5 - p6;
    const R m15 = p7 - p8;
    const R m16 = d3 + d4 - d7 - d8;
    const R m17 = d4 - d3 + d5 + d6;
    const R m18 = d6 - d5 + d7 - d8;

    // eq. guo_velocity: rho u = sum f c + F/2 (rux.. and the products below carry
    // the scale of g; u itself is unscaled)
    const R drho = kScaled ? m0 * is : m0;
    const R rho = k.rho0 + drho;
    const R inv_rho = kScaled ? fast_rcp(rho) * is : fast_rcp(rho);
    const R rux = jx + h * Fx, ruy = jy + h * Fy, ruz = jz + h * Fz;
    const R ux = rux * inv_rho, uy = ruy * inv_rho, uz = ruz * inv_rho;
    const R xx = rux * ux, yy = ruy * uy, zz = ruz * uz;   // rho u_a u_a
    const R ru2 = xx + yy + zz;

    // eq. meq_fm: the non-equilibrium parts the strain needs
    const R n1 = m1 - (R(-11) * m0 + R(19) * ru2);
    const R n9 = m9 - (R(2) * xx - yy - zz);
    const R n11 = m11 - (yy - zz);
    const R n13 = m13 - rux * uy;
    const R n14 = m14 - ruy * uz;
    const R n15 = m15 - rux * uz;

    // eq. yu_strain with s_1 = s_e, s_9 = 1/tau0 (explicit mode) or without the
    // s_1 term and s_9 = 1 (self-consistent mode, rescaled below); eq. strain_norm
    const R tr = k.a_e * n1;
    const R Sxx = -tr - k.b9 * n9;
    const R Syy = -tr + h * k.b9 * (n9 - R(3) * n11);
    const R Szz = -tr + h * k.b9 * (n9 + R(3) * n11);
    const R q = R(-3) * k.b9;
    const R Sxy = q * n13, Syz = q * n14, Sxz = q * n15;
    const R S2 = R(2) * (Sxx * Sxx + Syy * Syy + Szz * Szz) +
                 R(4) * (Sxy * Sxy + Sxz * Sxz + Syz * Syz);
    // eq. les_viscosity: tau_e = 1/2 + 3 (nu0 + C Delta^2 |S|) = tau0 + 3 C |S|
    R tau_t = (kScaled ? k.c3 * is : k.c3) * fast_sqrt(S2);
    if (k.self_consistent) {
        // (the empty asm keeps this a uniform branch instead of computing it
        // always and selecting, so the default mode pays nothing for it)
        asm volatile("");
        // |S| = X / tau_e with X = |S_1| (computed above with s_9 = 1, no m1
        // term): tau_e^2 - tau0 tau_e - c3 X = 0.  Its positive root, as the
        // increment over tau0 without cancellation:
        // tau_e - tau0 = 2 c3 X / (tau0 + sqrt(tau0^2 + 4 c3 X)).
        tau_t = R(2) * tau_t * fast_rcp(k.tau0 + fast_sqrt(k.tau0_sq + R(4) * tau_t));
    }
    const R tau_e = k.tau0 + tau_t;
    // |S|^2: S2 itself, or (|S_1| / tau_e)^2 in the self-consistent mode.  Only the
    // diagnostics read it; the step kernels drop it.
    const R S2u = kScaled ? S2 * (is * is) : S2;
    const R snorm2 = k.self_consistent ? S2u * fast_rcp(tau_e * tau_e) : S2u;

    CellMacro<R> out{drho, rho, ux, uy, uz, tau_t, snorm2};
    if constexpr (!kFull) {
        return out;
    } else {
        const R s_nu = fast_rcp(tau_e);
        // eq. meq_fm: force moments
        const R X = ux * Fx, Y = uy * Fy, Z = uz * Fz;
        const R uF = X + Y + Z;
        const R P = R(2) * X - Y - Z;
        const R Qw = Y - Z;
        const R third2 = R(2) / R(3);

        // eq. mrt_les_guo in moment space: m* = m - S (m - m_eq) + (I - S/2) F_m,
        // each row pre-divided by its norm n_r = (M M^T)_rr
        const R ge = R(1) - h * k.s_e, geps = R(1) - h * k.s_eps, gq = R(1) - h * k.s_q;
        const R gpi = R(1) - h * k.s_pi, gnu = R(1) - h * s_nu;
        const R t0 = m0 * R(1.0 / 19.0);
        const R t1 = (m1 - k.s_e * n1 + ge * R(38) * uF) * R(1.0 / 2394.0);
        const R t2 = (m2 - k.s_eps * (m2 + R(475.0 / 63.0) * ru2) + geps * R(-11) * uF) *
                     R(1.0 / 252.0);
        const R t3 = (rux + h * Fx) * R(0.1);
        const R t5 = (ruy + h * Fy) * R(0.1);
        const R t7 = (ruz + h * Fz) * R(0.1);
        const R t4 = (m4 - k.s_q * (m4 + third2 * rux) - gq * third2 * Fx) * R(1.0 / 40.0);
        const R t6 = (m6 - k.s_q * (m6 + third2 * ruy) - gq * third2 * Fy) * R(1.0 / 40.0);
        const R t8 = (m8 - k.s_q * (m8 + third2 * ruz) - gq * third2 * Fz) * R(1.0 / 40.0);
        const R t9 = (m9 - s_nu * n9 + gnu * R(2) * P) * R(1.0 / 36.0);
        const R t10 = ((R(1) - k.s_pi) * m10 - gpi * P) * R(1.0 / 72.0);
        const R t11 = (m11 - s_nu * n11 + gnu * R(2) * Qw) * R(1.0 / 12.0);
        const R t12 = ((R(1) - k.s_pi) * m12 - gpi * Qw) * R(1.0 / 24.0);
        const R t13 = (m13 - s_nu * n13 + gnu * (ux * Fy + uy * Fx)) * R(0.25);
        const R t14 = (m14 - s_nu * n14 + gnu * (uy * Fz + uz * Fy)) * R(0.25);
        const R t15 = (m15 - s_nu * n15 + gnu * (ux * Fz + uz * Fx)) * R(0.25);
        const R sm = (R(1) - k.s_m) * R(0.125);
        const R t16 = sm * m16, t17 = sm * m17, t18 = sm * m18;

        // g* = M^T (m* / n): even part E_k, odd part O_k per pair
        const R ea = t0 - R(11) * t1 - R(4) * t2;
        const R e0 = ea + R(2) * t9 - R(4) * t10;
        const R eyz = ea - t9 + R(2) * t10;
        const R e1 = eyz + t11 - R(2) * t12;
        const R e2 = eyz - t11 + R(2) * t12;
        const R o0 = t3 - R(4) * t4;
        const R o1 = t5 - R(4) * t6;
        const R o2 = t7 - R(4) * t8;
        const R ed = t0 + R(8) * t1 + t2;
        const R exy = ed + t9 + t10 + t11 + t12;
        const R eyz2 = ed - R(2) * (t9 + t10);
        const R exz = ed + t9 + t10 - t11 - t12;
        const R e3 = exy + t13, e4 = exy - t13;
        const R e5 = eyz2 + t14, e6 = eyz2 - t14;
        const R e7 = exz + t15, e8 = exz - t15;
        const R ax = t3 + t4, ay = t5 + t6, az = t7 + t8;
        const R o3 = ax + ay + t16 - t17;
        const R o4 = ax - ay + t16 + t17;
        const R o5 = ay + az + t17 - t18;
        const R o6 = ay - az + t17 + t18;
        const R o7 = ax + az - t16 + t18;
        const R o8 = ax - az - t16 - t18;

        g[0] = e0 + o0;  g[1] = e0 - o0;
        g[2] = e1 + o1;  g[3] = e1 - o1;
        g[4] = e2 + o2;  g[5] = e2 - o2;
        g[6] = e3 + o3;  g[7] = e3 - o3;
        g[8] = e4 + o4;  g[9] = e4 - o4;
        g[10] = e5 + o5; g[11] = e5 - o5;
        g[12] = e6 + o6; g[13] = e6 - o6;
        g[14] = e7 + o7; g[15] = e7 - o7;
        g[16] = e8 + o8; g[17] = e8 - o8;
        g[18] = t0 - R(30) * t1 + R(12) * t2;
        return out;
    }
}

}  // namespace lbm
