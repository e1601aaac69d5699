// lbm_kernels.hip — HIP kernels of the D3Q19 MRT-Smagorinsky LES hot path (gfx950).
//
// Layout in HBM: structure of arrays, one plane per velocity direction,
// state[i * plane + c] with c = x + nx (y + ny z) (x fastest), holding the
// deviation g = f - w_i rho0 in the storage type T (double, float, or a
// 16-bit float of sigma*g).  A plane is padded to a multiple of 128 elements
// so every plane starts 256-byte aligned.
//
// One thread owns one cell per launch; a 64-lane wavefront therefore reads and
// writes 64 consecutive cells of each plane.  Kernel shapes:
//   k_step      the fused stream-and-collide step (eq. mrt_les_guo): 19 loads,
//               collision in registers, 19 stores; AA even / AA odd / A-B pull
//   k_diag      per-cell tau_e, K_t, rho, u of the current state and FP64
//               power sums, reduced per block in a fixed order
//   k_moments, k_ktfield, k_gather_plane, k_scatter_plane, k_sample, k_init,
//   k_rowtab, k_xtab   set-up and observation kernels (not on the hot loop)
#include "lbm_device.hpp"

namespace lbm {

// ------------------------------------------------------------ the step ---
template <class Cd, int PAT, int NT>
__global__ __launch_bounds__(256) void k_step(LatticeArgs L) {
    const uint32_t cell = block_id(L) * 256u + threadIdx.x;
    if (cell >= L.ncell) return;
    step_cell<Cd, PAT, NT>(L, cell);
}

// Free streaming: the step's loads and stores with the identity for the
// collision (no force, no arithmetic beyond the storage codec, exact for every
// format).  Same block order, addressing and address barrier as k_step, so its
// time is the ceiling of the step's access pattern.
template <class Cd, int PAT>
__global__ __launch_bounds__(256) void k_stream(LatticeArgs L) {
    using R = typename Cd::R;
    const uint32_t cell = block_id(L) * 256u + threadIdx.x;
    if (cell >= L.ncell) return;
    const CellPos p = decode(cell, L);
    const Nbr nb = make_nbr(p, L);
    R g[19];
    load_cell<Cd, PAT>(PlaneTable{L.pa}, cell, nb, g, R(1));
    uint32_t cs = cell;
    asm volatile("" : "+v"(cs));
    store_cell<Cd, PAT>(PlaneTable{PAT == PAT_AB ? L.pb : L.pa}, cs, nb, g, R(1));
}

// ----------------------------------------------------- diagnostics ---
// Per-block FP64 partials: [0..3] sum of tau_t^p (p = 1..4, tau_t = tau_e - tau0),
// [4] min tau_t, [5] max tau_t, [6] sum delta rho, [7..9] sum rho u,
// [10] sum u.u/2, [11] sum rho u.u/2, [12] non-finite cells, [13] sum |S|^2,
// [14] sum tau_t |S|^2 (3 nu_t |S|^2), [15] sum F.u (power injected, eq. energy_balance),
// [16..18] sum u_i, [19..24] sum u_i u_j (xx, yy, zz, xy, xz, yz; Reynolds stresses).
constexpr int kDiagUsed = 25;
static_assert(kDiagUsed <= kDiagSlots, "diagnostic partials overflow their slots");

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <class Cd, int PAT>
__global__ __launch_bounds__(256) void k_diag(LatticeArgs L, double* partials) {
    using R = typename Cd::R;
    double acc[kDiagUsed];
#pragma unroll
    for (int j = 0; j < kDiagUsed; ++j) acc[j] = 0.0;
    acc[4] = INFINITY;
    acc[5] = -INFINITY;
    const CollideConst<R>& k = collide_const<R>(L);
    for (uint32_t cell = blockIdx.x * 256u + threadIdx.x; cell < L.ncell;
         cell += gridDim.x * 256u) {
        const CellPos p = decode(cell, L);
        const Nbr nb = make_nbr(p, L);
        R g[19];
        load_cell<Cd, PAT>(PlaneTable{L.pa}, cell, nb, g, inv_scale_of<R>(L));
        bool finite = true;
#pragma unroll
        for (int i = 0; i < 19; ++i) finite = finite && isfinite(g[i]);
        R Fx, Fy, Fz;
        force_at<R>(L, p, Fx, Fy, Fz);
        const CellMacro<R> m = collide<R, false>(g, Fx, Fy, Fz, k);
        const double tt = (double)m.tau_t;   // tau_e - tau0 = c3 |S| >= 0
        finite = finite && isfinite(tt);
        if (!finite) {
            acc[12] += 1.0;
            continue;
        }
        const double drho = (double)m.drho;
        const double rho = (double)k.rho0 + drho;
        const double ux = (double)m.ux, uy = (double)m.uy, uz = (double)m.uz;
        const double t2 = tt * tt;
        acc[0] += tt; acc[1] += t2; acc[2] += t2 * tt; acc[3] += t2 * t2;
        acc[4] = fmin(acc[4], tt); acc[5] = fmax(acc[5], tt);
        acc[6] += drho;
        acc[7] += rho * ux; acc[8] += rho * uy; acc[9] += rho * uz;
        const double uu = 0.5 * (ux * ux + uy * uy + uz * uz);
        acc[10] += uu; acc[11] += rho * uu;
        const double s2 = (double)m.snorm2;
        acc[13] += s2; acc[14] += tt * s2;
        acc[15] += (double)Fx * ux + (double)Fy * uy + (double)Fz * uz;
        acc[16] += ux; acc[17] += uy; acc[18] += uz;
        acc[19] += ux * ux; acc[20] += uy * uy; acc[21] += uz * uz;
        acc[22] += ux * uy; acc[23] += ux * uz; acc[24] += uy * uz;
    }
    __shared__ double red[4][kDiagUsed];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kDiagUsed; ++j) {
        double v = acc[j];
        v = (j == 4) ? wave_min(v) : ((j == 5) ? wave_max(v) : wave_sum(v));
        if (lane == 0) red[wv][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < kDiagUsed) {
        const int j = threadIdx.x;
        double v = red[0][j];
        for (int w = 1; w < 4; ++w)
            v = (j == 4) ? fmin(v, red[w][j]) : ((j == 5) ? fmax(v, red[w][j]) : v + red[w][j]);
        partials[(uint64_t)blockIdx.x * kDiagSlots + j] = v;
    }
}

// Reduce the per-block partials in a fixed order into result[0..kDiagUsed):
// block j reduces slot j (thread t folds blocks t, t + 256, ..., then a fixed
// tree over the 256 threads).
__global__ __launch_bounds__(256) void k_diag_final(const double* partials, int nblocks,
                                                    double* result) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double v = (j == 4) ? INFINITY : ((j == 5) ? -INFINITY : 0.0);
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        const double x = partials[(uint64_t)b * kDiagSlots + j];
        v = (j == 4) ? fmin(v, x) : ((j == 5) ? fmax(v, x) : v + x);
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double a = red[threadIdx.x], b = red[threadIdx.x + s];
            red[threadIdx.x] = (j == 4) ? fmin(a, b) : ((j == 5) ? fmax(a, b) : a + b);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) result[j] = red[0];
}

// ------------------------------------------------------ observation ---
template <class Cd, int PAT>
__global__ __launch_bounds__(256) void k_moments(LatticeArgs L, double* rho, double* u) {
    using R = typename Cd::R;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= L.ncell) return;
    const CellPos p = decode(cell, L);
    const Nbr nb = make_nbr(p, L);
    R g[19];
    load_cell<Cd, PAT>(PlaneTable{L.pa}, cell, nb, g, inv_scale_of<R>(L));
    R Fx, Fy, Fz;
    force_at<R>(L, p, Fx, Fy, Fz);
    const CellMacro<R> m = collide<R, false>(g, Fx, Fy, Fz, collide_const<R>(L));
    if (rho) rho[cell] = L.rho0 + (double)m.drho;
    if (u) {
        u[cell] = (double)m.ux;
        u[(uint64_t)L.ncell + cell] = (double)m.uy;
        u[2 * (uint64_t)L.ncell + cell] = (double)m.uz;
    }
}

// theta = tau_e - 1/2 of one cell of the current state (eq. les_viscosity), in
// FP64 from the kernel's own tau_t: the value behind the K_t field and the
// theta histogram.
template <class Cd, int PAT>
__device__ __forceinline__ double cell_theta(const LatticeArgs& L, uint32_t cell) {
    using R = typename Cd::R;
    const CellPos p = decode(cell, L);
    const Nbr nb = make_nbr(p, L);
    R g[19];
    load_cell<Cd, PAT>(PlaneTable{L.pa}, cell, nb, g, inv_scale_of<R>(L));
    R Fx, Fy, Fz;
    force_at<R>(L, p, Fx, Fy, Fz);
    const CellMacro<R> m = collide<R, false>(g, Fx, Fy, Fz, collide_const<R>(L));
    return (L.tau0 - 0.5) + (double)m.tau_t;
}

template <class Cd, int PAT>
__global__ __launch_bounds__(256) void k_ktfield(LatticeArgs L, float* kt) {
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= L.ncell) return;
    const double theta = cell_theta<Cd, PAT>(L, cell);
    kt[cell] = (float)(1.7320508075688772 * theta);   // K_t = sqrt(3) theta, ell = delta_x
}

// K_t of the cells of plane z: kt[x + nx y].
template <class Cd, int PAT>
__global__ __launch_bounds__(256) void k_ktslice(LatticeArgs L, uint32_t z, float* kt) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= L.nxy) return;
    const double theta = cell_theta<Cd, PAT>(L, i + L.nxy * z);
    kt[i] = (float)(1.7320508075688772 * theta);
}

// Fixed-bin histogram of theta: counts[0] below lo, counts[1 + b] for
// b = floor((theta - lo) * inv_w) in 0..nbins-1, counts[nbins + 1] at or above
// the top edge, counts[nbins + 2] non-finite.  Per-block LDS counts, then one
// 64-bit integer atomic per non-empty bin: the totals are exact.
template <class Cd, int PAT>
__global__ __launch_bounds__(256) void k_theta_hist(LatticeArgs L, double lo, double inv_w,
                                                    int nbins, unsigned long long* counts) {
    extern __shared__ unsigned int hist[];
    for (int k = threadIdx.x; k < nbins + 3; k += 256) hist[k] = 0u;
    __syncthreads();
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell < L.ncell) {
        const double theta = cell_theta<Cd, PAT>(L, cell);
        int b;
        if (!isfinite(theta)) {
            b = nbins + 2;
        } else if (theta < lo) {
            b = 0;
        } else {
            const double q = floor((theta - lo) * inv_w);
            b = q >= (double)nbins ? nbins + 1 : 1 + (int)q;
        }
        atomicAdd(&hist[b], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nbins + 3; k += 256)
        if (hist[k]) atomicAdd(&counts[k], (unsigned long long)hist[k]);
}

template <class Cd>
__global__ __launch_bounds__(256) void k_gather_plane(LatticeArgs L, int pat, int i, double* out) {
    using T = typename Cd::T;
    using R = typename Cd::R;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= L.ncell) return;
    const CellPos p = decode(cell, L);
    const Nbr nb = make_nbr(p, L);
    const T v = ((const T*)L.a)[canon_index(pat, i, cell, nb, L.plane)];
    out[cell] = (double)dec<Cd>(v, inv_scale_of<R>(L)) + w_of(i) * L.rho0;
}

template <class Cd>
__global__ __launch_bounds__(256) void k_scatter_plane(LatticeArgs L, int pat, int i,
                                                       const double* in) {
    using T = typename Cd::T;
    using R = typename Cd::R;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= L.ncell) return;
    const CellPos p = decode(cell, L);
    const Nbr nb = make_nbr(p, L);
    const R g = (R)(in[cell] - w_of(i) * L.rho0);
    ((T*)L.a)[canon_index(pat, i, cell, nb, L.plane)] = enc<Cd>(g, scale_of<R>(L));
}

template <class Cd>
__global__ __launch_bounds__(256) void k_sample(LatticeArgs L, int pat, const int64_t* cells,
                                                int64_t n, double* out) {
    using T = typename Cd::T;
    using R = typename Cd::R;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * 19) return;
    const int64_t j = t / 19;
    const int i = (int)(t - j * 19);
    const uint32_t cell = (uint32_t)cells[j];
    const CellPos p = decode(cell, L);
    const Nbr nb = make_nbr(p, L);
    const T v = ((const T*)L.a)[canon_index(pat, i, cell, nb, L.plane)];
    out[t] = (double)dec<Cd>(v, inv_scale_of<R>(L)) + w_of(i) * L.rho0;
}

// --------------------------------------------------------------- set-up ---
__device__ __forceinline__ uint64_t splitmix64(uint64_t v) {
    uint64_t z = v + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// f(x, 0) = f_eq(rho0, u0(x)) of App. A eq. feq, stored as the deviation
// w rho0 (3 c.u + 4.5 (c.u)^2 - 1.5 u.u) at the pattern's canonical slots.
template <class Cd>
__global__ __launch_bounds__(256) void k_init(LatticeArgs L, int pat, int kind, double amp,
                                              uint64_t key) {
    using T = typename Cd::T;
    using R = typename Cd::R;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= L.ncell) return;
    const CellPos p = decode(cell, L);
    const Nbr nb = make_nbr(p, L);
    const double twopi = 6.283185307179586;
    const double X = twopi * p.x / L.nx, Y = twopi * p.y / L.ny, Z = twopi * p.z / L.nz;
    double u[3] = {0.0, 0.0, 0.0};
    if (kind == LBM_INIT_TGV3D) {
        u[0] = amp * sin(X) * cos(Y) * cos(Z);
        u[1] = -amp * cos(X) * sin(Y) * cos(Z);
    } else if (kind == LBM_INIT_TGV2D) {
        u[0] = amp * sin(X) * cos(Y);
        u[1] = -amp * cos(X) * sin(Y);
    } else if (kind == LBM_INIT_SHEAR) {
        u[0] = amp * sin(Y);
    } else if (kind == LBM_INIT_NOISE) {
        for (int a = 0; a < 3; ++a) {
            const uint64_t hsh = splitmix64(key ^ (3ull * cell + (uint64_t)a));
            const double U = (double)(hsh >> 11) * 0x1.0p-53;
            u[a] = amp * (2.0 * U - 1.0);
        }
    }
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < 19; ++i) {
        const double cu = cx_of(i) * u[0] + cy_of(i) * u[1] + cz_of(i) * u[2];
        const double g = w_of(i) * L.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        ((T*)L.a)[canon_index(pat, i, cell, nb, L.plane)] = enc<Cd>((R)g, scale_of<R>(L));
    }
}

// Per-(y,z) force coefficients: every mode amp sin(alpha + 2 pi kx x/nx) with
// alpha = 2 pi (ky y/ny + kz z/nz) + phase is split by the angle-sum identity
// into the constant (kx = 0) or the sin/cos(2 pi |kx| x/nx) coefficients.
template <typename R>
__global__ __launch_bounds__(256) void k_rowtab(uint32_t ny, uint32_t nz,
                                                const lbm_force_mode* modes, int nm, R* rowc) {
    const uint32_t row = blockIdx.x * 256u + threadIdx.x;
    if (row >= ny * nz) return;
    const uint32_t z = row / ny, y = row - z * ny;
    double c[15];
    for (int j = 0; j < 15; ++j) c[j] = 0.0;
    for (int m = 0; m < nm; ++m) {
        const lbm_force_mode md = modes[m];
        const double alpha = 2.0 * M_PI * ((double)md.k[1] * y / ny + (double)md.k[2] * z / nz) +
                             md.phase;
        const double sa = sin(alpha), ca = cos(alpha);
        const int kx = md.k[0];
        if (kx == 0) {
            for (int a = 0; a < 3; ++a) c[a] += md.amp[a] * sa;
        } else {
            const int base = (kx == 1 || kx == -1) ? 3 : 9;
            const double sg = kx > 0 ? 1.0 : -1.0;
            for (int a = 0; a < 3; ++a) {
                c[base + a] += sg * md.amp[a] * ca;    // coefficient of sin(2 pi |kx| x/nx)
                c[base + 3 + a] += md.amp[a] * sa;     // coefficient of cos(2 pi |kx| x/nx)
            }
        }
    }
    for (int j = 0; j < 15; ++j) rowc[(uint64_t)row * 16 + j] = (R)c[j];
    rowc[(uint64_t)row * 16 + 15] = (R)0;
}

template <typename R>
__global__ __launch_bounds__(256) void k_xtab(uint32_t nx, R* xtab) {
    const uint32_t x = blockIdx.x * 256u + threadIdx.x;
    if (x >= nx) return;
    const double a1 = 2.0 * M_PI * ((double)x / nx), a2 = 2.0 * M_PI * (2.0 * x / nx);
    xtab[4 * x + 0] = (R)sin(a1);
    xtab[4 * x + 1] = (R)cos(a1);
    xtab[4 * x + 2] = (R)sin(a2);
    xtab[4 * x + 3] = (R)cos(a2);
}

// ------------------------------------------------------------ launchers ---
template <class Cd, typename Fn>
hipError_t dispatch_pat(int pat, Fn&& fn) {
    switch (pat) {
        case PAT_AA_EVEN: return fn(Cd{}, std::integral_constant<int, PAT_AA_EVEN>{});
        case PAT_AA_ODD: return fn(Cd{}, std::integral_constant<int, PAT_AA_ODD>{});
        case PAT_AB: return fn(Cd{}, std::integral_constant<int, PAT_AB>{});
    }
    return hipErrorInvalidValue;
}

template <typename Fn>
hipError_t dispatch(int precision, int pat, Fn&& fn) {
    switch (precision) {
        case LBM_FP64: return dispatch_pat<CdF64>(pat, fn);
        case LBM_FP32: return dispatch_pat<CdF32>(pat, fn);
        case LBM_FP16_DEV: return dispatch_pat<CdF16>(pat, fn);
        case LBM_BF16_DEV: return dispatch_pat<CdBF16>(pat, fn);
    }
    return hipErrorInvalidValue;
}

static inline dim3 grid_for(uint64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_tables(int precision, const LatticeArgs& L, const lbm_force_mode* d_modes,
                         int n_modes, hipStream_t s) {
    if (precision == LBM_FP64) {
        hipLaunchKernelGGL(k_rowtab<double>, grid_for((uint64_t)L.ny * L.nz), dim3(256), 0, s,
                           L.ny, L.nz, d_modes, n_modes, (double*)L.rowc);
        hipLaunchKernelGGL(k_xtab<double>, grid_for(L.nx), dim3(256), 0, s, L.nx,
                           (double*)L.xtab);
    } else {
        hipLaunchKernelGGL(k_rowtab<float>, grid_for((uint64_t)L.ny * L.nz), dim3(256), 0, s,
                           L.ny, L.nz, d_modes, n_modes, (float*)L.rowc);
        hipLaunchKernelGGL(k_xtab<float>, grid_for(L.nx), dim3(256), 0, s, L.nx,
                           (float*)L.xtab);
    }
    return hipGetLastError();
}

hipError_t launch_init(int precision, int pat, const LatticeArgs& L, int kind, double amp,
                       uint64_t seed, hipStream_t s) {
    // the host hashes the seed once, exactly as the per-cell hash does
    uint64_t z = seed + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    const uint64_t key = z ^ (z >> 31);
    return dispatch(precision, PAT_AA_EVEN, [&](auto cd, auto) {
        using Cd = decltype(cd);
        hipLaunchKernelGGL(k_init<Cd>, grid_for(L.ncell), dim3(256), 0, s, L, pat, kind, amp, key);
        return hipGetLastError();
    });
}

hipError_t launch_step(int precision, int pat, const LatticeArgs& L, hipStream_t s) {
    return dispatch(precision, pat, [&](auto cd, auto pt) {
        using Cd = decltype(cd);
        constexpr int P = decltype(pt)::value;
        if (L.nt_mode & 2)
            hipLaunchKernelGGL((k_step<Cd, P, 2>), grid_for(L.ncell), dim3(256), 0, s, L);
        else
            hipLaunchKernelGGL((k_step<Cd, P, 0>), grid_for(L.ncell), dim3(256), 0, s, L);
        return hipGetLastError();
    });
}

hipError_t launch_stream(int precision, int pat, const LatticeArgs& L, hipStream_t s) {
    return dispatch(precision, pat, [&](auto cd, auto pt) {
        using Cd = decltype(cd);
        constexpr int P = decltype(pt)::value;
        hipLaunchKernelGGL((k_stream<Cd, P>), grid_for(L.ncell), dim3(256), 0, s, L);
        return hipGetLastError();
    });
}

hipError_t launch_diag(int precision, int pat, const LatticeArgs& L, double* partials,
                       int nblocks, double* result, hipStream_t s) {
    hipError_t e = dispatch(precision, pat, [&](auto cd, auto pt) {
        using Cd = decltype(cd);
        constexpr int P = decltype(pt)::value;
        hipLaunchKernelGGL((k_diag<Cd, P>), dim3(nblocks), dim3(256), 0, s, L, partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_final, dim3(kDiagUsed), dim3(256), 0, s, (const double*)partials,
                       nblocks, result);
    return hipGetLastError();
}

hipError_t launch_moments(int precision, int pat, const LatticeArgs& L, double* rho, double* u,
                          hipStream_t s) {
    return dispatch(precision, pat, [&](auto cd, auto pt) {
        using Cd = decltype(cd);
        constexpr int P = decltype(pt)::value;
        hipLaunchKernelGGL((k_moments<Cd, P>), grid_for(L.ncell), dim3(256), 0, s, L, rho, u);
        return hipGetLastError();
    });
}

hipError_t launch_ktfield(int precision, int pat, const LatticeArgs& L, float* kt, hipStream_t s) {
    return dispatch(precision, pat, [&](auto cd, auto pt) {
        using Cd = decltype(cd);
        constexpr int P = decltype(pt)::value;
        hipLaunchKernelGGL((k_ktfield<Cd, P>), grid_for(L.ncell), dim3(256), 0, s, L, kt);
        return hipGetLastError();
    });
}

hipError_t launch_ktslice(int precision, int pat, const LatticeArgs& L, uint32_t z, float* kt,
                          hipStream_t s) {
    return dispatch(precision, pat, [&](auto cd, auto pt) {
        using Cd = decltype(cd);
        constexpr int P = decltype(pt)::value;
        hipLaunchKernelGGL((k_ktslice<Cd, P>), grid_for(L.nxy), dim3(256), 0, s, L, z, kt);
        return hipGetLastError();
    });
}

hipError_t launch_theta_hist(int precision, int pat, const LatticeArgs& L, double lo, double inv_w,
                             int nbins, unsigned long long* counts, hipStream_t s) {
    return dispatch(precision, pat, [&](auto cd, auto pt) {
        using Cd = decltype(cd);
        constexpr int P = decltype(pt)::value;
        hipLaunchKernelGGL((k_theta_hist<Cd, P>), grid_for(L.ncell), dim3(256),
                           (size_t)(nbins + 3) * sizeof(unsigned int), s, L, lo, inv_w, nbins,
                           counts);
        return hipGetLastError();
    });
}

hipError_t launch_gather_plane(int precision, int pat, const LatticeArgs& L, int i, double* out,
                               hipStream_t s) {
    return dispatch(precision, PAT_AA_EVEN, [&](auto cd, auto) {
        using Cd = decltype(cd);
        hipLaunchKernelGGL(k_gather_plane<Cd>, grid_for(L.ncell), dim3(256), 0, s, L, pat, i, out);
        return hipGetLastError();
    });
}

hipError_t launch_scatter_plane(int precision, int pat, const LatticeArgs& L, int i,
                                const double* in, hipStream_t s) {
    return dispatch(precision, PAT_AA_EVEN, [&](auto cd, auto) {
        using Cd = decltype(cd);
        hipLaunchKernelGGL(k_scatter_plane<Cd>, grid_for(L.ncell), dim3(256), 0, s, L, pat, i, in);
        return hipGetLastError();
    });
}

hipError_t launch_sample(int precision, int pat, const LatticeArgs& L, const int64_t* cells,
                         int64_t n, double* out, hipStream_t s) {
    return dispatch(precision, PAT_AA_EVEN, [&](auto cd, auto) {
        using Cd = decltype(cd);
        hipLaunchKernelGGL(k_sample<Cd>, grid_for((uint64_t)n * 19), dim3(256), 0, s, L, pat,
                           cells, n, out);
        return hipGetLastError();
    });
}

}  // namespace lbm
