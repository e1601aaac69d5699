// lbm_init_field.hip — the initial state from a velocity field held on the
// device: f(x, 0) = f_eq(rho(x), u(x)) of App. A eq. feq, for a run that starts
// from a given flow (one interpolated from a coarser lattice, say) instead of
// one of lbm_init_seeded's analytic fields.  Stored like those, as the
// deviation f - w_i rho0 at the pattern's canonical slots.
#include <string>

#include "lbm_device.hpp"

namespace lbm {
namespace {

// g_i = f_eq,i - w_i rho0 = w_i (rho - rho0 + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)).
template <class Cd>
__global__ __launch_bounds__(256) void k_init_velocity(LatticeArgs L, int pat, const double* u,
                                                       const double* rho) {
    using T = typename Cd::T;
    using R = typename Cd::R;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= L.ncell) return;
    const CellPos p = decode(cell, L);
    const Nbr nb = make_nbr(p, L);
    const uint64_t n = L.ncell;
    const double ux = u[cell], uy = u[n + cell], uz = u[2 * n + cell];
    const double r = rho ? rho[cell] : L.rho0;
    const double uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < 19; ++i) {
        const double cu = cx_of(i) * ux + cy_of(i) * uy + cz_of(i) * uz;
        const double g = w_of(i) * ((r - L.rho0) + r * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
        ((T*)L.a)[canon_index(pat, i, cell, nb, L.plane)] = enc<Cd>((R)g, scale_of<R>(L));
    }
}

lbm_status set_err(lbm_handle* h, lbm_status st, const std::string& m) {
    h->err = m;
    return st;
}

// Whether p is memory of device `dev` (device or managed allocation).
bool on_device(const void* p, int dev) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();   // host memory unknown to HIP: clear the error
        return false;
    }
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == dev;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_init_velocity(lbm_handle* h, const double* u, const double* rho) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (!u) return set_err(h, LBM_ERR_INVALID_ARG, "u is NULL");
    if (!on_device(u, h->device) || (rho && !on_device(rho, h->device)))
        return set_err(h, LBM_ERR_INVALID_ARG,
                       "u and rho must be device memory of the lattice's device");
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != h->device) e = hipSetDevice(h->device);
    if (e != hipSuccess) return set_err(h, LBM_ERR_DEVICE, "hipSetDevice failed");
    h->steps = 0;
    h->cur = 0;
    const int pat = h->cfg.streaming == LBM_STREAM_AB ? PAT_AB : PAT_AA_EVEN;
    const LatticeArgs L = current_args(h);
    const dim3 grid((unsigned)((L.ncell + 255) / 256));
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, dim3(256), 0, h->stream, L, pat, u, rho);
    };
    switch (h->cfg.precision) {
        case LBM_FP64: launch(k_init_velocity<CdF64>); break;
        case LBM_FP32: launch(k_init_velocity<CdF32>); break;
        case LBM_FP16_DEV: launch(k_init_velocity<CdF16>); break;
        case LBM_BF16_DEV: launch(k_init_velocity<CdBF16>); break;
        default: e = hipErrorInvalidValue;
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (prev >= 0 && prev != h->device) (void)hipSetDevice(prev);
    if (e != hipSuccess)
        return set_err(h, LBM_ERR_DEVICE, std::string("init kernel: ") + hipGetErrorString(e));
    h->initialized = true;
    return LBM_OK;
}
