// lbm_analysis.hip — on-device turbulence diagnostics of the current state:
// the shell-binned kinetic-energy spectrum (Sec. 2.2, eq. integral_length_scale
// with the squared modulus), longitudinal structure functions / flatness
// (Sec. 5.3), and the turbulence scales of Sec. 2.2 (integral scale,
// dissipation, Kolmogorov and Taylor scales, energy balance terms).  All start
// from the velocity with the half-force shift (eq. guo_velocity) that
// lbm_moments returns, computed on the device in FP64.
#include <hipfft/hipfft.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>
#include <vector>

#include "lbm_device.hpp"
#include "lbm_observe.hpp"

namespace lbm {

constexpr int kAnaBlocks = 1024;

// The binning kernels below sum in a fixed order, so that a spectrum is the
// same bit for bit on every call: each wave of a block takes whole rows (fixed
// ky, kz) of the R2C output c[nz][ny][nx/2+1] in turn, 64 values of kx at a
// time, and adds into a histogram of its own in LDS in program order; the block
// then adds its waves' histograms in wave order (and k_sum_rows its blocks'
// partial sums in block order).  A block has 1 to 4 waves, as many as let their
// histograms fit 64 KB of LDS.

// Per-block partial sums of 1/2 w |c|^2 / n^2 over the shells 0..kmax, |c|^2
// summed over ncomp transforms stored cstride apart (the velocity components);
// w = 2 for the kx > 0 modes that stand for a conjugate pair.  Along a row the shell index
// never decreases with kx, so equal shells are contiguous runs of lanes: a
// segmented scan over the 64 lanes sums each run, and the run's last lane adds
// that sum to the wave's histogram (one lane per shell, no two lanes on one bin).
__global__ __launch_bounds__(256) void k_shell_bin(const hipfftDoubleComplex* c, uint64_t cstride,
                                                   int ncomp, uint32_t nx, uint32_t ny,
                                                   uint32_t nz, int kmax, double inv_n2,
                                                   double* partials) {
    extern __shared__ double hist[];   // [waves][kmax + 1]
    const int nb = kmax + 1, waves = (int)(blockDim.x >> 6);
    for (int k = threadIdx.x; k < waves * nb; k += blockDim.x) hist[k] = 0.0;
    __syncthreads();
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    double* wh = hist + wave * nb;
    const uint32_t hx = nx / 2 + 1;
    const uint64_t rows = (uint64_t)ny * nz;
    for (uint64_t row = (uint64_t)blockIdx.x * waves + wave; row < rows;
         row += (uint64_t)gridDim.x * waves) {
        const uint32_t iy = (uint32_t)(row % ny), iz = (uint32_t)(row / ny);
        const double ky = iy <= ny / 2 ? (double)iy : (double)iy - ny;
        const double kz = iz <= nz / 2 ? (double)iz : (double)iz - nz;
        const double kyz2 = ky * ky + kz * kz;
        const hipfftDoubleComplex* crow = c + row * hx;
        for (uint32_t x0 = 0; x0 < hx; x0 += 64) {
            const uint32_t ix = x0 + (uint32_t)lane;
            const bool in = ix < hx;
            const double kx = (double)ix;
            const int shell = in ? (int)floor(sqrt(kx * kx + kyz2) + 0.5) : INT_MAX;
            // the row's shells only grow: once lane 0 is past kmax, so is the rest
            if (__shfl(shell, 0, 64) > kmax) break;
            double v = 0.0;
            if (in && shell <= kmax) {
                const double w = (ix == 0 || (nx % 2 == 0 && ix == nx / 2)) ? 1.0 : 2.0;
                double e = 0.0;   // |u_hat|^2 summed over the ncomp components
                for (int q = 0; q < ncomp; ++q) {
                    const hipfftDoubleComplex z = crow[(uint64_t)q * cstride + ix];
                    e += z.x * z.x + z.y * z.y;
                }
                v = 0.5 * w * e * inv_n2;
            }
            for (int d = 1; d < 64; d <<= 1) {   // segmented inclusive scan over the runs
                const double vu = __shfl_up(v, d, 64);
                const int su = __shfl_up(shell, d, 64);
                if (lane >= d && su == shell) v += vu;
            }
            const int next = __shfl_down(shell, 1, 64);
            if (in && shell <= kmax && (lane == 63 || next != shell)) wh[shell] += v;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        double s = hist[k];
        for (int w = 1; w < waves; ++w) s += hist[w * nb + k];
        partials[(uint64_t)blockIdx.x * nb + k] = s;
    }
}

// Per-block partial sums of w |c|^2 / n^2 binned by |k_x|, |k_y| and |k_z|
// separately (0..kmax each): partials[block][axis][k], axis 0, 1, 2 = x, y, z.
// w = 2 for the kx > 0 modes that stand for a conjugate pair (both members
// have the same |k_a|).  In a row every lane has its own |k_x| bin, and the
// whole row shares one |k_y| and one |k_z| bin: lane 0 adds the row's total,
// folded chunk by chunk over a fixed butterfly.
__global__ __launch_bounds__(256) void k_axis_bin(const hipfftDoubleComplex* c, uint32_t nx,
                                                  uint32_t ny, uint32_t nz, int kmax,
                                                  double inv_n2, double* partials) {
    extern __shared__ double hist[];   // [waves][3][kmax + 1]
    const int nb = 3 * (kmax + 1), waves = (int)(blockDim.x >> 6);
    for (int k = threadIdx.x; k < waves * nb; k += blockDim.x) hist[k] = 0.0;
    __syncthreads();
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    double* wh = hist + wave * nb;
    const uint32_t hx = nx / 2 + 1;
    const uint64_t rows = (uint64_t)ny * nz;
    for (uint64_t row = (uint64_t)blockIdx.x * waves + wave; row < rows;
         row += (uint64_t)gridDim.x * waves) {
        const uint32_t iy = (uint32_t)(row % ny), iz = (uint32_t)(row / ny);
        const int ay = (int)(iy <= ny / 2 ? iy : ny - iy);
        const int az = (int)(iz <= nz / 2 ? iz : nz - iz);
        const hipfftDoubleComplex* crow = c + row * hx;
        double total = 0.0;
        for (uint32_t x0 = 0; x0 < hx; x0 += 64) {
            const uint32_t ix = x0 + (uint32_t)lane;
            double p = 0.0;
            if (ix < hx) {
                const double w = (ix == 0 || (nx % 2 == 0 && ix == nx / 2)) ? 1.0 : 2.0;
                const hipfftDoubleComplex z = crow[ix];
                p = w * (z.x * z.x + z.y * z.y) * inv_n2;
                if ((int)ix <= kmax) wh[ix] += p;
            }
            for (int d = 32; d > 0; d >>= 1) p += __shfl_xor(p, d, 64);
            total += p;
        }
        if (lane == 0) {
            if (ay <= kmax) wh[kmax + 1 + ay] += total;
            if (az <= kmax) wh[2 * (kmax + 1) + az] += total;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        double s = hist[k];
        for (int w = 1; w < waves; ++w) s += hist[w * nb + k];
        partials[(uint64_t)blockIdx.x * nb + k] = s;
    }
}

// Threads per block of a binning kernel whose waves each keep `hist_bytes` of
// histogram: up to 4 waves within 64 KB of LDS.
static int bin_threads(size_t hist_bytes) {
    return 64 * (int)std::max<size_t>(1, std::min<size_t>(4, 65536 / hist_bytes));
}

// out[g][j] (+)= scale * sum over rows b of partials[g][b][j], one block per
// (column j, group g): thread t folds rows t, t + 256, ..., then a fixed tree
// over the block, so the order of the sum is the same on every call.
__global__ __launch_bounds__(256) void k_sum_rows(const double* partials, int rows, int cols,
                                                  double scale, int accumulate, double* out) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    const double* p = partials + (uint64_t)blockIdx.y * rows * cols;
    double s = 0.0;
    for (int b = threadIdx.x; b < rows; b += 256) s += p[(uint64_t)b * cols + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = out + (uint64_t)blockIdx.y * cols + j;
        *o = accumulate ? *o + red[0] * scale : red[0] * scale;
    }
}

__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// Per-block sums of du^2, du^3, |du|^3, du^4, |du|^5, du^6 for the separation
// rs[blockIdx.y] along each axis, du = u_a(x + r e_a) - u_a(x), periodic.
__global__ __launch_bounds__(256) void k_structure(const double* u, uint32_t nx, uint32_t ny,
                                                   uint32_t nz, const int32_t* rs, double* partials) {
    __shared__ double red[4];
    const uint32_t r = (uint32_t)rs[blockIdx.y];
    const uint32_t rx = r % nx, ry = r % ny, rz = r % nz;
    const uint64_t ncell = (uint64_t)nx * ny * nz;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x; c < ncell;
         c += (uint64_t)gridDim.x * 256) {
        const uint32_t x = (uint32_t)(c % nx);
        const uint64_t row = c / nx;
        const uint32_t y = (uint32_t)(row % ny), z = (uint32_t)(row / ny);
        const uint32_t xs = x + rx >= nx ? x + rx - nx : x + rx;
        const uint32_t ys = y + ry >= ny ? y + ry - ny : y + ry;
        const uint32_t zs = z + rz >= nz ? z + rz - nz : z + rz;
        const uint64_t c_x = (uint64_t)xs + (uint64_t)nx * row;
        const uint64_t c_y = x + (uint64_t)nx * (ys + (uint64_t)ny * z);
        const uint64_t c_z = x + (uint64_t)nx * (y + (uint64_t)ny * zs);
        const double d[3] = {u[c_x] - u[c], u[ncell + c_y] - u[ncell + c],
                             u[2 * ncell + c_z] - u[2 * ncell + c]};
        for (int a = 0; a < 3; ++a) {
            const double du = d[a], d2 = du * du, ad = fabs(du);
            acc[0] += d2;
            acc[1] += d2 * du;
            acc[2] += d2 * ad;
            acc[3] += d2 * d2;
            acc[4] += d2 * d2 * ad;
            acc[5] += d2 * d2 * d2;
        }
    }
    for (int m = 0; m < 6; ++m) {
        const double s = block_sum(acc[m], red);
        if (threadIdx.x == 0)
            partials[((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * 6 + m] = s;
    }
}

}  // namespace lbm

using namespace lbm;

namespace {

const char* fft_error(hipfftResult r) {
    switch (r) {
        case HIPFFT_SUCCESS: return "success";
        case HIPFFT_ALLOC_FAILED: return "allocation failed";
        case HIPFFT_INVALID_VALUE: return "invalid value";
        case HIPFFT_INVALID_SIZE: return "invalid size";
        default: return "hipFFT error";
    }
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

lbm_status set_err(lbm_handle* h, lbm_status st, const std::string& m) {
    h->err = m;
    return st;
}

lbm_status hip_err(lbm_handle* h, hipError_t e, const char* what) {
    return set_err(h, e == hipErrorOutOfMemory ? LBM_ERR_OUT_OF_MEMORY : LBM_ERR_DEVICE,
                   std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace lbm {

struct AnalysisCache {
    unsigned long long* hist = nullptr;   // theta histogram counts
    size_t hist_elems = 0;
    double* u = nullptr;                  // [3][ncell] velocity, FP64
    hipfftDoubleComplex* c = nullptr;     // [nz][ny][nx/2+1] transform of one component
    size_t c_elems = 0;
    double* part = nullptr;               // per-block partial sums
    size_t part_elems = 0;
    double* out = nullptr;                // reduced results
    size_t out_elems = 0;
    hipfftHandle plan = nullptr;
    bool has_plan = false;
    hipfftHandle plan3 = nullptr;         // the three components in one batched call
    bool has_plan3 = false;
    // snapshot (lbm_snapshot_begin / _end): completion event, the device K_t
    // plane and the page-locked results
    hipEvent_t ev_snap = nullptr;
    float* d_plane = nullptr;
    double* h_sums = nullptr;        // kStatSums reduced sums
    double* h_E = nullptr;           // spectrum, h_E_elems
    size_t h_E_elems = 0;
    float* h_plane = nullptr;        // nx * ny
    bool snap_pending = false;
    int snap_kmax = 0;
    int64_t snap_steps = 0;
};

void release_analysis(AnalysisCache* a) {
    if (!a) return;
    if (a->ev_snap) {
        (void)hipEventSynchronize(a->ev_snap);
        (void)hipEventDestroy(a->ev_snap);
    }
    if (a->d_plane) (void)hipFree(a->d_plane);
    if (a->h_sums) (void)hipHostFree(a->h_sums);
    if (a->h_E) (void)hipHostFree(a->h_E);
    if (a->h_plane) (void)hipHostFree(a->h_plane);
    if (a->has_plan) (void)hipfftDestroy(a->plan);
    if (a->has_plan3) (void)hipfftDestroy(a->plan3);
    if (a->hist) (void)hipFree(a->hist);
    if (a->u) (void)hipFree(a->u);
    if (a->c) (void)hipFree(a->c);
    if (a->part) (void)hipFree(a->part);
    if (a->out) (void)hipFree(a->out);
    delete a;
}

}  // namespace lbm

namespace {

AnalysisCache& cache(lbm_handle* h) {
    if (!h->ana) h->ana = new AnalysisCache();
    return *h->ana;
}

// Grow a cached device buffer to at least n elements of T.
template <typename T>
hipError_t ensure(T*& p, size_t& have, size_t n) {
    if (p && have >= n) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    have = 0;
    hipError_t e = hipMalloc((void**)&p, n * sizeof(T));
    if (e == hipSuccess) have = n;
    return e;
}

// Velocity (FP64, [3][ncell]) of the current state into the cached buffer.
lbm_status velocity(lbm_handle* h, const double** u) {
    AnalysisCache& a = cache(h);
    if (a.snap_pending)
        return set_err(h, LBM_ERR_STATE, "a snapshot is pending (lbm_snapshot_end first)");
    const size_t nc = h->args.ncell;
    if (!a.u) {
        hipError_t e = hipMalloc((void**)&a.u, 3 * nc * sizeof(double));
        if (e != hipSuccess) {
            a.u = nullptr;
            return hip_err(h, e, "hipMalloc(velocity)");
        }
    }
    hipError_t e = launch_moments(h->cfg.precision, current_pattern(h), current_args(h), nullptr,
                                  a.u, h->stream);
    if (e != hipSuccess) return hip_err(h, e, "moments kernel");
    *u = a.u;
    return LBM_OK;
}

// The handle's D2Z plan of its lattice (created on first use), bound to `stream`
// (the handle's stream by default).
lbm_status fft_plan(lbm_handle* h, AnalysisCache& a, hipStream_t stream) {
    if (!a.has_plan) {
        hipfftResult fr = hipfftPlan3d(&a.plan, (int)h->args.nz, (int)h->args.ny,
                                       (int)h->args.nx, HIPFFT_D2Z);
        if (fr != HIPFFT_SUCCESS)
            return set_err(h, LBM_ERR_DEVICE, std::string("hipfftPlan3d: ") + fft_error(fr));
        a.has_plan = true;
    }
    hipfftResult fr = hipfftSetStream(a.plan, stream);
    if (fr != HIPFFT_SUCCESS)
        return set_err(h, LBM_ERR_DEVICE, std::string("hipfftSetStream: ") + fft_error(fr));
    return LBM_OK;
}

// Lattices of up to 2^24 cells (256^3) transform the three velocity components in
// one batched call: at those sizes each transform's kernels are short and
// latency-bound, and batching them costs 16 bytes per cell more for the
// three-component transform buffer.  Larger lattices transform one component
// at a time into a one-component buffer, where the kernels are bandwidth-bound
// and the memory counts.
bool batched_fft(const lbm_handle* h) { return h->args.ncell <= (size_t(1) << 24); }

lbm_status fft_plan3(lbm_handle* h, AnalysisCache& a, hipStream_t stream) {
    if (!a.has_plan3) {
        const int nx = (int)h->args.nx, ny = (int)h->args.ny, nz = (int)h->args.nz;
        int n[3] = {nz, ny, nx}, inembed[3] = {nz, ny, nx}, onembed[3] = {nz, ny, nx / 2 + 1};
        const int idist = nz * ny * nx, odist = nz * ny * (nx / 2 + 1);
        hipfftResult fr = hipfftPlanMany(&a.plan3, 3, n, inembed, 1, idist, onembed, 1, odist,
                                         HIPFFT_D2Z, 3);
        if (fr != HIPFFT_SUCCESS)
            return set_err(h, LBM_ERR_DEVICE, std::string("hipfftPlanMany: ") + fft_error(fr));
        a.has_plan3 = true;
    }
    hipfftResult fr = hipfftSetStream(a.plan3, stream);
    if (fr != HIPFFT_SUCCESS)
        return set_err(h, LBM_ERR_DEVICE, std::string("hipfftSetStream: ") + fft_error(fr));
    return LBM_OK;
}

// Enqueue on `stream` the shell spectrum E[0..kmax] of the velocity u ([3][ncell])
// into a.out: the transforms, the per-block shell sums of each component and
// their fixed-order reduction.  a.c, a.part and a.out must be allocated
// (spectrum_buffers).
lbm_status enqueue_spectrum(lbm_handle* h, AnalysisCache& a, const double* u, int kmax,
                            hipStream_t stream) {
    const uint32_t nx = h->args.nx, ny = h->args.ny, nz = h->args.nz;
    const size_t nc = h->args.ncell, nmodes = (nx / 2 + 1) * (size_t)ny * nz;
    const bool batched = batched_fft(h);
    lbm_status st = batched ? fft_plan3(h, a, stream) : fft_plan(h, a, stream);
    if (st != LBM_OK) return st;
    const double inv_n2 = 1.0 / ((double)nc * (double)nc);
    const size_t shm = (size_t)(kmax + 1) * sizeof(double);
    const int bt = bin_threads(shm);
    hipfftResult fr = HIPFFT_SUCCESS;
    // batched: one binning pass sums the three components mode by mode;
    // otherwise each component's transform is binned and added in turn
    const int passes = batched ? 1 : 3, ncomp = batched ? 3 : 1;
    if (batched) fr = hipfftExecD2Z(a.plan3, (hipfftDoubleReal*)u, a.c);
    for (int c = 0; c < passes && fr == HIPFFT_SUCCESS; ++c) {
        if (!batched) {
            fr = hipfftExecD2Z(a.plan, (hipfftDoubleReal*)(u + (size_t)c * nc), a.c);
            if (fr != HIPFFT_SUCCESS) break;
        }
        hipLaunchKernelGGL(k_shell_bin, dim3(kAnaBlocks), dim3(bt), shm * (bt / 64), stream,
                           (const hipfftDoubleComplex*)a.c, (uint64_t)nmodes, ncomp, nx, ny, nz,
                           (int)kmax, inv_n2, a.part);
        hipLaunchKernelGGL(k_sum_rows, dim3(kmax + 1), dim3(256), 0, stream,
                           (const double*)a.part, kAnaBlocks, (int)(kmax + 1), 1.0, c > 0, a.out);
    }
    if (fr != HIPFFT_SUCCESS) return set_err(h, LBM_ERR_DEVICE, std::string("hipFFT: ") + fft_error(fr));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err(h, e, "spectrum kernels");
    return LBM_OK;
}

// The transform buffer and the partial and reduced sums of a spectrum to kmax.
hipError_t spectrum_buffers(lbm_handle* h, AnalysisCache& a, int kmax) {
    const size_t nmodes = (h->args.nx / 2 + 1) * (size_t)h->args.ny * h->args.nz;
    hipError_t e = ensure(a.c, a.c_elems, batched_fft(h) ? 3 * nmodes : nmodes);
    if (e == hipSuccess) e = ensure(a.part, a.part_elems, (size_t)kAnaBlocks * (kmax + 1));
    if (e == hipSuccess) e = ensure(a.out, a.out_elems, (size_t)(kmax + 1));
    return e;
}

}  // namespace

extern "C" {

lbm_status lbm_spectrum(lbm_handle* h, int32_t kmax, double* E) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (!E || kmax < 0 || kmax > 4096) return set_err(h, LBM_ERR_INVALID_ARG, "kmax must be 0..4096");
    if (!h->initialized) return set_err(h, LBM_ERR_STATE, "state not initialised");
    const double* u = nullptr;
    lbm_status st = velocity(h, &u);
    if (st != LBM_OK) return st;
    AnalysisCache& a = cache(h);
    hipError_t e = spectrum_buffers(h, a, kmax);
    if (e != hipSuccess) return hip_err(h, e, "hipMalloc(spectrum)");
    st = enqueue_spectrum(h, a, u, kmax, h->stream);
    if (st != LBM_OK) return st;
    const size_t shm = (size_t)(kmax + 1) * sizeof(double);
    e = hipMemcpyAsync(E, a.out, shm, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(h, e, "spectrum");
    return LBM_OK;
}

lbm_status lbm_snapshot_begin(lbm_handle* h, int32_t kmax, int32_t z) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (kmax < 0 || kmax > 4096) return set_err(h, LBM_ERR_INVALID_ARG, "kmax must be 0..4096");
    if (z < 0 || (uint32_t)z >= h->args.nz) return set_err(h, LBM_ERR_INVALID_ARG, "z outside 0..nz-1");
    if (!h->initialized) return set_err(h, LBM_ERR_STATE, "state not initialised");
    AnalysisCache& a = cache(h);
    if (a.snap_pending) return set_err(h, LBM_ERR_STATE, "a snapshot is already pending");
    const size_t nc = h->args.ncell, nxy = h->args.nxy;
    // buffers, created on first use and kept until lbm_destroy
    hipError_t e = hipSuccess;
    if (!a.u) e = hipMalloc((void**)&a.u, 3 * nc * sizeof(double));
    if (e == hipSuccess) e = spectrum_buffers(h, a, kmax);
    if (e == hipSuccess && !a.d_plane) e = hipMalloc((void**)&a.d_plane, nxy * sizeof(float));
    if (e == hipSuccess && !a.h_sums) e = hipHostMalloc((void**)&a.h_sums, kDiagSlots * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess && !a.h_plane) e = hipHostMalloc((void**)&a.h_plane, nxy * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess && a.h_E_elems < (size_t)kmax + 1) {
        if (a.h_E) (void)hipHostFree(a.h_E);
        a.h_E = nullptr;
        a.h_E_elems = 0;
        e = hipHostMalloc((void**)&a.h_E, ((size_t)kmax + 1) * sizeof(double), hipHostMallocDefault);
        if (e == hipSuccess) a.h_E_elems = (size_t)kmax + 1;
    }
    if (e == hipSuccess && !a.ev_snap) e = hipEventCreateWithFlags(&a.ev_snap, hipEventDisableTiming);
    if (e != hipSuccess) return hip_err(h, e, "snapshot buffers");
    // everything on the handle's stream, in order with the steps: the state reads,
    // the transforms of the velocity and the copies to page-locked memory
    double* sums = nullptr;
    e = launch_stats(h, &sums);
    const int pat = current_pattern(h);
    const LatticeArgs args = current_args(h);
    if (e == hipSuccess) e = launch_ktslice(h->cfg.precision, pat, args, (uint32_t)z, a.d_plane, h->stream);
    if (e == hipSuccess) e = launch_moments(h->cfg.precision, pat, args, nullptr, a.u, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(a.h_sums, sums, kStatSums * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(a.h_plane, a.d_plane, nxy * sizeof(float), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_err(h, e, "snapshot (state reads)");
    lbm_status st = enqueue_spectrum(h, a, a.u, kmax, h->stream);
    if (st != LBM_OK) return st;
    const size_t shm = (size_t)(kmax + 1) * sizeof(double);
    e = hipMemcpyAsync(a.h_E, a.out, shm, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipEventRecord(a.ev_snap, h->stream);
    if (e != hipSuccess) return hip_err(h, e, "snapshot (spectrum)");
    a.snap_pending = true;
    a.snap_kmax = kmax;
    a.snap_steps = h->steps;
    return LBM_OK;
}

lbm_status lbm_snapshot_end(lbm_handle* h, lbm_stats* stats, double* E, float* kt_plane) {
    if (!h) return LBM_ERR_INVALID_ARG;
    AnalysisCache* a = h->ana;
    if (!a || !a->snap_pending) return set_err(h, LBM_ERR_STATE, "no snapshot is pending");
    a->snap_pending = false;
    const hipError_t e = hipEventSynchronize(a->ev_snap);
    if (e != hipSuccess) return hip_err(h, e, "snapshot");
    if (E) memcpy(E, a->h_E, ((size_t)a->snap_kmax + 1) * sizeof(double));
    if (kt_plane) memcpy(kt_plane, a->h_plane, h->args.nxy * sizeof(float));
    if (stats) {
        fill_stats(h, a->h_sums, a->snap_steps, stats);
        if (stats->n_nonfinite > 0)
            return set_err(h, LBM_ERR_UNSTABLE, std::to_string(stats->n_nonfinite) + " non-finite cells");
    }
    return LBM_OK;
}

lbm_status lbm_theta_histogram(lbm_handle* h, double lo, double hi, int32_t nbins,
                               int64_t* counts) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (!counts || nbins < 1 || nbins > 4096)
        return set_err(h, LBM_ERR_INVALID_ARG, "nbins must be 1..4096 and counts non-NULL");
    if (!(std::isfinite(lo) && std::isfinite(hi) && hi > lo))
        return set_err(h, LBM_ERR_INVALID_ARG, "need finite lo < hi");
    if (!h->initialized) return set_err(h, LBM_ERR_STATE, "state not initialised");
    AnalysisCache& a = cache(h);
    const size_t n = (size_t)nbins + 3;
    hipError_t e = ensure(a.hist, a.hist_elems, n);
    if (e == hipSuccess) e = hipMemsetAsync(a.hist, 0, n * sizeof(unsigned long long), h->stream);
    if (e == hipSuccess)
        e = launch_theta_hist(h->cfg.precision, current_pattern(h), current_args(h), lo,
                              (double)nbins / (hi - lo), (int)nbins, a.hist, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts, a.hist, n * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(h, e, "theta histogram");
    return LBM_OK;
}

lbm_status lbm_spectra_1d(lbm_handle* h, int32_t kmax, double* E, double* ic) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (!E || kmax < 0 || kmax > 2048) return set_err(h, LBM_ERR_INVALID_ARG, "kmax must be 0..2048");
    if (!h->initialized) return set_err(h, LBM_ERR_STATE, "state not initialised");
    const uint32_t nx = h->args.nx, ny = h->args.ny, nz = h->args.nz;
    if (ic && (ny != nx || nz != nx))
        return set_err(h, LBM_ERR_INVALID_ARG, "the isotropy coefficient needs a cubic lattice");
    const size_t nc = h->args.ncell, nmodes = (nx / 2 + 1) * (size_t)ny * nz;
    const int cols = 3 * (kmax + 1);
    const double* u = nullptr;
    lbm_status st = velocity(h, &u);
    if (st != LBM_OK) return st;
    AnalysisCache& a = cache(h);
    hipError_t e = ensure(a.c, a.c_elems, nmodes);
    if (e == hipSuccess) e = ensure(a.part, a.part_elems, (size_t)kAnaBlocks * cols);
    if (e == hipSuccess) e = ensure(a.out, a.out_elems, (size_t)3 * cols);
    if (e != hipSuccess) return hip_err(h, e, "hipMalloc(one-dimensional spectra)");
    st = fft_plan(h, a, h->stream);
    if (st != LBM_OK) return st;
    const double inv_n2 = 1.0 / ((double)nc * (double)nc);
    hipfftResult fr = HIPFFT_SUCCESS;
    for (int c = 0; c < 3 && fr == HIPFFT_SUCCESS; ++c) {
        fr = hipfftExecD2Z(a.plan, (hipfftDoubleReal*)(u + (size_t)c * nc), a.c);
        if (fr != HIPFFT_SUCCESS) break;
        const size_t hb = (size_t)cols * sizeof(double);
        const int bt = bin_threads(hb);
        hipLaunchKernelGGL(k_axis_bin, dim3(kAnaBlocks), dim3(bt), hb * (bt / 64), h->stream,
                           (const hipfftDoubleComplex*)a.c, nx, ny, nz, (int)kmax, inv_n2,
                           a.part);
        hipLaunchKernelGGL(k_sum_rows, dim3(cols), dim3(256), 0, h->stream, (const double*)a.part,
                           kAnaBlocks, cols, 1.0, 0, a.out + (size_t)c * cols);
    }
    if (fr != HIPFFT_SUCCESS) return set_err(h, LBM_ERR_DEVICE, std::string("hipFFT: ") + fft_error(fr));
    e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(E, a.out, (size_t)3 * cols * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(h, e, "one-dimensional spectra");
    if (ic) {
        // App. spectral isotropy, with the isotropic relation between the
        // longitudinal and transverse spectra: IC = (E_L - k dE_L/dk) / (2 E_T),
        // E_L / E_T the means of the 3 longitudinal / 6 transverse spectra, the
        // slope k dE_L/dk = E_L dln E_L / dln k by a central difference in
        // log-log space; NaN where it is undefined.
        std::vector<double> EL(kmax + 1), ET(kmax + 1);
        const size_t K = (size_t)kmax + 1;
        for (size_t k = 0; k < K; ++k) {
            // E[c][a][k] at E[(3 c + a) K + k]
            EL[k] = (E[0 * K + k] + E[4 * K + k] + E[8 * K + k]) / 3.0;
            ET[k] = (E[3 * K + k] + E[6 * K + k] + E[1 * K + k] + E[7 * K + k] + E[2 * K + k] +
                     E[5 * K + k]) / 6.0;
        }
        for (size_t k = 0; k < K; ++k) {
            ic[k] = NAN;
            if (k >= 2 && k + 1 < K && EL[k + 1] > 0.0 && EL[k - 1] > 0.0 && ET[k] > 0.0) {
                const double slope = (log(EL[k + 1]) - log(EL[k - 1])) /
                                     (log((double)k + 1.0) - log((double)k - 1.0));
                ic[k] = (EL[k] - EL[k] * slope) / (2.0 * ET[k]);
            }
        }
    }
    return LBM_OK;
}

lbm_status lbm_structure_functions(lbm_handle* h, const int32_t* rs, int32_t nr, double* out) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (nr < 1 || nr > 65535 || !rs || !out) return set_err(h, LBM_ERR_INVALID_ARG, "bad rs/nr/out");
    for (int j = 0; j < nr; ++j)
        if (rs[j] < 1) return set_err(h, LBM_ERR_INVALID_ARG, "separations must be >= 1");
    if (!h->initialized) return set_err(h, LBM_ERR_STATE, "state not initialised");
    const uint32_t nx = h->args.nx, ny = h->args.ny, nz = h->args.nz;
    const size_t nc = h->args.ncell;
    DevBuf drs, part, res;
    const double* u = nullptr;
    lbm_status st = velocity(h, &u);
    if (st != LBM_OK) return st;
    const int nb = (int)std::min<size_t>(kAnaBlocks, (nc + 255) / 256);
    hipError_t e = hipMalloc(&drs.p, nr * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&part.p, (size_t)nr * nb * 6 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&res.p, (size_t)nr * 6 * sizeof(double));
    if (e != hipSuccess) return hip_err(h, e, "hipMalloc(structure functions)");
    e = hipMemcpyAsync(drs.p, rs, nr * sizeof(int32_t), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_err(h, e, "copy separations");
    hipLaunchKernelGGL(k_structure, dim3(nb, nr), dim3(256), 0, h->stream, u, nx,
                       ny, nz, (const int32_t*)drs.p, (double*)part.p);
    // rows of 6 sums per (r, block): reduce the blocks of each r in a fixed order
    hipLaunchKernelGGL(k_sum_rows, dim3(6, nr), dim3(256), 0, h->stream, (const double*)part.p,
                       nb, 6, 1.0 / (3.0 * nc), 0, (double*)res.p);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out, res.p, (size_t)nr * 6 * sizeof(double),
                                            hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(h, e, "structure functions");
    return LBM_OK;
}

lbm_status lbm_turbulence(lbm_handle* h, int32_t kmax, lbm_turbulence_stats* out) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (!out) return set_err(h, LBM_ERR_INVALID_ARG, "out is NULL");
    const uint32_t N = h->args.nx;
    if (h->args.ny != N || h->args.nz != N)
        return set_err(h, LBM_ERR_INVALID_ARG, "turbulence scales need a cubic lattice");
    const int32_t kall = (int32_t)(0.5 * sqrt(3.0) * N + 1.0);   // every shell present
    if (kmax <= 0 || kmax > kall) kmax = kall;
    if (kmax > 4096) return set_err(h, LBM_ERR_INVALID_ARG, "lattice too large for the spectrum");
    std::vector<double> E((size_t)kmax + 1);
    lbm_status st = lbm_spectrum(h, kmax, E.data());
    if (st != LBM_OK) return st;
    lbm_stats s;
    st = lbm_kt_stats(h, &s);
    if (st != LBM_OK) return st;
    // Sec. 2.2 with the shell index k of the N-cell box as the wavenumber
    // kappa = 2 pi k / N in lattice units; the mean flow (k = 0) is excluded.
    const double nu0 = (h->cfg.tau0 - 0.5) / 3.0;
    double e = 0.0, e_over_k = 0.0, k2e = 0.0;
    for (int32_t k = 1; k <= kmax; ++k) {
        const double kap = 2.0 * M_PI * k / N;
        e += E[k];
        e_over_k += E[k] / kap;
        k2e += kap * kap * E[k];
    }
    memset(out, 0, sizeof *out);
    out->kmax = kmax;
    out->energy = s.energy;
    out->energy_spec = e;
    out->u_rms = sqrt(2.0 * e / 3.0);                        // eq. rms_velocity
    out->integral_scale = e > 0.0 ? 0.75 * M_PI * e_over_k / e : NAN;   // eq. integral_length_scale
    out->eps_spec = 2.0 * nu0 * k2e;                          // eq. dissipation_rate
    out->eps_strain = nu0 * s.strain2;                        // 2 nu0 <S:S>
    out->eps_sgs = s.nut_strain2;
    out->injection = s.injection;                             // <F.u>
    const double eps = out->eps_spec;
    out->eta = eps > 0.0 ? pow(nu0 * nu0 * nu0 / eps, 0.25) : NAN;          // eq. kolmogorov_scale
    out->taylor = eps > 0.0 ? sqrt(15.0 * nu0 * out->u_rms * out->u_rms / eps) : NAN;  // eq. taylor_microscale
    out->re_lambda = out->u_rms * out->taylor / nu0;
    // isotropy: Reynolds stresses of the fluctuations about the mean velocity
    const double* m = s.u_mean;
    const double R[3][3] = {
        {s.uu[0] - m[0] * m[0], s.uu[3] - m[0] * m[1], s.uu[4] - m[0] * m[2]},
        {s.uu[3] - m[0] * m[1], s.uu[1] - m[1] * m[1], s.uu[5] - m[1] * m[2]},
        {s.uu[4] - m[0] * m[2], s.uu[5] - m[1] * m[2], s.uu[2] - m[2] * m[2]}};
    const double tr = R[0][0] + R[1][1] + R[2][2];
    double b[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) b[i][j] = tr > 0.0 ? R[i][j] / tr - (i == j ? 1.0 / 3.0 : 0.0) : NAN;
    double b2 = 0.0, b3 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            b2 += b[i][j] * b[j][i];
            for (int k = 0; k < 3; ++k) b3 += b[i][j] * b[j][k] * b[k][i];
        }
    for (int i = 0; i < 3; ++i) out->energy_frac[i] = tr > 0.0 ? R[i][i] / tr : NAN;
    out->b[0] = b[0][0]; out->b[1] = b[1][1]; out->b[2] = b[2][2];
    out->b[3] = b[0][1]; out->b[4] = b[0][2]; out->b[5] = b[1][2];
    out->II_b = -0.5 * b2;
    out->III_b = b3 / 3.0;
    out->lumley_xi = cbrt(0.5 * out->III_b);
    out->lumley_eta = sqrt(fmax(0.0, -out->II_b / 3.0));
    return LBM_OK;
}

}  // extern "C"
