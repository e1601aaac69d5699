// lbm_internal.hpp — handle layout and kernel launchers shared by the C-ABI
// front end (lbm_api.hip), the kernels (lbm_kernels.hip) and the batched
// stepping (lbm_batch.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "d3q19_mrt.hpp"
#include "lbm_index.hpp"

namespace lbm {

// Access patterns of the population state.
//   AA_EVEN: f_i(x) is at slot i of cell x          (AA, even step count)
//   AA_ODD : f_i(x) is at slot opp(i) of cell x-c_i (AA, odd step count)
//   AB     : f_i(x) is at slot i of cell x-c_i in the current array
enum Pattern : int { PAT_AA_EVEN = 0, PAT_AA_ODD = 1, PAT_AB = 2 };

// Everything a kernel needs about one lattice, passed by value.
struct LatticeArgs {
    void* a;                 // population array (AA: the only one; AB: current source)
    void* b;                 // AB: destination; AA: == a
    uint64_t plane;          // elements per direction plane (padded); plane bytes < 2^32
    char* pa[19];            // plane i of a: a + i * plane * element bytes
    char* pb[19];            // plane i of b (precomputed on the host: kernels take the
                             // 64-bit plane bases from kernel arguments, no scalar math)
    uint32_t nx, ny, nz, nxy, ncell;
    DivMagic mx, my;         // division by nx (cell -> row) and ny (row -> z)
    const void* rowc;        // force row coefficients [ny*nz][16] in R, or null
    const void* xtab;        // [nx][4] sin/cos of the first two x harmonics, in R
    CollideConst<double> kd; // collision constants for FP64 arithmetic
    CollideConst<float> kf;  // the same rounded to FP32 on the host
    double tau0, rho0;
    double sigma, inv_sigma; // FP16/BF16 storage scale
    float sigma_f, inv_sigma_f;
    int32_t xcd_remap;       // step-kernel block order: 0 dispatch order, 1 one contiguous
                             // range per XCD, K >= 2 chunks of K blocks in turn
    int32_t nt_mode;         // step kernel: bit 1 non-temporal stores
    uint32_t elem_bytes;     // bytes per stored population
    uint32_t pad_;
};

// Kernel launchers (lbm_kernels.hip).  All return the launch status.
hipError_t launch_tables(int precision, const LatticeArgs& L, const lbm_force_mode* d_modes,
                         int n_modes, hipStream_t s);
hipError_t launch_init(int precision, int pat, const LatticeArgs& L, int kind, double amp,
                       uint64_t seed, hipStream_t s);
hipError_t launch_step(int precision, int pat, const LatticeArgs& L, hipStream_t s);
hipError_t launch_stream(int precision, int pat, const LatticeArgs& L, hipStream_t s);
hipError_t launch_diag(int precision, int pat, const LatticeArgs& L, double* partials,
                       int nblocks, double* result, hipStream_t s);
hipError_t launch_moments(int precision, int pat, const LatticeArgs& L, double* rho, double* u,
                          hipStream_t s);
hipError_t launch_ktfield(int precision, int pat, const LatticeArgs& L, float* kt, hipStream_t s);
hipError_t launch_ktslice(int precision, int pat, const LatticeArgs& L, uint32_t z, float* kt,
                          hipStream_t s);
hipError_t launch_theta_hist(int precision, int pat, const LatticeArgs& L, double lo, double inv_w,
                             int nbins, unsigned long long* counts, hipStream_t s);
hipError_t launch_gather_plane(int precision, int pat, const LatticeArgs& L, int i, double* out,
                               hipStream_t s);
hipError_t launch_scatter_plane(int precision, int pat, const LatticeArgs& L, int i,
                                const double* in, hipStream_t s);
hipError_t launch_sample(int precision, int pat, const LatticeArgs& L, const int64_t* cells,
                         int64_t n, double* out, hipStream_t s);
// Two steps in one pass (lbm_tb2.hip): A/B pull from L.a into L.b.
bool tb2_supported(int precision);
hipError_t launch_step_tb2(int precision, const LatticeArgs& L, hipStream_t s);

constexpr int kDiagBlocks = 1024;   // fixed grid of the diagnostic reduction
constexpr int kDiagSlots = 32;      // doubles per block partial

}  // namespace lbm

namespace lbm {
struct AnalysisCache;                      // lbm_analysis.hip
void release_analysis(AnalysisCache* a);   // NULL-safe
}  // namespace lbm

struct lbm_handle {
    lbm_config cfg;                          // copy; force_modes points into `modes`
    std::vector<lbm_force_mode> modes;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_state = false;
    void* state_base = nullptr;              // whole state allocation (or caller buffer)
    void* state[2] = {nullptr, nullptr};
    size_t plane_elems = 0, elem_bytes = 0, state_bytes = 0;
    void* rowc = nullptr;
    void* xtab = nullptr;
    lbm_force_mode* d_modes = nullptr;
    double* partials = nullptr;              // [kDiagBlocks][kDiagSlots] + result
    double* staging = nullptr;               // lazily sized device staging
    size_t staging_elems = 0;
    int64_t* d_cells = nullptr;
    size_t d_cells_cap = 0;
    int64_t steps = 0;
    int cur = 0;                             // AB: index of the current array
    bool initialized = false;
    lbm::LatticeArgs args{};
    // graph of steps_per_graph steps, captured on first use
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;
    // FFT plan and velocity / transform buffers of the analysis calls, created
    // on first use and kept until lbm_destroy
    lbm::AnalysisCache* ana = nullptr;
    std::string err;
};

namespace lbm {
// Current pattern and arrays of a handle for its step count / AB parity.
int current_pattern(const lbm_handle* h);
LatticeArgs current_args(const lbm_handle* h);
// Point a (source) and b (destination) of L at two population arrays, with their planes.
void set_arrays(LatticeArgs& L, void* a, void* b);
// Advance h's bookkeeping after one launched step.
void advance(lbm_handle* h);
}  // namespace lbm
