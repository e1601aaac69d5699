// lbm_observe.hpp — host-side helpers shared by the C-ABI calls that observe
// the state (lbm_api.hip: lbm_kt_stats; lbm_analysis.hip: the snapshot).  Not
// part of the public ABI.
#pragma once

#include "lbm_internal.hpp"

namespace lbm {

// Number of reduced sums k_diag / k_diag_final produce (their layout is
// documented at k_diag in lbm_kernels.hip).
constexpr int kStatSums = 25;
static_assert(kStatSums <= kDiagSlots, "reduced sums overflow the result slots");

// Enqueue the domain reductions of the current state on h's stream; *result
// receives the device address of the kStatSums reduced sums.
hipError_t launch_stats(lbm_handle* h, double** result);

// lbm_stats of the reduced sums r[0..kStatSums) of a state `steps` steps old.
void fill_stats(const lbm_handle* h, const double* r, int64_t steps, lbm_stats* out);

}  // namespace lbm
