// Regime diagnostics (Section 2): parameters and launch wrappers of the shift-to-pixel
// histogram kernel, shared by that kernel and the host side of libepr.
#pragma once

#include <hip/hip_runtime.h>

#include "epr_internal.h"

namespace epr {

// eta_s = c_s ||D tau|| with c_s = L delta_s / p^2; scale = n_bins / eta_max.  Both are rounded
// to float on the host, where the bin decision's precision starts.
constexpr int kMaxBins = 1023;
constexpr int kRegimeRows = 4;   // image rows per workgroup
struct RegimeParams {
  int n_lines;
  int n_bins;
  float scale;
  float c[kMaxLines];
};

// Clears counts [n_lines][n_bins + 1] and adds the histogram of tau to it.
hipError_t launch_regime(const float* tau, int ny, int nx, const RegimeParams& rp,
                         unsigned* counts, hipStream_t s);
// Sets n 32-bit words to zero with a kernel (no memset node).
hipError_t launch_fill_u32(unsigned* p, int n, hipStream_t s);
hipError_t set_regime_attributes();

}  // namespace epr
