// Regime diagnostics (Section 2): per-line histogram of the shift-to-pixel ratio
// eta_s = ||Delta_s|| / p = c_s ||D tau||, c_s = L delta_s / p^2, over a thickness map.
//
// One pass over tau (4 bytes per pixel).  Each workgroup owns kRegimeRows rows, bins every
// pixel for every line into an LDS histogram with LDS atomics, and adds its non-zero bins to
// the device histogram with global integer atomics.  Integer sums do not depend on the order,
// so the counts are exact and deterministic.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "epr_internal.h"
#include "regime.h"

namespace epr {

// Correctly rounded float square root of x >= 0.  The hardware estimate is within an ulp or
// so; it is moved one ulp at a time while x lies beyond the midpoint to a neighbour.  A
// midpoint of two adjacent floats has at most 25 significant bits, so its square, and hence
// every comparison, is exact in double.
__device__ __forceinline__ float sqrt_rn(float x) {
  if (!(x > 0.f)) return x;  // 0 (and NaN) unchanged
  float s = __builtin_amdgcn_sqrtf(x);
  const double xd = x;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float up = __int_as_float(__float_as_int(s) + 1);
    const double mh = 0.5 * ((double)s + (double)up);
    if (xd > mh * mh) s = up;
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float dn = __int_as_float(__float_as_int(s) - 1);
    const double ml = 0.5 * ((double)s + (double)dn);
    if (xd < ml * ml) s = dn;
  }
  return s;
}

// Each bin decision is taken in float32 with every operation rounded on its own (no fused
// multiply-add): g = sqrt(Dx*Dx + Dy*Dy), eta = c_s g, v = eta * scale, bin = min(floor(v),
// n_bins).  NaN lands in the last bin.
__global__ __launch_bounds__(256) void k_regime(const float* __restrict__ tau, int ny, int nx,
                                                RegimeParams rp, unsigned* __restrict__ counts) {
#pragma clang fp contract(off)
  extern __shared__ unsigned hist[];
  const int L = rp.n_lines, nb1 = rp.n_bins + 1, nh = L * nb1;
  for (int i = threadIdx.x; i < nh; i += 256) hist[i] = 0u;
  __syncthreads();
  gptr<const float> t = G(tau);
  const float cap = (float)rp.n_bins;
  const int y0 = blockIdx.x * kRegimeRows;
  const int y1 = min(y0 + kRegimeRows, ny);
  for (int y = y0; y < y1; ++y) {
    for (int x = threadIdx.x; x < nx; x += 256) {
      const float gx = d_x(t, y, x, nx);
      const float gy = d_y(t, y, x, ny, nx);
      const float g = sqrt_rn(gx * gx + gy * gy);
      for (int s = 0; s < L; ++s) {
        const float v = (rp.c[s] * g) * rp.scale;
        const float b = fminf(floorf(v), cap);
        const int bin = (b >= 0.f) ? (int)b : rp.n_bins;  // (fminf maps NaN to cap already)
        atomicAdd(&hist[s * nb1 + bin], 1u);
      }
    }
  }
  __syncthreads();
  gptr<unsigned> out = G(counts);
  for (int i = threadIdx.x; i < nh; i += 256) {
    const unsigned v = hist[i];
    if (v) atomicAdd(&out[i], v);
  }
}

// Clear n 32-bit words (a fill kernel rather than a memset node, so the sequence can be
// captured into a graph).
__global__ __launch_bounds__(256) void k_fill_u32(unsigned* __restrict__ p, int n, unsigned v) {
  gptr<unsigned> q = G(p);
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) q[i] = v;
}

hipError_t launch_regime(const float* tau, int ny, int nx, const RegimeParams& rp,
                         unsigned* counts, hipStream_t s) {
  const int nh = rp.n_lines * (rp.n_bins + 1);
  hipLaunchKernelGGL(k_fill_u32, dim3((nh + 255) / 256), dim3(256), 0, s, counts, nh, 0u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = (ny + kRegimeRows - 1) / kRegimeRows;
  hipLaunchKernelGGL(k_regime, dim3(nb), dim3(256), sizeof(unsigned) * (size_t)nh, s, tau, ny,
                     nx, rp, counts);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, int n, hipStream_t s) {
  const int nb = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_fill_u32, dim3(nb), dim3(256), 0, s, p, n, 0u);
  return hipGetLastError();
}

hipError_t set_regime_attributes() {
  return hipFuncSetAttribute((const void*)k_regime, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(unsigned) * kMaxLines * (kMaxBins + 1)));
}

}  // namespace epr
