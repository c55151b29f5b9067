// Vector-Jacobian product of the non-local forward model (Eqs. 2-5) with respect to the phase
// and absorption maps, for the autograd backward.
//
// P = sum_s M_s(u_s)[I_s], I_s = w_s exp(-a_s A), u_s = b_s D phase.  With g = dL/dP:
//   dL/dI_s  = M_s^* g   (bilinear interpolation of g at the mapped point, Eq. 4)
//   dL/du_s  = I_s * gradient of that interpolant with respect to the mapped point
//              (constant inside a cell: the splat is piecewise linear in u)
//   grad_A   = sum_s -a_s I_s dL/dI_s
//   grad_phi = D_x^T Gx + D_y^T Gy,  G = sum_s b_s dL/du_s
// The ray map is recomputed from the phase; nothing is kept from the forward call.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "epr_internal.h"

namespace epr {

constexpr int kVjpThreads = 256;

__global__ __launch_bounds__(kVjpThreads) void k_vjp(KArgs a, float* __restrict__ Gx,
                                                     float* __restrict__ Gy,
                                                     float* __restrict__ gA) {
  const ProbDesc& p = a.p;
  const int nx = p.nx, ny = p.ny, L = p.lp.n;
  const int i = blockIdx.x * kVjpThreads + threadIdx.x;
  if (i >= nx * ny) return;
  const int y = i / nx, x = i - y * nx;
  gptr<const float> g = G(p.d);  // incoming gradient dL/dP
  const float gxs = d_x(G(p.Y), y, x, nx);
  const float gys = d_y(G(p.Y), y, x, ny, nx);
  const float av = G(p.X)[i];
  float sa = 0.f, sx = 0.f, sy = 0.f;
  for (int s = 0; s < L; ++s) {
    const float I = p.lp.w[s] * expf(-p.lp.a[s] * av);
    const float bs = p.lp.b[s];
    const float ux = bs * gxs, uy = bs * gys;
    const float fx = floorf(ux), fy = floorf(uy);
    const float dx = ux - fx, dy = uy - fy;
    const int x0 = x + (int)fx, y0 = y + (int)fy;
    float g00 = 0.f, g10 = 0.f, g01 = 0.f, g11 = 0.f;  // g_ij: paper's tap w_ij
    const bool xin0 = x0 >= 0 && x0 < nx, xin1 = x0 + 1 >= 0 && x0 + 1 < nx;
    if (y0 >= 0 && y0 < ny) {
      if (xin0) g00 = g[(size_t)y0 * nx + x0];
      if (xin1) g10 = g[(size_t)y0 * nx + x0 + 1];
    }
    if (y0 + 1 >= 0 && y0 + 1 < ny) {
      if (xin0) g01 = g[(size_t)(y0 + 1) * nx + x0];
      if (xin1) g11 = g[(size_t)(y0 + 1) * nx + x0 + 1];
    }
    const float gI = (1.f - dy) * ((1.f - dx) * g00 + dx * g10) + dy * ((1.f - dx) * g01 + dx * g11);
    const float gux = I * ((1.f - dy) * (g10 - g00) + dy * (g11 - g01));
    const float guy = I * ((1.f - dx) * (g01 - g00) + dx * (g11 - g10));
    sa -= p.lp.a[s] * I * gI;
    sx += bs * gux;
    sy += bs * guy;
  }
  gA[i] = sa;
  Gx[i] = sx;
  Gy[i] = sy;
}

// Transpose of D along one axis of length n applied to g at index j (row-major access through
// `at`): D has rows (-1, 1) at 0, (-1/2, 0, 1/2) inside and (-1, 1) at n-1.
template <class F>
__device__ __forceinline__ float d_transpose(F at, int j, int n) {
  if (j == 0) return -at(0) - 0.5f * at(1);
  if (j == 1) return at(0) - 0.5f * at(2);
  if (j == n - 2) return 0.5f * at(n - 3) - at(n - 1);
  if (j == n - 1) return 0.5f * at(n - 2) + at(n - 1);
  return 0.5f * (at(j - 1) - at(j + 1));
}

__global__ __launch_bounds__(kVjpThreads) void k_vjp_transpose(KArgs a,
                                                               const float* __restrict__ Gx,
                                                               const float* __restrict__ Gy,
                                                               float* __restrict__ gphi) {
  const ProbDesc& p = a.p;
  const int nx = p.nx, ny = p.ny;
  const int i = blockIdx.x * kVjpThreads + threadIdx.x;
  if (i >= nx * ny) return;
  const int y = i / nx, x = i - y * nx;
  const float* rowx = Gx + (size_t)y * nx;
  const float tx = d_transpose([&](int k) { return rowx[k]; }, x, nx);
  const float ty = d_transpose([&](int k) { return Gy[(size_t)k * nx + x]; }, y, ny);
  gphi[i] = tx + ty;
}

hipError_t launch_vjp(const KArgs& a, int total_blocks, size_t, hipStream_t s, float* gx,
                      float* gy, float* ga) {
  hipLaunchKernelGGL(k_vjp, dim3(total_blocks), dim3(kVjpThreads), 0, s, a, gx, gy, ga);
  return hipGetLastError();
}

hipError_t launch_vjp_transpose(const KArgs& a, int total_blocks, hipStream_t s,
                                const float* gx, const float* gy, float* gphase) {
  hipLaunchKernelGGL(k_vjp_transpose, dim3(total_blocks), dim3(kVjpThreads), 0, s, a, gx, gy,
                     gphase);
  return hipGetLastError();
}

hipError_t set_vjp_attributes() { return hipSuccess; }

}  // namespace epr
