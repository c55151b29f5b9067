// Vector-Jacobian products of the forward models (Eqs. 1-5) with respect to the phase and
// absorption maps, for the autograd backward.
//
// Non-local model: P = sum_s M_s(u_s)[I_s], I_s = w_s exp(-a_s A), u_s = b_s D phase.  With
// g = dL/dP:
//   dL/dI_s  = M_s^* g   (bilinear interpolation of g at the mapped point, Eq. 4)
//   dL/du_s  = I_s * gradient of that interpolant with respect to the mapped point
//              (constant inside a cell: the splat is piecewise linear in u)
//   grad_A   = sum_s -a_s I_s dL/dI_s
//   grad_phi = D_x^T Gx + D_y^T Gy,  G = sum_s b_s dL/du_s
// The ray map is recomputed from the phase; nothing is kept from the forward call.
//
// XDEP: x-dependent spectrum (Methods 4.3 remark).  Both maps are the thickness tau, and
// w_s, a_s (= mu_s), b_s and q_s are read at each pixel's column; the caller adds the transposed
// shift gradients to grad_A (k_vjp_transpose with `accumulate`) to obtain dL/dtau.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "epr_internal.h"

namespace epr {

constexpr int kVjpThreads = 256;

// {w_s, a_s, b_s, q_s} of line s at column x
template <bool XDEP>
__device__ __forceinline__ float4 line_wabq(const ProbDesc& p, int x, int s) {
  if constexpr (XDEP) return xcol_at(p, x, s);
  else return make_float4(p.lp.w[s], p.lp.a[s], p.lp.b[s], p.lp.q[s]);
}

template <bool XDEP>
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
    const float4 c = line_wabq<XDEP>(p, x, s);
    const float I = c.x * expf(-c.y * av);
    const float bs = c.z;
    const float ux = bs * gxs, uy = bs * gys;
    // cell and in-cell position as the splat forms them
    const float dx = __builtin_amdgcn_fractf(ux), dy = __builtin_amdgcn_fractf(uy);
    const int x0 = x + floor_to_int(ux), y0 = y + floor_to_int(uy);
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
    sa -= c.y * I * gI;
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

// gphi = D_x^T Gx + D_y^T Gy, or (accumulate) that added to gphi.
__global__ __launch_bounds__(kVjpThreads) void k_vjp_transpose(KArgs a,
                                                               const float* __restrict__ Gx,
                                                               const float* __restrict__ Gy,
                                                               float* __restrict__ gphi,
                                                               int accumulate) {
  const ProbDesc& p = a.p;
  const int nx = p.nx, ny = p.ny;
  const int i = blockIdx.x * kVjpThreads + threadIdx.x;
  if (i >= nx * ny) return;
  const int y = i / nx, x = i - y * nx;
  const float* rowx = Gx + (size_t)y * nx;
  const float tx = d_transpose([&](int k) { return rowx[k]; }, x, nx);
  const float ty = d_transpose([&](int k) { return Gy[(size_t)k * nx + x]; }, y, ny);
  gphi[i] = accumulate ? gphi[i] + (tx + ty) : tx + ty;
}

// ---------------------------------------------------------------------------------------------
// Local closures (Eq. 1) and the diffraction-pressure term of the second-order non-local model.
// Per line s, with u = b_s D Y, I = w_s exp(-a_s X), A = sqrt(I), Q = (D_x D_x A + D_y D_y A) / A,
// k = D^T G and h_ab = the transpose of D_a D_b applied to G (G = dL/dP, common to all lines):
//   first order    dI = G - (u_x k_x + u_y k_y),      du_x = -I k_x,  du_y = -I k_y
//   second order   dI += 1/2 (u_x^2 h_xx + u_x u_y (h_xy + h_yx) + u_y^2 h_yy)
//                  du_x += 1/2 I (2 u_x h_xx + u_y (h_xy + h_yx)),  du_y likewise
//   pressure       dI += -q_s (D_x Q k_x + D_y Q k_y)
//                  dQ = -q_s (D_x^T(I k_x) + D_y^T(I k_y)),  t = dQ / A
//                  dI += (lap^T t - t Q) / (2 A)
// then grad_A += -a_s I dI and G_x += b_s du_x, G_y += b_s du_y (grad_phi = D_x^T G_x + D_y^T G_y
// by k_vjp_transpose).  The pressure part takes three passes over per-line planes: A, then Q
// (D D A), then t (which replaces A).
// ---------------------------------------------------------------------------------------------

// D along one axis of length n applied to the sequence at(.) at index j.
template <class F>
__device__ __forceinline__ float d_apply(F at, int j, int n) {
  if (j == 0) return at(1) - at(0);
  if (j == n - 1) return at(n - 1) - at(n - 2);
  return 0.5f * (at(j + 1) - at(j - 1));
}

// I_s at a pixel of column x whose map value is xv
template <bool XDEP>
__device__ __forceinline__ float line_intensity(const ProbDesc& p, int x, int s, float xv) {
  const float4 c = line_wabq<XDEP>(p, x, s);
  return c.x * expf(-c.y * xv);
}

// A_s = sqrt(I_s) into plane s of `work` ([L][ny][nx]).
template <bool XDEP>
__global__ __launch_bounds__(kVjpThreads) void k_vjp_sqrt_i(KArgs a, float* __restrict__ work) {
  const ProbDesc& p = a.p;
  const int n = p.nx * p.ny;
  const int i = blockIdx.x * kVjpThreads + threadIdx.x;
  if (i >= n) return;
  const float xv = p.X[i];
  const int x = i % p.nx;
  for (int s = 0; s < p.lp.n; ++s) work[(size_t)s * n + i] = sqrtf(line_intensity<XDEP>(p, x, s, xv));
}

// Q_s = (D_x D_x A_s + D_y D_y A_s) / A_s from the A planes in `work`, into the planes of `q`.
__global__ __launch_bounds__(kVjpThreads) void k_vjp_q(KArgs a, const float* __restrict__ work,
                                                       float* __restrict__ q) {
  const ProbDesc& p = a.p;
  const int nx = p.nx, ny = p.ny, n = nx * ny;
  const int i = blockIdx.x * kVjpThreads + threadIdx.x;
  if (i >= n) return;
  const int y = i / nx, x = i - y * nx;
  for (int s = 0; s < p.lp.n; ++s) {
    const float* A = work + (size_t)s * n;
    const float* row = A + (size_t)y * nx;
    const float dxx = d_apply([&](int m) { return d_apply([&](int k) { return row[k]; }, m, nx); }, x, nx);
    const float dyy = d_apply([&](int m) { return d_apply([&](int k) { return A[(size_t)k * nx + x]; }, m, ny); }, y, ny);
    q[(size_t)s * n + i] = (dxx + dyy) / row[x];
  }
}

// t_s = dQ_s / A_s, dQ_s = -q_s (D_x^T(I_s k_x) + D_y^T(I_s k_y)), replacing A_s in `work`.
// (XDEP: q_s varies along x and scales the pressure term after its outer derivative, so the
// row factor is D_x^T(q_s g) and the column factor q_s(x) D_y^T g.)
template <bool XDEP>
__global__ __launch_bounds__(kVjpThreads) void k_vjp_t(KArgs a, float* __restrict__ work) {
  const ProbDesc& p = a.p;
  const int nx = p.nx, ny = p.ny, n = nx * ny;
  const int i = blockIdx.x * kVjpThreads + threadIdx.x;
  if (i >= n) return;
  const int y = i / nx, x = i - y * nx;
  const float* g = p.d;
  const float* X = p.X;
  for (int s = 0; s < p.lp.n; ++s) {
    // k_x at (y, m) and k_y at (m, x)
    const float ty = d_transpose([&](int m) {
      return line_intensity<XDEP>(p, x, s, X[(size_t)m * nx + x]) *
             d_transpose([&](int k) { return g[(size_t)k * nx + x]; }, m, ny);
    }, y, ny);
    float dq;
    if constexpr (XDEP) {
      const float tx = d_transpose([&](int m) {
        return line_intensity<XDEP>(p, m, s, X[(size_t)y * nx + m]) *
               d_transpose([&](int k) { return xcol_at(p, k, s).w * g[(size_t)y * nx + k]; }, m, nx);
      }, x, nx);
      dq = -(tx + xcol_at(p, x, s).w * ty);
    } else {
      const float tx = d_transpose([&](int m) {
        return line_intensity<XDEP>(p, m, s, X[(size_t)y * nx + m]) *
               d_transpose([&](int k) { return g[(size_t)y * nx + k]; }, m, nx);
      }, x, nx);
      dq = -p.lp.q[s] * (tx + ty);
    }
    float* A = work + (size_t)s * n;
    A[i] = dq / A[i];
  }
}

// Per-pixel gradients of every line, summed: ORDER 1 or 2 (local closures), or 3 (the pressure
// term alone, added to the transport's gradients already in gA).  `work` holds t, `q` holds Q
// (both unused for ORDER 1).
template <int ORDER, bool XDEP>
__global__ __launch_bounds__(kVjpThreads) void k_vjp_local(KArgs a, const float* __restrict__ work,
                                                           const float* __restrict__ q,
                                                           float* __restrict__ Gx,
                                                           float* __restrict__ Gy,
                                                           float* __restrict__ gA) {
  const ProbDesc& p = a.p;
  const int nx = p.nx, ny = p.ny, n = nx * ny;
  const int i = blockIdx.x * kVjpThreads + threadIdx.x;
  if (i >= n) return;
  const int y = i / nx, x = i - y * nx;
  const float* g = p.d;
  const float* grow = g + (size_t)y * nx;
  auto kxat = [&](int yy, int xx) { return d_transpose([&](int k) { return g[(size_t)yy * nx + k]; }, xx, nx); };
  auto kyat = [&](int yy, int xx) { return d_transpose([&](int k) { return g[(size_t)k * nx + xx]; }, yy, ny); };
  const float kx = d_transpose([&](int k) { return grow[k]; }, x, nx);
  const float ky = kyat(y, x);
  float hxx = 0.f, hyy = 0.f, hxy = 0.f, hyx = 0.f;
  if (ORDER == 2) {
    hxx = d_transpose([&](int m) { return kxat(y, m); }, x, nx);
    hyy = d_transpose([&](int m) { return kyat(m, x); }, y, ny);
    hxy = d_transpose([&](int m) { return kxat(m, x); }, y, ny);   // transpose of D_x D_y
    hyx = d_transpose([&](int m) { return kyat(y, m); }, x, nx);   // transpose of D_y D_x
  }
  float px = 0.f, py = 0.f;
  if (ORDER != 3) {
    px = d_x(G(p.Y), y, x, nx);
    py = d_y(G(p.Y), y, x, ny, nx);
  }
  const float xv = p.X[i];
  float sa = 0.f, sx = 0.f, sy = 0.f;
  for (int s = 0; s < p.lp.n; ++s) {
    const float4 c = line_wabq<XDEP>(p, x, s);
    const float I = c.x * expf(-c.y * xv);
    float dI = 0.f;
    if (ORDER != 3) {
      const float bs = c.z;
      const float ux = bs * px, uy = bs * py;
      dI = g[i] - (ux * kx + uy * ky);
      float dux = -I * kx, duy = -I * ky;
      if (ORDER == 2) {
        const float hm = hxy + hyx;
        dI += 0.5f * (ux * ux * hxx + ux * uy * hm + uy * uy * hyy);
        dux += 0.5f * I * (2.f * ux * hxx + uy * hm);
        duy += 0.5f * I * (ux * hm + 2.f * uy * hyy);
      }
      sx += bs * dux;
      sy += bs * duy;
    }
    if (ORDER >= 2) {
      const float* Qs = q + (size_t)s * n;
      const float* T = work + (size_t)s * n;
      const float dqx = d_x(G(Qs), y, x, nx), dqy = d_y(G(Qs), y, x, ny, nx);
      if constexpr (XDEP) {
        const float kqx = d_transpose([&](int k) { return xcol_at(p, k, s).w * grow[k]; }, x, nx);
        dI += -(dqx * kqx + dqy * (c.w * ky));
      } else {
        dI += -c.w * (dqx * kx + dqy * ky);
      }
      const float* trow = T + (size_t)y * nx;
      const float ltx = d_transpose([&](int m) { return d_transpose([&](int k) { return trow[k]; }, m, nx); }, x, nx);
      const float lty = d_transpose([&](int m) { return d_transpose([&](int k) { return T[(size_t)k * nx + x]; }, m, ny); }, y, ny);
      dI += (ltx + lty - trow[x] * Qs[i]) / (2.f * sqrtf(I));
    }
    sa -= c.y * I * dI;
  }
  if (ORDER == 3) {
    gA[i] += sa;
  } else {
    gA[i] = sa;
    Gx[i] = sx;
    Gy[i] = sy;
  }
}

template <bool XDEP>
hipError_t launch_vjp_local_t(const KArgs& a, int total_blocks, hipStream_t s, int order,
                              float* work, float* q, float* gx, float* gy, float* ga) {
  const dim3 grid(total_blocks), block(kVjpThreads);
  if (order >= 2) {
    hipLaunchKernelGGL(k_vjp_sqrt_i<XDEP>, grid, block, 0, s, a, work);
    hipLaunchKernelGGL(k_vjp_q, grid, block, 0, s, a, work, q);
    hipLaunchKernelGGL(k_vjp_t<XDEP>, grid, block, 0, s, a, work);
  }
  if (order == 1)
    hipLaunchKernelGGL((k_vjp_local<1, XDEP>), grid, block, 0, s, a, work, q, gx, gy, ga);
  else if (order == 2)
    hipLaunchKernelGGL((k_vjp_local<2, XDEP>), grid, block, 0, s, a, work, q, gx, gy, ga);
  else
    hipLaunchKernelGGL((k_vjp_local<3, XDEP>), grid, block, 0, s, a, work, q, gx, gy, ga);
  return hipGetLastError();
}

hipError_t launch_vjp_local(const KArgs& a, int total_blocks, hipStream_t s, int order,
                            float* work, float* q, float* gx, float* gy, float* ga) {
  return a.p.xcol ? launch_vjp_local_t<true>(a, total_blocks, s, order, work, q, gx, gy, ga)
                  : launch_vjp_local_t<false>(a, total_blocks, s, order, work, q, gx, gy, ga);
}

hipError_t launch_vjp(const KArgs& a, int total_blocks, size_t, hipStream_t s, float* gx,
                      float* gy, float* ga) {
  if (a.p.xcol)
    hipLaunchKernelGGL(k_vjp<true>, dim3(total_blocks), dim3(kVjpThreads), 0, s, a, gx, gy, ga);
  else
    hipLaunchKernelGGL(k_vjp<false>, dim3(total_blocks), dim3(kVjpThreads), 0, s, a, gx, gy, ga);
  return hipGetLastError();
}

hipError_t launch_vjp_transpose(const KArgs& a, int total_blocks, hipStream_t s,
                                const float* gx, const float* gy, float* gphase,
                                int accumulate) {
  hipLaunchKernelGGL(k_vjp_transpose, dim3(total_blocks), dim3(kVjpThreads), 0, s, a, gx, gy,
                     gphase, accumulate);
  return hipGetLastError();
}

hipError_t set_vjp_attributes() { return hipSuccess; }

}  // namespace epr
