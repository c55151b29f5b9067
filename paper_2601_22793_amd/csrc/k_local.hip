// Local O(L^2) closure (Eq. 1, Methods 4.1) with the fused spectral sum, residual and split.
//
// Per line s, with u = b_s D Y (pixels), I = w_s exp(-a_s X), A = sqrt(I):
//   P_s = I - [D_x(I u_x) + D_y(I u_y)]
//       + 1/2 [D_x D_x(I u_x^2) + D_x D_y(I u_x u_y) + D_y D_x(I u_y u_x) + D_y D_y(I u_y^2)]
//       - q_s [D_x(I D_x Q) + D_y(I D_y Q)],     Q = (D_x D_x A + D_y D_y A) / A,
// with D the central difference inside the image and the one-sided difference on its edges,
// exactly as the composition of derivatives is written in Eq. 1.  Order 1 keeps the first
// bracket only.  Order 3 is the second-order non-local model: the transported prediction
// M_s[I_s], already in e (the splat's per-line output), plus the diffraction-pressure term.  A workgroup owns a 16 x 16 output tile and evaluates the nested derivatives
// on shrinking squares of a 24 x 24 LDS region (halo 4: Q needs A two pixels further out than
// the outer derivative of the diffraction-pressure term, which is one pixel out).
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "epr_internal.h"

namespace epr {

constexpr int kLT = kLocalTile;
constexpr int kLH = kLocalHalo;
constexpr int kLR = kLT + 2 * kLH;  // region side (24)
constexpr int kLN = kLR * kLR;
constexpr int kLocalThreads = 256;

// D along x / y of a region field at region point (ly, lx) whose image coordinate is (y, x).
__device__ __forceinline__ float rdx(const float* F, int ly, int lx, int x, int nx) {
  const float* row = F + ly * kLR;
  if (x == 0) return row[lx + 1] - row[lx];
  if (x == nx - 1) return row[lx] - row[lx - 1];
  return 0.5f * (row[lx + 1] - row[lx - 1]);
}
__device__ __forceinline__ float rdy(const float* F, int ly, int lx, int y, int ny) {
  if (y == 0) return F[(ly + 1) * kLR + lx] - F[ly * kLR + lx];
  if (y == ny - 1) return F[ly * kLR + lx] - F[(ly - 1) * kLR + lx];
  return 0.5f * (F[(ly + 1) * kLR + lx] - F[(ly - 1) * kLR + lx]);
}

// Iterate over the region points at halo level <= h that lie inside the image.
#define FOR_LEVEL(h, BODY)                                                   \
  {                                                                          \
    const int side_ = kLT + 2 * (h);                                         \
    for (int i_ = threadIdx.x; i_ < side_ * side_; i_ += kLocalThreads) {     \
      const int ly = kLH - (h) + i_ / side_;                                 \
      const int lx = kLH - (h) + i_ % side_;                                 \
      const int y = ry0 + ly, x = rx0 + lx;                                  \
      if (y < 0 || y >= ny || x < 0 || x >= nx) continue;                    \
      const int o = ly * kLR + lx;                                           \
      BODY                                                                   \
    }                                                                        \
    __syncthreads();                                                         \
  }

// XDEP: x-dependent spectrum, every line constant is read at the point's column.
template <bool XDEP>
__device__ __forceinline__ void local_body(const ProbDesc& p, int local, int mode, int order) {
  extern __shared__ float sm[];
  float* fI = sm;
  float* fA = fI + kLN;
  float* fDxA = fA + kLN;
  float* fDyA = fDxA + kLN;
  float* fQ = fDyA + kLN;
  float* fIx = fQ + kLN;
  float* fIy = fIx + kLN;
  float* fPxx = fIy + kLN;
  float* fPxy = fPxx + kLN;
  float* fPyy = fPxy + kLN;
  float* fGx = fPyy + kLN;
  float* fGy = fGx + kLN;
  float* fFxx = fGy + kLN;
  float* fFxy = fFxx + kLN;
  float* fFyx = fFxy + kLN;
  float* fFyy = fFyx + kLN;
  float* Pl = fFyy + kLN;  // [L][kLT][kLT]

  const int nx = p.nx, ny = p.ny, L = p.lp.n;
  const int ntx = (nx + kLT - 1) / kLT;
  const int ty0 = (local / ntx) * kLT, tx0 = (local - (local / ntx) * ntx) * kLT;
  const int ry0 = ty0 - kLH, rx0 = tx0 - kLH;
  gptr<const float> X = G(p.X);
  gptr<const float> Y = G(p.Y);

  for (int s = 0; s < L; ++s) {
    const float ws = p.lp.w[s], as = p.lp.a[s], bs = p.lp.b[s], qs = p.lp.q[s];
    // level 4: I and A
    FOR_LEVEL(kLH, {
      float cw = ws;
      float ca = as;
      if constexpr (XDEP) {
        const float4 c = xcol_at(p, x, s);
        cw = c.x;
        ca = c.y;
      }
      const float I = cw * expf(-ca * X[(size_t)y * nx + x]);
      fI[o] = I;
      fA[o] = sqrtf(I);
    })
    // level 3: D A
    FOR_LEVEL(3, {
      fDxA[o] = rdx(fA, ly, lx, x, nx);
      fDyA[o] = rdy(fA, ly, lx, y, ny);
    })
    // level 2: Q and the transport products
    FOR_LEVEL(2, {
      const float I = fI[o];
      float cb = bs;
      if constexpr (XDEP) cb = xcol_at(p, x, s).z;
      const float ux = cb * d_x(Y, y, x, nx);
      const float uy = cb * d_y(Y, y, x, ny, nx);
      fIx[o] = I * ux;
      fIy[o] = I * uy;
      fPxx[o] = I * ux * ux;
      fPxy[o] = I * ux * uy;
      fPyy[o] = I * uy * uy;
      fQ[o] = (rdx(fDxA, ly, lx, x, nx) + rdy(fDyA, ly, lx, y, ny)) / fA[o];
    })
    // level 1: first derivatives of the second-order products, I D Q
    FOR_LEVEL(1, {
      fFxx[o] = rdx(fPxx, ly, lx, x, nx);
      fFxy[o] = rdy(fPxy, ly, lx, y, ny);
      fFyx[o] = rdx(fPxy, ly, lx, x, nx);
      fFyy[o] = rdy(fPyy, ly, lx, y, ny);
      const float I = fI[o];
      fGx[o] = I * rdx(fQ, ly, lx, x, nx);
      fGy[o] = I * rdy(fQ, ly, lx, y, ny);
    })
    // level 0: the closure
    FOR_LEVEL(0, {
      float P;
      float cq = qs;
      if constexpr (XDEP) cq = xcol_at(p, x, s).w;
      if (order == kOrderTransportWkb1) {
        const float t3 = rdx(fGx, ly, lx, x, nx) + rdy(fGy, ly, lx, y, ny);
        P = G(p.e)[((size_t)s * ny + y) * nx + x] - cq * t3;
      } else {
      const float t1 = rdx(fIx, ly, lx, x, nx) + rdy(fIy, ly, lx, y, ny);
      P = fI[o] - t1;
      if (order >= 2) {
        const float t2 = rdx(fFxx, ly, lx, x, nx) + rdx(fFxy, ly, lx, x, nx) +
                         rdy(fFyx, ly, lx, y, ny) + rdy(fFyy, ly, lx, y, ny);
        const float t3 = rdx(fGx, ly, lx, x, nx) + rdy(fGy, ly, lx, y, ny);
        P += 0.5f * t2 - cq * t3;
      }
      }
      Pl[(s * kLT + (ly - kLH)) * kLT + (lx - kLH)] = P;
    })
  }

  float se = 0.f, sd = 0.f;
  for (int i = threadIdx.x; i < kLT * kLT; i += kLocalThreads) {
    const int ly = i / kLT, lx = i - ly * kLT;
    const int y = ty0 + ly, x = tx0 + lx;
    if (y >= ny || x >= nx) continue;
    const size_t pix = (size_t)y * nx + x;
    float P = 0.f, S = 0.f;
    for (int s = 0; s < L; ++s) {
      const float v = Pl[s * kLT * kLT + i];
      P += v;
      S += fmaxf(v, 0.f);
    }
    if (mode == kLocalForward) {
      G(p.out)[pix] = P;
    } else if (mode == kLocalLines) {
      for (int s = 0; s < L; ++s) G(p.e)[(size_t)s * nx * ny + pix] = Pl[s * kLT * kLT + i];
    } else {
      const float dv = G(p.d)[pix];
      const float e = dv - P;
      se += e * e;
      sd += dv * dv;
      const bool hole = !(S > 1e-30f);
      const float inv = hole ? 0.f : 1.f / S;
      for (int s = 0; s < L; ++s) {
        float fw = p.lp.w[s];
        if constexpr (XDEP) fw = xcol_at(p, x, s).x;
        const float share = hole ? fw : fmaxf(Pl[s * kLT * kLT + i], 0.f) * inv;
        G(p.e)[(size_t)s * nx * ny + pix] = share * e;
      }
    }
  }
  if (mode == kLocalSplit && p.resid != nullptr) {
    __shared__ float red[2][kLocalThreads / 64];
    se = wave_sum(se);
    sd = wave_sum(sd);
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = se;
      red[1][threadIdx.x >> 6] = sd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float te = 0.f, td = 0.f;
      for (int w = 0; w < kLocalThreads / 64; ++w) {
        te += red[0][w];
        td += red[1][w];
      }
      G(p.resid)[2 * local] = te;
      G(p.resid)[2 * local + 1] = td;
    }
  }
}

template <bool B>
__global__ __launch_bounds__(kLocalThreads) void k_local(KArgs a,
                                                         const ProbDesc* __restrict__ table,
                                                         int order) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), local_body<false>, a.mode, order);
}
// x-dependent spectrum
template <bool B>
__global__ __launch_bounds__(kLocalThreads) void k_local_x(KArgs a,
                                                           const ProbDesc* __restrict__ table,
                                                           int order) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), local_body<true>, a.mode, order);
}

hipError_t launch_local(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, int order) {
  if (a.xdep && a.table)
    hipLaunchKernelGGL(k_local_x<true>, dim3(total_blocks), dim3(kLocalThreads), lds, s, a,
                       a.table, order);
  else if (a.table)
    hipLaunchKernelGGL(k_local<true>, dim3(total_blocks), dim3(kLocalThreads), lds, s, a, a.table,
                       order);
  else if (a.p.xcol)
    hipLaunchKernelGGL(k_local_x<false>, dim3(total_blocks), dim3(kLocalThreads), lds, s, a,
                       a.table, order);
  else
    hipLaunchKernelGGL(k_local<false>, dim3(total_blocks), dim3(kLocalThreads), lds, s, a, a.table,
                       order);
  return hipGetLastError();
}

size_t lds_local(int n_lines) {
  return sizeof(float) * ((size_t)16 * kLN + (size_t)n_lines * kLT * kLT);
}

hipError_t set_local_attributes() {
  const int mx = 160 * 1024 - 64;
  for (const void* f : {(const void*)k_local<false>, (const void*)k_local<true>,
                        (const void*)k_local_x<false>, (const void*)k_local_x<true>}) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace epr
