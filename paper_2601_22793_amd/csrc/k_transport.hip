// Non-local transport kernels (Methods 4.2): max-shift reduction, the LDS-tiled conservative
// bilinear splat with the fused spectral sum / residual / split (Eq. 5, Methods 4.4), and the
// residual-norm reduction.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "epr_internal.h"

namespace epr {

// ---------------------------------------------------------------------------------------------
// max |D_x Y| and max |D_y Y| over the image: one partial pair per workgroup.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void maxgrad_body(const ProbDesc& p, int local, int) {
  const int nx = p.nx, ny = p.ny;
  const int n = nx * ny;
  const float* __restrict__ Y = p.Y;
  float mx = 0.f, my = 0.f;
  for (int i = local * 256 + threadIdx.x; i < n; i += kMaxgBlocks * 256) {
    const int y = i / nx, x = i - y * nx;
    mx = fmaxf(mx, fabsf(d_x(Y, y, x, nx)));
    my = fmaxf(my, fabsf(d_y(Y, y, x, ny, nx)));
  }
  __shared__ float red[2][4];
  mx = wave_max(mx);
  my = wave_max(my);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = mx;
    red[1][w] = my;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    p.maxg[2 * local] = fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3]));
    p.maxg[2 * local + 1] = fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3]));
  }
}

template <bool B>
__global__ __launch_bounds__(256) void k_maxgrad(KArgs a) {
  EPR_DISPATCH(B, a, blockIdx.x, maxgrad_body, 0);
}

// ---------------------------------------------------------------------------------------------
// Splat.  A workgroup owns a TY x TX tile of the detector and accumulates, for every line, the
// bilinear deposits of all sources whose mapped footprint can reach the tile (sources within
// the halo H derived on the device from the max-gradient partials) in LDS with LDS atomics.
// Each detector pixel is written by exactly one workgroup: no global atomics.
//   forward mode: out = sum_s P_s
//   split mode  : e = d - sum_s P_s, e_s = pi_s e with pi_s = max(P_s,0)/sum max(P_s',0)
//                 (w_s where that sum is zero), written to e[s]; optional residual partials.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void splat_body(const ProbDesc& p, int local, int mode) {
  extern __shared__ float acc[];
  __shared__ float red[2][kSplatThreads / 64];
  const int nx = p.nx, ny = p.ny;
  const int TX = p.splat_tx, TY = p.splat_ty;
  const int L = p.lp.n;
  const int ntx = (nx + TX - 1) / TX;
  const int ty0 = (local / ntx) * TY;
  const int tx0 = (local - (local / ntx) * ntx) * TX;
  const int tid = threadIdx.x;
  const int tile = TX * TY;

  // halo from the max-gradient partials
  float gx = 0.f, gy = 0.f;
  for (int i = tid; i < kMaxgBlocks; i += kSplatThreads) {
    gx = fmaxf(gx, p.maxg[2 * i]);
    gy = fmaxf(gy, p.maxg[2 * i + 1]);
  }
  gx = wave_max(gx);
  gy = wave_max(gy);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = gx;
    red[1][tid >> 6] = gy;
  }
  for (int i = tid; i < L * tile; i += kSplatThreads) acc[i] = 0.f;
  __syncthreads();
  gx = red[0][0];
  gy = red[1][0];
#pragma unroll
  for (int w = 1; w < kSplatThreads / 64; ++w) {
    gx = fmaxf(gx, red[0][w]);
    gy = fmaxf(gy, red[1][w]);
  }
  const int hx = halo_from(p.lp.b_absmax, gx);
  const int hy = halo_from(p.lp.b_absmax, gy);

  const int sy0 = max(ty0 - hy, 0), sy1 = min(ty0 + TY - 1 + hy, ny - 1);
  const int sx0 = max(tx0 - hx, 0), sx1 = min(tx0 + TX - 1 + hx, nx - 1);
  const int wsrc = sx1 - sx0 + 1;
  const int nsrc = wsrc * (sy1 - sy0 + 1);
  const float* __restrict__ X = p.X;
  const float* __restrict__ Y = p.Y;

  for (int i = tid; i < nsrc; i += kSplatThreads) {
    const int r = i / wsrc;
    const int sy = sy0 + r, sx = sx0 + (i - r * wsrc);
    const float gxs = d_x(Y, sy, sx, nx);
    const float gys = d_y(Y, sy, sx, ny, nx);
    const float xv = X[(size_t)sy * nx + sx];
    for (int s = 0; s < L; ++s) {
      const float I = p.lp.w[s] * expf(-p.lp.a[s] * xv);
      const float ux = p.lp.b[s] * gxs, uy = p.lp.b[s] * gys;
      const float fx = floorf(ux), fy = floorf(uy);
      const float dx = ux - fx, dy = uy - fy;
      const int lx = sx + (int)fx - tx0;
      const int ly = sy + (int)fy - ty0;
      float* as = acc + s * tile;
      const float i0 = I * (1.f - dy), i1 = I * dy;
      if (ly >= 0 && ly < TY) {
        if (lx >= 0 && lx < TX) atomicAdd(&as[ly * TX + lx], i0 * (1.f - dx));
        if (lx + 1 >= 0 && lx + 1 < TX) atomicAdd(&as[ly * TX + lx + 1], i0 * dx);
      }
      if (ly + 1 >= 0 && ly + 1 < TY) {
        if (lx >= 0 && lx < TX) atomicAdd(&as[(ly + 1) * TX + lx], i1 * (1.f - dx));
        if (lx + 1 >= 0 && lx + 1 < TX) atomicAdd(&as[(ly + 1) * TX + lx + 1], i1 * dx);
      }
    }
  }
  __syncthreads();

  float se = 0.f, sd = 0.f;
  for (int i = tid; i < tile; i += kSplatThreads) {
    const int ly = i / TX, lx = i - ly * TX;
    const int y = ty0 + ly, x = tx0 + lx;
    if (y >= ny || x >= nx) continue;
    const size_t pix = (size_t)y * nx + x;
    float P = 0.f, S = 0.f;
    for (int s = 0; s < L; ++s) {
      const float v = acc[s * tile + i];
      P += v;
      S += fmaxf(v, 0.f);
    }
    if (mode == kSplatForward) {
      p.out[pix] = P;
    } else {
      const float dv = p.d[pix];
      const float e = dv - P;
      se += e * e;
      sd += dv * dv;
      const bool hole = !(S > 1e-30f);
      const float inv = hole ? 0.f : 1.f / S;
      for (int s = 0; s < L; ++s) {
        const float share = hole ? p.lp.w[s] : fmaxf(acc[s * tile + i], 0.f) * inv;
        p.e[(size_t)s * nx * ny + pix] = share * e;
      }
    }
  }
  if (mode == kSplatSplit && p.resid != nullptr) {
    __syncthreads();
    se = wave_sum(se);
    sd = wave_sum(sd);
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = se;
      red[1][tid >> 6] = sd;
    }
    __syncthreads();
    if (tid == 0) {
      float te = 0.f, td = 0.f;
      for (int w = 0; w < kSplatThreads / 64; ++w) {
        te += red[0][w];
        td += red[1][w];
      }
      p.resid[2 * local] = te;
      p.resid[2 * local + 1] = td;
    }
  }
}

template <bool B>
__global__ __launch_bounds__(kSplatThreads) void k_splat(KArgs a) {
  EPR_DISPATCH(B, a, xcd_remap(blockIdx.x, gridDim.x), splat_body, a.mode);
}

// Reduce the residual partials of problem 0 into hist_slot = ||e|| / ||d||.
__global__ __launch_bounds__(256) void k_resid_reduce(KArgs a, float* hist_slot) {
  const int nb = blocks_splat(a.p);
  const float* __restrict__ resid = a.p.resid;
  float te = 0.f, td = 0.f;
  for (int i = threadIdx.x; i < nb; i += 256) {
    te += resid[2 * i];
    td += resid[2 * i + 1];
  }
  __shared__ float red[2][4];
  te = wave_sum(te);
  td = wave_sum(td);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = te;
    red[1][threadIdx.x >> 6] = td;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    te = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    td = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    hist_slot[0] = td > 0.f ? sqrtf(te / td) : 0.f;
  }
}

hipError_t launch_maxgrad(const KArgs& a, int total_blocks, hipStream_t s) {
  if (a.table)
    hipLaunchKernelGGL(k_maxgrad<true>, dim3(total_blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_maxgrad<false>, dim3(total_blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_splat(const KArgs& a, int total_blocks, size_t lds, hipStream_t s) {
  if (a.table)
    hipLaunchKernelGGL(k_splat<true>, dim3(total_blocks), dim3(kSplatThreads), lds, s, a);
  else
    hipLaunchKernelGGL(k_splat<false>, dim3(total_blocks), dim3(kSplatThreads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_resid_reduce(const KArgs& a, float* hist_slot, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_reduce, dim3(1), dim3(256), 0, s, a, hist_slot);
  return hipGetLastError();
}

hipError_t set_transport_attributes() {
  const int mx = 160 * 1024 - 64;
  hipError_t e = hipFuncSetAttribute((const void*)k_splat<false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, mx);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_splat<true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, mx);
}

}  // namespace epr
