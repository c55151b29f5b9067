// Spectral kernels: back-transport + row real FFT, column FFT with the fused Paganin-type
// filter (Section 2), and row inverse real FFT with the fused update and single-thickness
// projection (Methods 4.4, Eq. 7).
//
// Real transforms of length nx use the half-length complex trick: z[m] = r[2m] + i r[2m+1],
// Z = FFT_{nx/2}(z), X[k] = (Z[k] + conj Z[M-k])/2 - i W^k (Z[k] - conj Z[M-k])/2 with
// W = exp(-2 pi i / nx), and the mirror relation for the inverse.  All transforms are
// unnormalised; the product of their gains (ny * nx/2) is removed by the filter's scale.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "epr_internal.h"
#include "fft_lds.h"

namespace epr {

constexpr int kRowEmax = kRows * (kMaxDim / 2);  // complex elements of a row-block FFT
constexpr int kColEmax = kColBlock * kMaxDim;    // complex elements of a column-block FFT

// Bilinear interpolation of e at (x + ux, y + uy) with zeros off the grid (Eq. 4).
__device__ __forceinline__ float interp_zero(const float* __restrict__ e, int ny, int nx, int y,
                                             int x, float ux, float uy) {
  const float fx = floorf(ux), fy = floorf(uy);
  const float dx = ux - fx, dy = uy - fy;
  const int x0 = x + (int)fx, y0 = y + (int)fy;
  float v00 = 0.f, v01 = 0.f, v10 = 0.f, v11 = 0.f;
  const bool xin0 = x0 >= 0 && x0 < nx, xin1 = x0 + 1 >= 0 && x0 + 1 < nx;
  if (y0 >= 0 && y0 < ny) {
    const float* row = e + (size_t)y0 * nx;
    if (xin0) v00 = row[x0];
    if (xin1) v10 = row[x0 + 1];
  }
  if (y0 + 1 >= 0 && y0 + 1 < ny) {
    const float* row = e + (size_t)(y0 + 1) * nx;
    if (xin0) v01 = row[x0];
    if (xin1) v11 = row[x0 + 1];
  }
  // w00 v(y0,x0) + w10 v(y0,x0+1) + w01 v(y0+1,x0) + w11 v(y0+1,x0+1)
  return (1.f - dy) * ((1.f - dx) * v00 + dx * v10) + dy * ((1.f - dx) * v01 + dx * v11);
}

// ---------------------------------------------------------------------------------------------
// Row pass: per (line s, block of kRows rows) compute r_s (gather of e_s at the mapped points,
// or a copy of e_s), then the real FFT of each row, stored as column blocks of the half
// spectrum.  In gather-only mode r_s goes to p.out and no transform is done (epr_adjoint).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void rowfft_body(const ProbDesc& p, int local, int mode) {
  extern __shared__ float2 buf[];
  const int nx = p.nx, ny = p.ny, M = nx >> 1;
  const int nrb = (ny + kRows - 1) / kRows;
  const int s = local / nrb;
  const int y0 = (local - s * nrb) * kRows;
  const float* __restrict__ es = p.e + (size_t)s * nx * ny;
  const float* __restrict__ Y = p.Y;
  const float bs = p.lp.b[s];
  float* fb = reinterpret_cast<float*>(buf);

  for (int i = threadIdx.x; i < kRows * nx; i += kFftThreads) {
    const int r = i / nx, x = i - r * nx, y = y0 + r;
    float v = 0.f;
    if (y < ny) {
      if (mode == kRowCopyFft) {
        v = es[(size_t)y * nx + x];
      } else {
        const float ux = bs * d_x(Y, y, x, nx);
        const float uy = bs * d_y(Y, y, x, ny, nx);
        v = interp_zero(es, ny, nx, y, x, ux, uy);
      }
      if (mode == kRowGatherOnly) p.out[(size_t)s * nx * ny + (size_t)y * nx + x] = v;
    }
    fb[(((x >> 1) * kRows + r) << 1) + (x & 1)] = v;
  }
  if (mode == kRowGatherOnly) return;
  __syncthreads();
  fft_lds<kFftThreads, kRowEmax>(buf, kRows, p.row);

  const float2* __restrict__ W = p.row_tw;
  float2* __restrict__ out = p.spec + (size_t)s * p.nblk * ny * kColBlock;
  const int nout = p.nblk * kColBlock * kRows;
  for (int i = threadIdx.x; i < nout; i += kFftThreads) {
    const int c = i % kColBlock;
    const int r = (i / kColBlock) % kRows;
    const int blk = i / (kColBlock * kRows);
    const int k = blk * kColBlock + c;
    const int y = y0 + r;
    if (y >= ny) continue;
    float2 X = make_float2(0.f, 0.f);
    if (k <= M) {
      const float2 zk = buf[(k == M ? 0 : k) * kRows + r];
      const float2 zm = cconj(buf[(k == 0 ? 0 : M - k) * kRows + r]);
      const float2 A = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
      const float2 B = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y - zm.y));
      const float2 WB = cmul(W[k], B);  // the table holds W^k for k < nx, so W^M = -1 too
      X = make_float2(A.x + WB.y, A.y - WB.x);  // X = A - i W B
    }
    out[((size_t)blk * ny + y) * kColBlock + c] = X;
  }
}

template <bool B>
__global__ __launch_bounds__(kFftThreads) void k_rowfft(KArgs a) {
  EPR_DISPATCH(B, a, xcd_remap(blockIdx.x, gridDim.x), rowfft_body, a.mode);
}

// ---------------------------------------------------------------------------------------------
// Column pass: per (line s, block of kColBlock frequencies) forward FFT along y, multiply by
// scale / (1 + h_s (fx^2 + fy^2)), inverse FFT along y (via conjugation), in place.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void colfft_body(const ProbDesc& p, int local, int) {
  extern __shared__ float2 buf[];
  const int ny = p.ny, nx = p.nx;
  const int s = local / p.nblk;
  const int blk = local - s * p.nblk;
  float2* __restrict__ g = p.spec + ((size_t)s * p.nblk + blk) * ny * kColBlock;
  const int n = ny * kColBlock;
  {
    const float4* __restrict__ g4 = reinterpret_cast<const float4*>(g);
    float4* b4 = reinterpret_cast<float4*>(buf);
    for (int i = threadIdx.x; i < n / 2; i += kFftThreads) b4[i] = g4[i];
  }
  __syncthreads();
  fft_lds<kFftThreads, kColEmax>(buf, kColBlock, p.col);

  const float hs = p.lp.h[s];
  const float scale = p.lp.spec_scale;
  const float inv_ny = 1.f / (float)ny, inv_nx = 1.f / (float)nx;
  for (int i = threadIdx.x; i < n; i += kFftThreads) {
    const int j = i / kColBlock;
    const int c = i - j * kColBlock;
    const float fy = (float)(j <= (ny >> 1) ? j : j - ny) * inv_ny;
    const float fx = (float)(blk * kColBlock + c) * inv_nx;
    const float H = scale / (1.f + hs * (fx * fx + fy * fy));
    const float2 v = buf[i];
    buf[i] = make_float2(v.x * H, -v.y * H);
  }
  __syncthreads();
  fft_lds<kFftThreads, kColEmax>(buf, kColBlock, p.col);
  {
    float4* __restrict__ g4 = reinterpret_cast<float4*>(g);
    const float4* b4 = reinterpret_cast<const float4*>(buf);
    for (int i = threadIdx.x; i < n / 2; i += kFftThreads) {
      const float4 v = b4[i];
      g4[i] = make_float4(v.x, -v.y, v.z, -v.w);
    }
  }
}

template <bool B>
__global__ __launch_bounds__(kFftThreads) void k_colfft(KArgs a) {
  EPR_DISPATCH(B, a, xcd_remap(blockIdx.x, gridDim.x), colfft_body, 0);
}

// ---------------------------------------------------------------------------------------------
// Row inverse pass: per block of kRows rows, for every line: inverse real FFT of the filtered
// half spectrum -> dI_s; then either write dI_s (precondition mode) or accumulate the
// projection of I_s + omega dI_s onto one thickness (solve mode) and write tau.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void rowinv_body(const ProbDesc& p, int local, int mode) {
  extern __shared__ float2 buf[];
  const int nx = p.nx, ny = p.ny, M = nx >> 1;
  const int y0 = local * kRows;
  const int L = p.lp.n;
  const int npix = kRows * nx;
  const bool solve = mode == kRowInvSolve;
  const float2* __restrict__ W = p.row_tw;
  // projection accumulators live in LDS after the transform buffer
  float* acc = reinterpret_cast<float*>(buf + kRows * (M + 1));
  if (solve)
    for (int i = threadIdx.x; i < npix; i += kFftThreads) acc[i] = 0.f;

  for (int s = 0; s < L; ++s) {
    const float2* __restrict__ sp = p.spec + (size_t)s * p.nblk * ny * kColBlock;
    const int nin = p.nblk * kColBlock * kRows;
    for (int i = threadIdx.x; i < nin; i += kFftThreads) {
      const int c = i % kColBlock;
      const int r = (i / kColBlock) % kRows;
      const int blk = i / (kColBlock * kRows);
      const int k = blk * kColBlock + c;
      const int y = y0 + r;
      if (k > M) continue;
      buf[k * kRows + r] = (y < ny) ? sp[((size_t)blk * ny + y) * kColBlock + c]
                                    : make_float2(0.f, 0.f);
    }
    __syncthreads();
    // Z[k] = E_k + i O_k, E_k = (X_k + conj X_{M-k})/2, O_k = (X_k - conj X_{M-k})/2 W^-k;
    // store conj(Z) so that a forward FFT followed by conjugation inverts it.
    const int half = M >> 1;
    for (int i = threadIdx.x; i < (half + 1) * kRows; i += kFftThreads) {
      const int k = i / kRows, r = i - k * kRows;
      const float2 xk = buf[k * kRows + r];
      const float2 xm = buf[(M - k) * kRows + r];
      {
        const float2 xmc = cconj(xm);
        const float2 E = make_float2(0.5f * (xk.x + xmc.x), 0.5f * (xk.y + xmc.y));
        const float2 D = make_float2(0.5f * (xk.x - xmc.x), 0.5f * (xk.y - xmc.y));
        const float2 O = cmul(D, cconj(W[k]));
        const float2 Z = make_float2(E.x - O.y, E.y + O.x);
        buf[k * kRows + r] = cconj(Z);
      }
      if (k != 0 && 2 * k != M) {
        const float2 xkc = cconj(xk);
        const float2 E = make_float2(0.5f * (xm.x + xkc.x), 0.5f * (xm.y + xkc.y));
        const float2 D = make_float2(0.5f * (xm.x - xkc.x), 0.5f * (xm.y - xkc.y));
        const float2 O = cmul(D, cconj(W[M - k]));
        const float2 Z = make_float2(E.x - O.y, E.y + O.x);
        buf[(M - k) * kRows + r] = cconj(Z);
      }
    }
    __syncthreads();
    fft_lds<kFftThreads, kRowEmax>(buf, kRows, p.row);

    const float ws = p.lp.w[s], as = p.lp.a[s], mws = p.lp.mw[s];
    const float invw = p.lp.inv_w[s], fl = p.lp.floor_[s], om = p.relax;
    const float* fb = reinterpret_cast<const float*>(buf);
    for (int i = threadIdx.x; i < npix; i += kFftThreads) {
      const int r = i / nx, x = i - r * nx, y = y0 + r;
      if (y >= ny) continue;
      const float v = fb[(((x >> 1) * kRows + r) << 1) + (x & 1)];
      const float dI = (x & 1) ? -v : v;  // conj of the transform output
      if (solve) {
        const float I = ws * expf(-as * p.tau[(size_t)y * nx + x]);
        const float It = fmaxf(I + om * dI, fl);
        acc[i] += mws * logf(It * invw);
      } else {
        p.out[(size_t)s * nx * ny + (size_t)y * nx + x] = dI;
      }
    }
    __syncthreads();
  }

  if (solve) {
    const float inv_den = p.lp.inv_den, pc = p.lp.phase_coef;
    for (int i = threadIdx.x; i < npix; i += kFftThreads) {
      const int r = i / nx, x = i - r * nx, y = y0 + r;
      if (y >= ny) continue;
      const float t = -acc[i] * inv_den;
      p.tau[(size_t)y * nx + x] = t;
      if (p.phase_out) p.phase_out[(size_t)y * nx + x] = pc * t;
    }
  }
}

template <bool B>
__global__ __launch_bounds__(kFftThreads) void k_rowinv(KArgs a) {
  EPR_DISPATCH(B, a, xcd_remap(blockIdx.x, gridDim.x), rowinv_body, a.mode);
}

#define EPR_LAUNCH2(K, a, grid, block, lds, s)                                   \
  do {                                                                            \
    if ((a).table)                                                                \
      hipLaunchKernelGGL(K<true>, dim3(grid), dim3(block), lds, s, a);            \
    else                                                                          \
      hipLaunchKernelGGL(K<false>, dim3(grid), dim3(block), lds, s, a);           \
  } while (0)

hipError_t launch_rowfft(const KArgs& a, int total_blocks, size_t lds, hipStream_t s) {
  EPR_LAUNCH2(k_rowfft, a, total_blocks, kFftThreads, lds, s);
  return hipGetLastError();
}
hipError_t launch_colfft(const KArgs& a, int total_blocks, size_t lds, hipStream_t s) {
  EPR_LAUNCH2(k_colfft, a, total_blocks, kFftThreads, lds, s);
  return hipGetLastError();
}
hipError_t launch_rowinv(const KArgs& a, int total_blocks, size_t lds, hipStream_t s) {
  EPR_LAUNCH2(k_rowinv, a, total_blocks, kFftThreads, lds, s);
  return hipGetLastError();
}

hipError_t set_spectral_attributes() {
  const int mx = 160 * 1024 - 64;
  const void* fns[] = {(const void*)k_rowfft<false>, (const void*)k_rowfft<true>,
                       (const void*)k_colfft<false>, (const void*)k_colfft<true>,
                       (const void*)k_rowinv<false>, (const void*)k_rowinv<true>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace epr
