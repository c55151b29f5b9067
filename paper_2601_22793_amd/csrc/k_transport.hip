// Non-local transport kernels (Methods 4.2): max-shift reduction, the LDS-tiled conservative
// bilinear splat with the fused spectral sum / residual / split (Eq. 5, Methods 4.4), and the
// residual-norm reduction.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dev_common.h"
#include "epr_internal.h"

namespace epr {

// ---------------------------------------------------------------------------------------------
// max |D_x Y|, max |D_y Y| and min X over the image: one partial triple per workgroup.
// ---------------------------------------------------------------------------------------------
constexpr int kMaxgThreads = 1024;  // (a band is a few rows: many loads in flight per workgroup)

__device__ __forceinline__ void maxgrad_body(const ProbDesc& p, int local, int) {
  const int nx = p.nx, ny = p.ny;
  gptr<const float> Y = G(p.Y);
  gptr<const float> X = G(p.X);
  float mx = 0.f, my = 0.f, mn = INFINITY;
  // each workgroup takes one band of whole rows, so that the rows above and below a pixel are
  // read by the same workgroup (from its caches) rather than fetched again by others
  const int y0 = (int)(((long long)local * ny) / kMaxgBlocks);
  const int y1 = (int)(((long long)(local + 1) * ny) / kMaxgBlocks);
  if ((nx & 3) == 0 && ((reinterpret_cast<uintptr_t>(p.Y) | reinterpret_cast<uintptr_t>(p.X)) & 15) == 0) {
    // 4 consecutive pixels per item: three float4 loads (rows y-1, y, y+1) and the two
    // neighbours of the segment; clamping reproduces the one-sided edge differences
    const int nq = nx >> 2;
    const int n = nq * (y1 - y0);
    for (int i = threadIdx.x; i < n; i += kMaxgThreads) {
      const int yb = i / nq;
      const int y = y0 + yb, x = (i - yb * nq) << 2;
      const int yl = max(y - 1, 0), yh = min(y + 1, ny - 1);
      const float sy = (yh - yl == 2) ? 0.5f : 1.f;
      const float4 c = ldg((gptr<const float4>)Y, (unsigned)(__mul24(y, nx) + x) >> 2);
      const float4 u = ldg((gptr<const float4>)Y, (unsigned)(__mul24(yl, nx) + x) >> 2);
      const float4 d = ldg((gptr<const float4>)Y, (unsigned)(__mul24(yh, nx) + x) >> 2);
      const float4 xv = ldg((gptr<const float4>)X, (unsigned)(__mul24(y, nx) + x) >> 2);
      const float l = ldg(Y, (unsigned)(__mul24(y, nx) + max(x - 1, 0)));
      const float r = ldg(Y, (unsigned)(__mul24(y, nx) + min(x + 4, nx - 1)));
      // x differences: the first/last pixel of the row use one-sided differences
      const float g0 = (x == 0) ? c.y - c.x : 0.5f * (c.y - l);
      const float g1 = 0.5f * (c.z - c.x);
      const float g2 = 0.5f * (c.w - c.y);
      const float g3 = (x + 4 == nx) ? c.w - c.z : 0.5f * (r - c.z);
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(g0), fabsf(g1)), fmaxf(fabsf(g2), fabsf(g3))));
      const float h0 = fabsf(sy * (d.x - u.x)), h1 = fabsf(sy * (d.y - u.y));
      const float h2 = fabsf(sy * (d.z - u.z)), h3 = fabsf(sy * (d.w - u.w));
      my = fmaxf(my, fmaxf(fmaxf(h0, h1), fmaxf(h2, h3)));
      mn = fminf(mn, fminf(fminf(xv.x, xv.y), fminf(xv.z, xv.w)));
    }
  } else {
    const int n = nx * (y1 - y0);
    for (int i = threadIdx.x; i < n; i += kMaxgThreads) {
      const int yb = i / nx;
      const int y = y0 + yb, x = i - yb * nx;
      mx = fmaxf(mx, fabsf(d_x(Y, y, x, nx)));
      my = fmaxf(my, fabsf(d_y(Y, y, x, ny, nx)));
      mn = fminf(mn, ldg(X, (unsigned)(__mul24(y, nx) + x)));
    }
  }
  constexpr int kWaves = kMaxgThreads / 64;
  __shared__ float red[3][kWaves];
  mx = wave_max(mx);
  my = wave_max(my);
  mn = -wave_max(-mn);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = mx;
    red[1][w] = my;
    red[2][w] = mn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = red[0][0], b = red[1][0], c = red[2][0];
    for (int k = 1; k < kWaves; ++k) {
      a = fmaxf(a, red[0][k]);
      b = fmaxf(b, red[1][k]);
      c = fminf(c, red[2][k]);
    }
    gptr<float> mg = G(p.maxg);
    mg[3 * local] = a;
    mg[3 * local + 1] = b;
    mg[3 * local + 2] = c;
  }
}

template <bool B>
__global__ __launch_bounds__(kMaxgThreads) void k_maxgrad(KArgs a, const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, blockIdx.x, maxgrad_body, 0);
}

// ---------------------------------------------------------------------------------------------
// Splat.  A workgroup owns a TY x TX tile of the detector and accumulates, for every line, the
// bilinear deposits of all sources whose mapped footprint can reach the tile (sources within
// the halo H derived on the device from the max-gradient partials) in LDS with LDS atomics.
// Each detector pixel is written by exactly one workgroup: no global atomics.
//   forward mode: out = sum_s P_s
//   split mode  : e = d - sum_s P_s, e_s = pi_s e with pi_s = max(P_s,0)/sum max(P_s',0)
//                 (w_s where that sum is zero), written to e[s]; optional residual partials.
// NL bounds the line count at compile time so that the per-line constants sit in registers
// for the whole source loop: a scalar load inside the loop would make every iteration wait
// for all outstanding LDS atomics (they share one counter).
// ---------------------------------------------------------------------------------------------
// Stencil of D Y at a source (y, x) and X there, as loaded: the gradient is formed where the
// sample is used, so the loads of the next source stay in flight meanwhile.  Clamped
// neighbours make the differences one-sided on the edges (same values as d_x / d_y).
struct SourceSample {
  float xr, xl, yr, yl, xv;
};

__device__ __forceinline__ SourceSample load_source(gptr<const float> X, gptr<const float> Y,
                                                    int y, int x, int ny, int nx) {
  const int xl = max(x - 1, 0), xr = min(x + 1, nx - 1);
  const int yl = max(y - 1, 0), yr = min(y + 1, ny - 1);
  const int row = __mul24(y, nx);
  SourceSample s;
  s.xr = ldg(Y, (unsigned)(row + xr));
  s.xl = ldg(Y, (unsigned)(row + xl));
  s.yr = ldg(Y, (unsigned)(__mul24(yr, nx) + x));
  s.yl = ldg(Y, (unsigned)(__mul24(yl, nx) + x));
  s.xv = ldg(X, (unsigned)(row + x));
  return s;
}

// The same samples for a source at least one pixel inside every edge: one offset per lane, the
// neighbours at fixed distances from it (central differences everywhere).
__device__ __forceinline__ SourceSample load_source_inner(gptr<const float> X, gptr<const float> Y,
                                                          int y, int x, int nx) {
  const unsigned o = (unsigned)(__mul24(y, nx) + x);
  SourceSample s;
  s.xr = ldg(Y, o + 1);
  s.xl = ldg(Y, o - 1);
  s.yr = ldg(Y + nx, o);
  s.yl = ldg(Y, o - (unsigned)nx);
  s.xv = ldg(X, o);
  return s;
}

// a * b + c with a 24-bit signed multiply (full rate; b wave-uniform).  Written as the
// instruction itself: the optimiser would otherwise widen an index multiply whose operand range
// it has narrowed (from a bounds test) into a quarter-rate 32-bit multiply.
__device__ __forceinline__ int mad24(int a, int b, int c) {
  int d;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "s"(b), "v"(c));
  return d;
}

// Largest footprint window (pixels) accumulated in fixed point; wider windows fall back to
// LDS float atomics.
constexpr float kFixedWindowMax = 4096.f;

// XDEP: x-dependent spectrum, the line constants of every source and target come from its
// column (lp.w, lp.a and lp.a_hi then bound them over the columns).
template <int NL, bool XDEP>
__device__ __forceinline__ void splat_body(const ProbDesc& p, int local, int mode) {
  // Per line, accumulators for the tile plus a one-pixel border (TY+2) x (TX+2), origin
  // (ty0-1, tx0-1): a source whose 2x2 footprint touches the tile deposits all four weights
  // without per-corner bounds checks; the border is discarded.
  extern __shared__ unsigned int acc_u[];
  float* acc_f = reinterpret_cast<float*>(acc_u);
  __shared__ float red[3][kSplatThreads / 64];
  const int nx = p.nx, ny = p.ny;
  const int TX = p.splat_tx, TY = p.splat_ty;
  const int ptile = (TX + 2) * (TY + 2);
  const int L = p.lp.n;
  const int ntx = (nx + TX - 1) / TX;
  const int ty0 = (local / ntx) * TY;
  const int tx0 = (local - (local / ntx) * ntx) * TX;
  const int tid = threadIdx.x;

  float lw[NL], la2[NL], lb[NL];
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    lw[s] = s < L ? p.lp.w[s] : 0.f;
    la2[s] = s < L ? p.lp.a[s] * 1.4426950408889634f : 0.f;  // exp(-a x) = exp2(-a log2(e) x)
    lb[s] = s < L ? p.lp.b[s] : 0.f;
  }

  // halo and minimum of X from the max-gradient partials
  float gx = 0.f, gy = 0.f, xmin = INFINITY;
  gptr<const float> mg = G(p.maxg);
  for (int i = tid; i < kMaxgBlocks; i += kSplatThreads) {
    gx = fmaxf(gx, ldg(mg, (unsigned)(3 * i)));
    gy = fmaxf(gy, ldg(mg, (unsigned)(3 * i + 1)));
    xmin = fminf(xmin, ldg(mg, (unsigned)(3 * i + 2)));
  }
  gx = wave_max(gx);
  gy = wave_max(gy);
  xmin = -wave_max(-xmin);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = gx;
    red[1][tid >> 6] = gy;
    red[2][tid >> 6] = xmin;
  }
  for (int i = tid; i < L * ptile; i += kSplatThreads) acc_u[i] = 0u;
  __syncthreads();
  gx = red[0][0];
  gy = red[1][0];
  xmin = red[2][0];
#pragma unroll
  for (int w = 1; w < kSplatThreads / 64; ++w) {
    gx = fmaxf(gx, red[0][w]);
    gy = fmaxf(gy, red[1][w]);
    xmin = fminf(xmin, red[2][w]);
  }
  const int hx = halo_from(p.lp.b_absmax, gx);
  const int hy = halo_from(p.lp.b_absmax, gy);

  // Fixed-point accumulation (integer LDS atomics: several times the throughput of float
  // atomics, and order-independent).  Every source deposits at most its intensity, which is at
  // most w_s exp(-a_s min X), into one pixel, and at most (2hx+2)(2hy+2) sources reach a pixel,
  // so with scale_s = 2^30 / (w_s exp(-a_s min X) window) no sum can exceed 2^30.
  const float window = (float)(2 * hx + 2) * (float)(2 * hy + 2);
  float scale[NL], inv_scale[NL];
  bool fixed = window <= kFixedWindowMax;
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    // (x-dependent: the largest w_s with the a_s bound that maximises exp(-a_s min X))
    const float la2b = (XDEP && xmin < 0.f && s < L) ? p.lp.a_hi[s] * 1.4426950408889634f : la2[s];
    const float imax = lw[s] * __builtin_amdgcn_exp2f(-la2b * xmin);
    scale[s] = 1073741824.f / (imax * window);
    inv_scale[s] = 1.f / scale[s];
    if (s < L && !(scale[s] > 0.f && scale[s] < 3.0e38f && inv_scale[s] > 0.f)) fixed = false;
  }
  // deposits are formed directly in accumulator units: w_s scale_s (fixed point) or w_s
  float lws[NL];
#pragma unroll
  for (int s = 0; s < NL; ++s) lws[s] = fixed ? lw[s] * scale[s] : lw[s];

  const int sy0 = max(ty0 - hy, 0), sy1 = min(ty0 + TY - 1 + hy, ny - 1);
  const int sx0 = max(tx0 - hx, 0), sx1 = min(tx0 + TX - 1 + hx, nx - 1);
  const int wsrc = sx1 - sx0 + 1;
  const int nsrc = wsrc * (sy1 - sy0 + 1);
  gptr<const float> X = G(p.X);
  gptr<const float> Y = G(p.Y);

  // The source loop and the read-back, specialised for the common case (every line of the
  // bound in use, fixed-point accumulation, the default tile): no per-line tests are left in it.
  float se = 0.f, sd = 0.f;
  auto tile = [&](auto full, auto inner) {
    constexpr bool FULL = decltype(full)::value;
    // INNER: every source of the tile lies at least one pixel inside the image
    constexpr bool INNER = decltype(inner)::value;
    // the full specialisation runs the default tile: its sizes are compile-time constants, so
    // a footprint's second row and each line's accumulator are immediate offsets
    const int TXk = FULL ? kSplatTileX : TX, TYk = FULL ? kSplatTileY : TY;
    const int PXk = TXk + 2, ptk = (TXk + 2) * (TYk + 2);
    const int pxm = __builtin_amdgcn_readfirstlane(PXk);  // row stride, a scalar operand
    const int plane = nx * ny;  // line stride of e (every offset below 2^31: L nx ny <= 16 * 4096^2)
    // source index i = r * wsrc + c, advanced incrementally (no division in the loop)
    const int step_r = kSplatThreads / wsrc, step_c = kSplatThreads - step_r * wsrc;
    int r = tid / wsrc, c = tid - r * wsrc;
    SourceSample cur;
    if (tid < nsrc)
      cur = INNER ? load_source_inner(X, Y, sy0 + r, sx0 + c, nx)
                  : load_source(X, Y, sy0 + r, sx0 + c, ny, nx);
    for (int i = tid; i < nsrc; i += kSplatThreads) {
      // The loads of `cur` were issued one iteration ago: wait for them here, before the next
      // source's loads are issued (the vector-memory counter is in order, so a wait placed at
      // the first use of `cur` would also wait for the next source's loads).  LDS atomics are
      // not waited for.
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) expcnt(7) lgkmcnt(15)
      __builtin_amdgcn_sched_barrier(0);
      const int sy = sy0 + r, sx = sx0 + c;
      // footprint corner for a zero shift, relative to the bordered tile origin (ty0-1, tx0-1)
      const int rx = sx - tx0 + 1, ry = sy - ty0 + 1;
      const float dgx = cur.xr - cur.xl, dgy = cur.yr - cur.yl;
      // central differences inside, one-sided on the edges; INNER: central everywhere, with the
      // halving folded into the line constant ((b / 2) g == b (g / 2) exactly)
      float cgx = dgx, cgy = dgy;
      if constexpr (!INNER) {
        if (sx > 0 && sx < nx - 1) cgx = 0.5f * dgx;
        if (sy > 0 && sy < ny - 1) cgy = 0.5f * dgy;
      }
      r += step_r;
      c += step_c;
      if (c >= wsrc) {
        c -= wsrc;
        ++r;
      }
      SourceSample nxt;
      if (i + kSplatThreads < nsrc)
        nxt = INNER ? load_source_inner(X, Y, sy0 + r, sx0 + c, nx)
                    : load_source(X, Y, sy0 + r, sx0 + c, ny, nx);
#pragma unroll
      for (int s = 0; s < NL; ++s) {
        if (FULL || s < L) {
          float sb = INNER ? 0.5f * lb[s] : lb[s], sw = lws[s], sa2 = la2[s];
          if constexpr (XDEP) {
            const float4 c = xcol_at(p, sx, s);
            sb = INNER ? 0.5f * c.z : c.z;
            sw = (FULL || fixed) ? c.x * scale[s] : c.x;
            sa2 = c.y * 1.4426950408889634f;
          }
          const float ux = sb * cgx, uy = sb * cgy;
          const int lx = rx + floor_to_int(ux), ly = ry + floor_to_int(uy);
          if ((unsigned)lx <= (unsigned)TXk && (unsigned)ly <= (unsigned)TYk) {
            // hardware exp2 (v_exp_f32, about one ulp for the normal results met here)
            const float I = sw * __builtin_amdgcn_exp2f(-sa2 * cur.xv);
            // fractional parts x - floor(x) in one instruction each (v_fract_f32, which keeps
            // them below 1 where the subtraction would round up to 1)
            const float dx = __builtin_amdgcn_fractf(ux), dy = __builtin_amdgcn_fractf(uy);
            const int o = s * ptk + mad24(ly, pxm, lx);
            // bilinear weights, all >= 0: w10 + w00 = i0, w11 + w01 = i1, i0 + i1 = I
            const float i1 = I * dy, i0 = I - i1;
            if (FULL || fixed) {
              // nearest accumulator unit (the weights are non-negative): w + 1/2 is formed
              // directly, h10 = i0 dx + 1/2 and h00 = (i0 + 1) - h10 = i0 (1 - dx) + 1/2, then
              // truncated
              const float h10 = fmaf(i0, dx, 0.5f), h00 = (i0 + 1.f) - h10;
              const float h11 = fmaf(i1, dx, 0.5f), h01 = (i1 + 1.f) - h11;
              atomicAdd(&acc_u[o], (unsigned)h00);
              atomicAdd(&acc_u[o + 1], (unsigned)h10);
              atomicAdd(&acc_u[o + PXk], (unsigned)h01);
              atomicAdd(&acc_u[o + PXk + 1], (unsigned)h11);
            } else {
              const float w10 = i0 * dx, w00 = i0 - w10, w11 = i1 * dx, w01 = i1 - w11;
              atomicAdd(&acc_f[o], w00);
              atomicAdd(&acc_f[o + 1], w10);
              atomicAdd(&acc_f[o + PXk], w01);
              atomicAdd(&acc_f[o + PXk + 1], w11);
            }
          }
        }
      }
      cur = nxt;
    }
    __syncthreads();

    for (int i = tid; i < TXk * TYk; i += kSplatThreads) {
      const int ly = i / TXk, lx = i - ly * TXk;
      const int y = ty0 + ly, x = tx0 + lx;
      if (y >= ny || x >= nx) continue;
      const unsigned pix = (unsigned)(__mul24(y, nx) + x);
      const int o = (ly + 1) * PXk + lx + 1;
      float Pv[NL];
      float P = 0.f, S = 0.f;
#pragma unroll
      for (int s = 0; s < NL; ++s) {
        Pv[s] = 0.f;
        if (FULL || s < L)
          Pv[s] = (FULL || fixed) ? (float)acc_u[s * ptk + o] * inv_scale[s] : acc_f[s * ptk + o];
        P += Pv[s];
        if (!FULL) S += fmaxf(Pv[s], 0.f);
      }
      // fixed-point sums are never negative: the positive parts are the predictions themselves
      if (FULL) S = P;
      if (mode == kSplatForward) {
        stg(G(p.out), pix, P);
      } else if (mode == kSplatLines) {
#pragma unroll
        for (int s = 0; s < NL; ++s)
          if (FULL || s < L) stg(G(p.e), (unsigned)(s * plane) + pix, Pv[s]);
      } else {
        const float dv = ldg(G((const float*)p.d), pix);
        const float e = dv - P;
        se += e * e;
        sd += dv * dv;
        const bool hole = !(S > 1e-30f);
        const float inv = hole ? 0.f : 1.f / S;
#pragma unroll
        for (int s = 0; s < NL; ++s) {
          if (FULL || s < L) {
            float fw = lw[s];
            if constexpr (XDEP) fw = xcol_at(p, x, s).x;
            const float share = hole ? fw : (FULL ? Pv[s] : fmaxf(Pv[s], 0.f)) * inv;
            stg(G(p.e), (unsigned)(s * plane) + pix, share * e);
          }
        }
      }
    }
  };
  const bool inner = sy0 >= 1 && sy1 <= ny - 2 && sx0 >= 1 && sx1 <= nx - 2;
  if (fixed && L == NL && TX == kSplatTileX && TY == kSplatTileY) {
    if (inner)
      tile(std::true_type{}, std::true_type{});
    else
      tile(std::true_type{}, std::false_type{});
  } else {
    tile(std::false_type{}, std::false_type{});
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
      G(p.resid)[2 * local] = te;
      G(p.resid)[2 * local + 1] = td;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Detector-level sum, residual and split on an oversampled internal grid.  e holds each line's
// prediction P_s on the internal grid (ny x nx); every thread owns one detector pixel: it bins
// the f x f internal pixels of each line (their mean), sums the lines, forms e = d - P and the
// positivity-weighted split e_s, and writes e_s to the same f x f internal pixels (replication),
// in place.  Residual partial sums as in the splat.
// ---------------------------------------------------------------------------------------------
template <int NL, int F>
__device__ __forceinline__ void binsplit_body(const ProbDesc& p, int local, int) {
  const int nx = p.nx, ny = p.ny;
  const int nxd = nx / F, nyd = ny / F;
  const int L = p.lp.n;
  const int i = local * 256 + threadIdx.x;
  float se = 0.f, sd = 0.f;
  if (i < nyd * nxd) {
    const int Y = i / nxd, X = i - Y * nxd;
    const unsigned base = (unsigned)(__mul24(F * Y, nx) + F * X);
    gptr<float> e = G(p.e);
    float Pv[NL];
    float P = 0.f, S = 0.f;
#pragma unroll
    for (int s = 0; s < NL; ++s) {
      Pv[s] = 0.f;
      if (s < L) {
        gptr<const float> es = (gptr<const float>)(e + (size_t)s * nx * ny);
        float acc = 0.f;
#pragma unroll
        for (int r = 0; r < F; ++r)
#pragma unroll
          for (int c = 0; c < F; ++c) acc += ldg(es, base + (unsigned)(r * nx + c));
        Pv[s] = acc * (1.f / (F * F));
      }
      P += Pv[s];
      S += fmaxf(Pv[s], 0.f);
    }
    if (p.d == nullptr) {
      // forward model only: the detector intensity, no residual
      stg(G(p.out), (unsigned)i, P);
    } else {
      const float dv = ldg(G((const float*)p.d), (unsigned)i);
      const float ev = dv - P;
      se = ev * ev;
      sd = dv * dv;
      const bool hole = !(S > 1e-30f);
      const float inv = hole ? 0.f : 1.f / S;
#pragma unroll
      for (int s = 0; s < NL; ++s) {
        if (s < L) {
          float fw = p.lp.w[s];
          if (hole && p.xcol) {
            // x-dependent spectrum: the line's weight averaged over the f internal columns
            fw = 0.f;
#pragma unroll
            for (int c = 0; c < F; ++c) fw += xcol_at(p, F * X + c, s).x;
            fw *= 1.f / F;
          }
          const float v = (hole ? fw : fmaxf(Pv[s], 0.f) * inv) * ev;
          gptr<float> es = e + (size_t)s * nx * ny;
#pragma unroll
          for (int r = 0; r < F; ++r)
#pragma unroll
            for (int c = 0; c < F; ++c) stg(es, base + (unsigned)(r * nx + c), v);
        }
      }
    }
  }
  if (p.resid != nullptr && p.d != nullptr) {
    __shared__ float red[2][4];
    se = wave_sum(se);
    sd = wave_sum(sd);
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = se;
      red[1][threadIdx.x >> 6] = sd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      G(p.resid)[2 * local] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
      G(p.resid)[2 * local + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
  }
}

template <bool B, int NL, int F>
__global__ __launch_bounds__(256) void k_binsplit(KArgs a, const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, blockIdx.x, (binsplit_body<NL, F>), 0);
}

template <int NL, int F>
void launch_binsplit_nf(const KArgs& a, int total_blocks, hipStream_t s) {
  if (a.table)
    hipLaunchKernelGGL((k_binsplit<true, NL, F>), dim3(total_blocks), dim3(256), 0, s, a, a.table);
  else
    hipLaunchKernelGGL((k_binsplit<false, NL, F>), dim3(total_blocks), dim3(256), 0, s, a, a.table);
}

template <int NL>
hipError_t launch_binsplit_n(const KArgs& a, int total_blocks, hipStream_t s, int f) {
  if (f == 2)
    launch_binsplit_nf<NL, 2>(a, total_blocks, s);
  else if (f == 4)
    launch_binsplit_nf<NL, 4>(a, total_blocks, s);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Transpose of the detector binning for every line: the detector values r[s] copied to their
// f x f internal pixels, divided by f^2 (one internal pixel per thread).
__global__ __launch_bounds__(256) void k_unbin_lines(const float* __restrict__ r,
                                                     float* __restrict__ out, int ny, int nx,
                                                     int f, int lines) {
  const int n = ny * nx;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n * lines) return;
  const int s = i / n, j = i - s * n;
  const int y = j / nx, x = j - y * nx;
  const int nxd = nx / f;
  const float inv = 1.f / (float)(f * f);
  out[i] = inv * r[(size_t)s * (n / (f * f)) + (size_t)(y / f) * nxd + x / f];
}

hipError_t launch_unbin_lines(const float* r, float* out, int ny, int nx, int f, int lines,
                              hipStream_t s) {
  const long long total = (long long)ny * nx * lines;
  hipLaunchKernelGGL(k_unbin_lines, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, r, out,
                     ny, nx, f, lines);
  return hipGetLastError();
}

// f: the oversampling factor of the launch's problems (2 or 4).  A problem with no data
// (p.d null) gets its binned prediction in p.out instead of a split residual.
hipError_t launch_binsplit(const KArgs& a, int total_blocks, hipStream_t s, int lines, int f) {
  if (lines <= 1) return launch_binsplit_n<1>(a, total_blocks, s, f);
  if (lines <= 2) return launch_binsplit_n<2>(a, total_blocks, s, f);
  if (lines <= 4) return launch_binsplit_n<4>(a, total_blocks, s, f);
  if (lines <= 8) return launch_binsplit_n<8>(a, total_blocks, s, f);
  return launch_binsplit_n<16>(a, total_blocks, s, f);
}

template <bool B, int NL>
__global__ __launch_bounds__(kSplatThreads) void k_splat(KArgs a,
                                                        const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), (splat_body<NL, false>), a.mode);
}
// x-dependent spectrum
template <bool B, int NL>
__global__ __launch_bounds__(kSplatThreads) void k_splat_x(KArgs a,
                                                          const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), (splat_body<NL, true>), a.mode);
}

// Reduce the nb residual partials of the problem into hist_slot = ||e|| / ||d||.
__global__ __launch_bounds__(256) void k_resid_reduce(KArgs a, float* hist_slot, int nb) {
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
    hipLaunchKernelGGL(k_maxgrad<true>, dim3(total_blocks), dim3(kMaxgThreads), 0, s, a, a.table);
  else
    hipLaunchKernelGGL(k_maxgrad<false>, dim3(total_blocks), dim3(kMaxgThreads), 0, s, a, a.table);
  return hipGetLastError();
}

template <int NL>
void launch_splat_nl(const KArgs& a, int total_blocks, size_t lds, hipStream_t s) {
  if (a.xdep && a.table)
    hipLaunchKernelGGL((k_splat_x<true, NL>), dim3(total_blocks), dim3(kSplatThreads), lds, s,
                       a, a.table);
  else if (a.table)
    hipLaunchKernelGGL((k_splat<true, NL>), dim3(total_blocks), dim3(kSplatThreads), lds, s, a,
                       a.table);
  else if (a.p.xcol)
    hipLaunchKernelGGL((k_splat_x<false, NL>), dim3(total_blocks), dim3(kSplatThreads), lds, s,
                       a, a.table);
  else
    hipLaunchKernelGGL((k_splat<false, NL>), dim3(total_blocks), dim3(kSplatThreads), lds, s, a,
                       a.table);
}

// `lines` is the largest line count of the problems in the launch.
hipError_t launch_splat(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, int lines) {
  if (lines <= 1) launch_splat_nl<1>(a, total_blocks, lds, s);
  else if (lines <= 2) launch_splat_nl<2>(a, total_blocks, lds, s);
  else if (lines <= 4) launch_splat_nl<4>(a, total_blocks, lds, s);
  else if (lines <= 8) launch_splat_nl<8>(a, total_blocks, lds, s);
  else launch_splat_nl<16>(a, total_blocks, lds, s);
  return hipGetLastError();
}

hipError_t launch_resid_reduce(const KArgs& a, float* hist_slot, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_reduce, dim3(1), dim3(256), 0, s, a, hist_slot, nb);
  return hipGetLastError();
}

hipError_t set_transport_attributes() {
  const int mx = 160 * 1024 - 1024;  // (room for the static LDS of the reductions)
  const void* fns[] = {(const void*)k_splat<false, 1>, (const void*)k_splat<true, 1>,
                       (const void*)k_splat<false, 2>, (const void*)k_splat<true, 2>,
                       (const void*)k_splat<false, 4>, (const void*)k_splat<true, 4>,
                       (const void*)k_splat<false, 8>, (const void*)k_splat<true, 8>,
                       (const void*)k_splat<false, 16>, (const void*)k_splat<true, 16>,
                       (const void*)k_splat_x<false, 1>, (const void*)k_splat_x<true, 1>, (const void*)k_splat_x<false, 2>, (const void*)k_splat_x<true, 2>,
                       (const void*)k_splat_x<false, 4>, (const void*)k_splat_x<true, 4>, (const void*)k_splat_x<false, 8>, (const void*)k_splat_x<true, 8>,
                       (const void*)k_splat_x<false, 16>, (const void*)k_splat_x<true, 16>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace epr
