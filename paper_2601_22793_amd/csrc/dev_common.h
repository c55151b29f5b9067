// Device helpers shared by the kernels: workgroup -> problem lookup, XCD-aware block order,
// the derivative operator and small reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "epr_internal.h"

namespace epr {

// The dispatcher hands workgroup b to XCD (b mod 8).  Give each XCD one contiguous range of
// logical blocks so that neighbouring tiles / row blocks, which re-read each other's halo,
// run behind the same L2.  Bijective on [0, nblocks).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int xcd = bid & 7, idx = bid >> 3;
  const int base = xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q;
  return base + idx;
}

// Problem of a batched launch owning logical block `bid` (wave-uniform), and the block index
// inside it.
__device__ __forceinline__ int find_problem(const KArgs& a, int bid, int& local) {
  int lo = 0, hi = a.nprob;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.starts[mid] <= bid) lo = mid; else hi = mid;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  local = bid - a.starts[lo];
  return lo;
}

// Kernels are instantiated twice: BATCHED = false reads the single problem straight from the
// kernel-argument segment (never taking its address, which would copy it to scratch);
// BATCHED = true reads its problem from the table at a wave-uniform index.  The table comes in
// as its own `const ProbDesc* __restrict__` kernel argument: nothing the kernel stores can
// alias it, so its fields are fetched with scalar loads into SGPRs.
#define EPR_DISPATCH(BATCHED, a, table, bid, BODY, ...)          \
  do {                                                            \
    int local_;                                                   \
    if constexpr (BATCHED) {                                      \
      const int pi_ = find_problem((a), (bid), local_);           \
      BODY((table)[pi_], local_, __VA_ARGS__);                    \
    } else {                                                      \
      local_ = (bid);                                             \
      BODY((a).p, local_, __VA_ARGS__);                           \
    }                                                             \
  } while (0)

// Pointers read from the problem table are generic (flat) pointers; the kernels only ever
// pass device memory, so re-typing them as global lets the loads and stores use a scalar base
// plus a 32-bit vector offset instead of 64-bit flat addresses.
// (The host pass of hipcc also parses device bodies; there the type is a plain pointer.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <class T>
using gptr = T*;
#endif
template <class T>
__device__ __forceinline__ gptr<T> G(T* p) {
  return (gptr<T>)p;
}

// Row offsets y * nx are formed with 24-bit multiplies (__mul24, full rate; the 32-bit integer
// multiply is quarter rate): rows and widths are at most 4096.
//
// Element idx of a device array addressed by a 32-bit byte offset from a wave-uniform base:
// the access compiles to a scalar base plus a 32-bit vector offset instead of a 64-bit vector
// address computed per lane.  Every array (one image, one line's image or spectrum) is far
// below 4 GiB.
template <class T>
__device__ __forceinline__ T ldg(gptr<const T> base, unsigned idx) {
  return *(gptr<const T>)((gptr<const char>)base + idx * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ void stg(gptr<T> base, unsigned idx, T v) {
  *(gptr<T>)((gptr<char>)base + idx * (unsigned)sizeof(T)) = v;
}

// Derivative operator D (pixel units): central difference inside, first-order one-sided
// difference on the first and last sample of each axis.
__device__ __forceinline__ float d_x(gptr<const float> f, int y, int x, int nx) {
  const unsigned row = (unsigned)(y * nx);
  if (x == 0) return ldg(f, row + 1) - ldg(f, row);
  if (x == nx - 1) return ldg(f, row + nx - 1) - ldg(f, row + nx - 2);
  return 0.5f * (ldg(f, row + x + 1) - ldg(f, row + x - 1));
}
__device__ __forceinline__ float d_y(gptr<const float> f, int y, int x, int ny, int nx) {
  if (y == 0) return ldg(f, (unsigned)(nx + x)) - ldg(f, (unsigned)x);
  if (y == ny - 1) return ldg(f, (unsigned)((ny - 1) * nx + x)) - ldg(f, (unsigned)((ny - 2) * nx + x));
  return 0.5f * (ldg(f, (unsigned)((y + 1) * nx + x)) - ldg(f, (unsigned)((y - 1) * nx + x)));
}

// Constants of line s at column x of an x-dependent spectrum: {w, a, b, q} and
// {mw, 1/w, floor, 0} (ProbDesc::xcol).
__device__ __forceinline__ float4 xcol_at(const ProbDesc& p, int x, int s) {
  return ldg(G(p.xcol), (unsigned)((x * p.lp.n + s) * 2));
}
__device__ __forceinline__ float4 xproj_at(const ProbDesc& p, int x, int s) {
  return ldg(G(p.xcol), (unsigned)((x * p.lp.n + s) * 2 + 1));
}

// floor(x) as an integer in one instruction (v_cvt_flr_i32_f32; |x| well inside the int range)
__device__ __forceinline__ int floor_to_int(float x) {
  int r;
  __asm__("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Halo (in pixels, per axis) that covers every source whose bilinear footprint can reach a
// tile: H = floor(max |u|) + 1, with max |u| = max_s |b_s| * max |D Y| (rounding is monotone,
// so this bounds every per-source shift computed as b_s * D Y).  Capped at the image size.
__device__ __forceinline__ int halo_from(float bmax, float gmax) {
  const float h = floorf(bmax * gmax) + 1.0f;
  return (h < (float)kMaxDim) ? (int)h : kMaxDim;  // also maps NaN to kMaxDim
}

}  // namespace epr
