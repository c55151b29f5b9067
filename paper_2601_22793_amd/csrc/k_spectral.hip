// Spectral kernels: back-transport + row real FFT, column FFT with the fused Paganin-type
// filter (Section 2), and row inverse real FFT with the fused update and single-thickness
// projection (Methods 4.4, Eq. 7).
//
// Real transforms of length nx use the half-length complex trick: z[m] = r[2m] + i r[2m+1],
// Z = FFT_{nx/2}(z), X[k] = (Z[k] + conj Z[M-k])/2 - i W^k (Z[k] - conj Z[M-k])/2 with
// W = exp(-2 pi i / nx), and the mirror relation for the inverse.  All transforms are
// unnormalised; the product of their gains (ny * nx/2) is removed by the filter's scale.
//
// Every kernel is instantiated for two size classes, NT = 512 threads (nx, ny <= 2048) and
// NT = 1024 threads (<= 4096), so that each thread holds at most 8 (rows) or 16 (columns)
// complex values per FFT stage and 16 pixels of a row block.  Global memory phases issue all
// of a thread's loads before using any of them.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "epr_internal.h"
#include "fft_lds.h"

#ifndef EPR_ROWFFT_WAVES
#define EPR_ROWFFT_WAVES 8
#endif

namespace epr {

typedef __attribute__((address_space(1))) void gvoid_t;  // global memory
typedef __attribute__((address_space(3))) void lvoid_t;  // LDS

template <int NT>
struct SizeClass {
  static constexpr int kMaxNx = 4 * NT;                     // 2048 or 4096
  static constexpr int kRowEmax = kRows * (kMaxNx / 2);     // complex values of a row block
  static constexpr int kColEmax = kColBlock * kMaxNx;       // complex values of a column block
  static constexpr int kPix = kRows * kMaxNx / NT;          // pixels of a row block per thread
  static constexpr int kSpecPerThread = (kRows * (kMaxNx / 2 + kColBlock) + NT - 1) / NT;
  static constexpr int kColF4 = kColEmax / 2 / NT;          // float4 per thread, column block
};

// Bilinear interpolation weights and taps of e at (x + ux, y + uy), zero off the grid
// (Eq. 4): v = w00 e(y0,x0) + w10 e(y0,x0+1) + w01 e(y0+1,x0) + w11 e(y0+1,x0+1).
struct Taps {
  float v00, v10, v01, v11, dx, dy;
};

__device__ __forceinline__ Taps load_taps(gptr<const float> e, int ny, int nx, int y, int x,
                                          float ux, float uy) {
  Taps t;
  t.dx = __builtin_amdgcn_fractf(ux);  // x - floor(x), kept below 1 (as the splat forms it)
  t.dy = __builtin_amdgcn_fractf(uy);
  const int x0 = x + floor_to_int(ux), y0 = y + floor_to_int(uy);
  const bool xin0 = (unsigned)x0 < (unsigned)nx, xin1 = (unsigned)(x0 + 1) < (unsigned)nx;
  const bool yin0 = (unsigned)y0 < (unsigned)ny, yin1 = (unsigned)(y0 + 1) < (unsigned)ny;
  // clamp the addresses, zero the values: every lane issues the same four loads
  const int cx0 = min(max(x0, 0), nx - 1), cx1 = min(max(x0 + 1, 0), nx - 1);
  const int cy0 = min(max(y0, 0), ny - 1), cy1 = min(max(y0 + 1, 0), ny - 1);
  const int r0 = __mul24(cy0, nx), r1 = __mul24(cy1, nx);
  const float a = ldg(e, (unsigned)(r0 + cx0)), b = ldg(e, (unsigned)(r0 + cx1));
  const float c = ldg(e, (unsigned)(r1 + cx0)), d = ldg(e, (unsigned)(r1 + cx1));
  t.v00 = (yin0 && xin0) ? a : 0.f;
  t.v10 = (yin0 && xin1) ? b : 0.f;
  t.v01 = (yin1 && xin0) ? c : 0.f;
  t.v11 = (yin1 && xin1) ? d : 0.f;
  return t;
}

// (1 - dy)((1 - dx) v00 + dx v10) + dy((1 - dx) v01 + dx v11), as three linear interpolations
// (a subtraction and a multiply-add each)
__device__ __forceinline__ float taps_value(const Taps& t) {
  const float a = fmaf(t.dx, t.v10 - t.v00, t.v00);
  const float b = fmaf(t.dx, t.v11 - t.v01, t.v01);
  return fmaf(t.dy, b - a, a);
}

// Back-transport of line s at column x = tid + j NT of the kRows rows from y0 (Eq. 4, the
// adjoint of the splat): v[r] = bilinear sample of e_s at (x, y0 + r) + b_s D Y, zero off the
// grid.  A wave whose stencil lies inside the image (wave-uniform test) reads it at one column
// offset per lane from wave-uniform row pointers; if then every tap of the wave is inside the
// image too (a wave vote), the four taps are read at one offset per lane from four
// wave-uniform base pointers, with no clamps or selects.  Every path computes the same values.
template <int NT, bool XDEP>
__device__ __forceinline__ void gather_column(const ProbDesc& p, gptr<const float> es,
                                              gptr<const float> Y, int s, float bs, int y0, int j,
                                              float (&v)[kRows]) {
  const int nx = p.nx, ny = p.ny;
  const int tid = threadIdx.x;
  const int xw = __builtin_amdgcn_readfirstlane((tid & ~63) + j * NT);  // the wave's first column
  const int x = min(tid + j * NT, nx - 1);  // columns past the row: a clamped pixel, discarded
  float cb = bs;
  if constexpr (XDEP) cb = xcol_at(p, x, s).z;
  if (xw >= 1 && xw + 64 <= nx - 1 && y0 >= 1 && y0 + kRows <= ny - 1) {
    // central differences everywhere: D Y = (Y(x+1) - Y(x-1)) / 2, likewise in y; rows
    // y0 - 1 .. y0 + kRows from wave-uniform row pointers, the column neighbours at immediate
    // offsets
    const unsigned xo = (unsigned)x;
    float ga[kRows], gb[kRows], gc[kRows], gd[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const gptr<const float> Yr = Y + (y0 + r) * nx;
      ga[r] = ldg(Yr, xo + 1);
      gb[r] = ldg(Yr, xo - 1);
      gc[r] = ldg(Y + (y0 + r + 1) * nx, xo);
      gd[r] = ldg(Y + (y0 + r - 1) * nx, xo);
    }
    // b (0.5 (a - b)) == (0.5 b) (a - b): the halving is exact, so this is the value the
    // clamped path computes
    const float hb = 0.5f * cb;
    float ux[kRows], uy[kRows];
    unsigned off[kRows];
    bool inside = true;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      ux[r] = hb * (ga[r] - gb[r]);
      uy[r] = hb * (gc[r] - gd[r]);
      const int xt = x + floor_to_int(ux[r]), yt = y0 + r + floor_to_int(uy[r]);
      inside = inside && (unsigned)xt <= (unsigned)(nx - 2) && (unsigned)yt <= (unsigned)(ny - 2);
      off[r] = (unsigned)(__mul24(yt, nx) + xt);
    }
    if (__all(inside)) {
      const gptr<const float> e10 = es + 1, e01 = es + nx, e11 = es + nx + 1;
      Taps t[kRows];
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        t[r].v00 = ldg(es, off[r]);
        t[r].v10 = ldg(e10, off[r]);
        t[r].v01 = ldg(e01, off[r]);
        t[r].v11 = ldg(e11, off[r]);
        t[r].dx = __builtin_amdgcn_fractf(ux[r]);
        t[r].dy = __builtin_amdgcn_fractf(uy[r]);
      }
#pragma unroll
      for (int r = 0; r < kRows; ++r) v[r] = taps_value(t[r]);
    } else {
      Taps t[kRows];
#pragma unroll
      for (int r = 0; r < kRows; ++r) t[r] = load_taps(es, ny, nx, y0 + r, x, ux[r], uy[r]);
#pragma unroll
      for (int r = 0; r < kRows; ++r) v[r] = taps_value(t[r]);
    }
    return;
  }
  // near the edges: clamped stencil (one-sided differences on the first and last row and
  // column), clamped taps; rows past the image sample a clamped pixel, discarded
  float ga[kRows], gb[kRows], gc[kRows], gd[kRows];
  bool cy[kRows];
  const int xl = max(x - 1, 0), xh = min(x + 1, nx - 1);
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int y = min(y0 + r, ny - 1);
    const int yl = max(y - 1, 0), yh = min(y + 1, ny - 1);
    ga[r] = ldg(Y, (unsigned)(__mul24(y, nx) + xh));
    gb[r] = ldg(Y, (unsigned)(__mul24(y, nx) + xl));
    gc[r] = ldg(Y, (unsigned)(__mul24(yh, nx) + x));
    gd[r] = ldg(Y, (unsigned)(__mul24(yl, nx) + x));
    cy[r] = yh - yl == 2;
  }
  const bool cx = xh - xl == 2;
  Taps t[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const float gx = cx ? 0.5f * (ga[r] - gb[r]) : ga[r] - gb[r];
    const float gy = cy[r] ? 0.5f * (gc[r] - gd[r]) : gc[r] - gd[r];
    t[r] = load_taps(es, ny, nx, min(y0 + r, ny - 1), x, cb * gx, cb * gy);
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) v[r] = taps_value(t[r]);
}

// Float offset, in a row-transform buffer (kRows rows, padded), of the thread's pixel in row r
// and column x = tid + j NT: sample x is the real (even x) or imaginary (odd x) part of complex
// element x / 2.  NT / 2 is a multiple of 32, so the offset is a per-thread base plus a
// compile-time constant and the LDS accesses take immediate offsets.
// CNT sequences interleaved (kRows rows of one line, or of several lines one after another).
template <int NT, int CNT = kRows>
struct RowPix {
  static_assert((NT / 2) % (1 << kLdsPadShift) == 0, "row pixel layout");
  static constexpr int kJ = 2 * CNT * (NT / 2 + ((NT / 2) >> kLdsPadShift));
  int base;
  __device__ __forceinline__ explicit RowPix(int tid)
      : base(2 * CNT * ((tid >> 1) + (tid >> (kLdsPadShift + 1))) + (tid & 1)) {}
  __device__ __forceinline__ int at(int r, int j) const { return base + j * kJ + 2 * r; }
};

// W_nx^k (0 <= k <= nx/2) of the real-transform split from the table of the half-length
// transform, W_M^j with M = nx/2: W_nx^(2j) = W_M^j and W_nx^(2j+1) = W_M^j W_nx^1.
__device__ __forceinline__ float2 half_tw(const TwTable& tw, float2 w1, int k) {
  const float2 w = tw(k >> 1);
  return (k & 1) ? cmul(w, w1) : w;
}

// ---------------------------------------------------------------------------------------------
// Row pass: per (line s, block of kRows rows) compute r_s (gather of e_s at the mapped points,
// or a copy of e_s), then the real FFT of each row, stored as column blocks of the half
// spectrum.  In gather-only mode r_s goes to p.out and no transform is done (epr_adjoint).
// ---------------------------------------------------------------------------------------------
// XDEP: x-dependent spectrum, b_s of the gather is read at each pixel's column.
template <int NT, bool XDEP>
__device__ __forceinline__ void rowfft_body(const ProbDesc& p, int local, int mode) {
  using SC = SizeClass<NT>;
  extern __shared__ float2 buf[];
  const int nx = p.nx, ny = p.ny, M = nx >> 1;
  // lines vary fastest: the blocks of one row block (all lines) share the thickness stencil,
  // and with the XCD-contiguous block order they run behind one L2
  const int L = p.lp.n;
  const int rb = local / L;
  const int s = local - rb * L;
  const int y0 = rb * kRows;
  gptr<const float> es = G(p.e) + (size_t)s * nx * ny;
  gptr<const float> Y = G(p.Y);
  const float bs = p.lp.b[s];
  const int tid = threadIdx.x;
  float* fb = reinterpret_cast<float*>(buf);
  const bool gather = mode != kRowCopyFft;
  // twiddle table after the transform buffer; its loads overlap the gather
  const TwTable tw = load_twiddles(kRows * lds_rows(M), p.row, tid, NT);

  // the thread's pixels: column x = tid + j NT of each of the kRows rows; the kRows values of
  // one column are loaded together and go straight into the transform buffer (complex index
  // x/2, real part for even x, imaginary for odd x)
  constexpr int kPerRow = SC::kMaxNx / NT;
  const RowPix<NT> pix(tid);
#pragma unroll
  for (int j = 0; j < kPerRow; ++j) {
    // a wave whose columns all lie past the row (narrow images in a size class) has nothing
    // to load or store in this column chunk
    if (__builtin_amdgcn_readfirstlane((tid & ~63) + j * NT) >= nx) continue;
    float v[kRows];
    if (gather) {
      gather_column<NT, XDEP>(p, es, Y, s, bs, y0, j, v);
    } else {
      // columns or rows past the image read a clamped in-bounds pixel; the value is discarded
      const int x = min(tid + j * NT, nx - 1);
#pragma unroll
      for (int r = 0; r < kRows; ++r)
        v[r] = ldg(es, (unsigned)(__mul24(min(y0 + r, ny - 1), nx) + x));
    }
    const int x = tid + j * NT;
    if (x < nx) {
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        const int y = y0 + r;
        const float val = (y < ny) ? v[r] : 0.f;
        fb[pix.at(r, j)] = val;
        if (mode == kRowGatherOnly && y < ny) stg(G(p.out) + (size_t)s * nx * ny, (unsigned)(__mul24(y, nx) + x), val);
      }
    }
  }
  if (mode == kRowGatherOnly) return;
  __syncthreads();
  fft_lds<kRows, NT, SC::kRowEmax, 1>(0, p.row, tw);

  // Split of the half-length transform Z into the half spectrum X, one pair (k, M - k) per
  // item: with A = (Z[k] + conj Z[M-k]) / 2, B = (Z[k] - conj Z[M-k]) / 2 and W = W_nx,
  //   X[k] = A - i W^k B,   X[M-k] = conj(A) - i conj(W^k B)
  // (W^(M-k) = -conj W^k).  Items k = 0 .. M/2 cover every frequency 0 .. M; for even M the
  // item k = M/2 is its own mirror.  Then the unused columns of the last block are zeroed.
  // Item i: column c = i % 4 of block i / 16, row (i / 4) % 4, so that the X[k] of 16
  // consecutive items form one 128-byte tile row group.
  const float2 w1 = G(p.row_tw)[1];
  gptr<float2> out = G(p.spec) + (size_t)s * p.nblk * ny * kColBlock;
  const int nk = M / 2 + 1;
  const int npair = (nk + kColBlock - 1) / kColBlock * (kColBlock * kRows);
  const int nitem = npair + (p.nblk * kColBlock - (M + 1)) * kRows;
  for (int i = tid; i < nitem; i += NT) {
    if (i < npair) {
      const int c = i % kColBlock;
      const int r = (i / kColBlock) % kRows;
      const int k = (i / (kColBlock * kRows)) * kColBlock + c;
      const int y = y0 + r;
      if (k >= nk || y >= ny) continue;
      const int km = M - k;
      const float2 zk = buf[lds_index<kRows>(k, r)];
      const float2 zm = cconj(buf[lds_index<kRows>(k == 0 ? 0 : km, r)]);
      const float2 A = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
      const float2 B = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y - zm.y));
      const float2 WB = cmul(half_tw(tw, w1, k), B);
      stg(out, (unsigned)(((k >> 2) * ny + y) * kColBlock + (k & 3)),
          make_float2(A.x + WB.y, A.y - WB.x));                 // A - i W B
      if (km != k)
        stg(out, (unsigned)(((km >> 2) * ny + y) * kColBlock + (km & 3)),
            make_float2(A.x - WB.y, -A.y - WB.x));              // conj A - i conj(W B)
    } else {
      // zero padding: frequencies M + 1 .. 4 nblk - 1 of every row
      const int j = i - npair;
      const int k = M + 1 + j / kRows, y = y0 + j % kRows;
      if (y < ny) stg(out, (unsigned)(((k >> 2) * ny + y) * kColBlock + (k & 3)), make_float2(0.f, 0.f));
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Row pass over K lines per workgroup, one after the other (the problem's lines in groups of K,
// the last group may be short).  The lines of a row block share its thickness stencil: after
// the first line it comes from the workgroup's own L1 instead of being fetched again by
// another workgroup.  The transform buffer is reused line by line.  K is a compile-time
// constant: the line bodies are laid out one after the other, which keeps the register
// allocation of one line (a run-time loop over lines spills).
// ---------------------------------------------------------------------------------------------
template <int NT, bool XDEP, int K, int I = 0>
__device__ __forceinline__ void rowfft_group_lines(const ProbDesc& p, int base, int n, int mode) {
  if constexpr (I < K) {
    if (I < n) {
      if (I > 0) __syncthreads();  // the previous line's split has read the buffer and table
      rowfft_body<NT, XDEP>(p, base + I, mode);
      rowfft_group_lines<NT, XDEP, K, I + 1>(p, base, n, mode);
    }
  }
}

template <int NT, bool XDEP, int K>
__device__ __forceinline__ void rowfft_group_body(const ProbDesc& p, int local, int mode) {
  const int L = p.lp.n;
  const int ng = (L + K - 1) / K;
  const int rb = local / ng;
  const int g0 = (local - rb * ng) * K;
  rowfft_group_lines<NT, XDEP, K>(p, rb * L + g0, min(K, L - g0), mode);
}


template <bool B, int NT, int K>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(EPR_ROWFFT_WAVES))) void k_rowfft(KArgs a, const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), (rowfft_group_body<NT, false, K>), a.mode);
}
// x-dependent spectrum
template <bool B, int NT, int K>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(EPR_ROWFFT_WAVES))) void k_rowfft_x(KArgs a, const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), (rowfft_group_body<NT, true, K>), a.mode);
}

// ---------------------------------------------------------------------------------------------
// Column pass: per (line s, block of kColBlock frequencies) forward FFT along y, multiply by
// scale / (1 + h_s (fx^2 + fy^2)), inverse FFT along y (via conjugation), in place.  The block
// is one contiguous run of ny * kColBlock complex values.
// ---------------------------------------------------------------------------------------------
// EMAX: complex values of the largest column block the instance transforms (lengths up to
// EMAX / kColBlock are compiled in).
template <int NT, int EMAX = SizeClass<NT>::kColEmax>
__device__ __forceinline__ void colfft_body(const ProbDesc& p, int local, int) {
  constexpr int kColF4 = (EMAX / 2 + NT - 1) / NT;  // float4 per thread, column block
  extern __shared__ float2 buf[];
  const int ny = p.ny, nx = p.nx;
  const int s = local / p.nblk;
  const int blk = local - s * p.nblk;
  gptr<float2> g = G(p.spec) + ((size_t)s * p.nblk + blk) * ny * kColBlock;
  // output: in place, or the spectra of one preconditioner block (block-wise preconditioner)
  gptr<float2> go = G(p.spec_out ? p.spec_out : p.spec) + ((size_t)s * p.nblk + blk) * ny * kColBlock;
  const int n4 = ny * kColBlock / 2;
  const int tid = threadIdx.x;
  const TwTable tw = load_twiddles(kColBlock * lds_rows(ny), p.col, tid, NT);
  {
    // the block is one contiguous run: copy it to LDS with direct global->LDS loads, 16 bytes
    // per lane, one 1 KiB chunk (32 rows) per wave and instruction (no registers involved);
    // each chunk lands after its padding row
    gptr<const float4> g4 = (gptr<const float4>)g;
    float4* b4 = reinterpret_cast<float4*>(buf);
    const int lane = tid & 63, wave = tid >> 6;
    for (int base = wave * 64; base < n4; base += NT) {
      if (base + lane < n4)
        __builtin_amdgcn_global_load_lds((const gvoid_t*)((gptr<const char>)g4 + (unsigned)((base + lane) * 16)),
                                         (lvoid_t*)(b4 + base + 2 * (base >> 6)), 16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);  // all loads of this wave have landed in LDS
  }
  __syncthreads();
  ColumnFilter filt;
  filt.h = p.lp.h[s];
  filt.scale = p.lp.spec_scale;
  filt.inv_ny = 1.f / (float)ny;
  filt.inv_nx = 1.f / (float)nx;
  filt.ny = ny;
  filt.col0 = blk * kColBlock;
  // compile-time lengths store the result from their last stage; the others from LDS here
  if (!fft_filter_ifft_lds<kColBlock, NT, EMAX, 2>(0, p.col, tw, filt, go)) {
    gptr<float4> g4 = (gptr<float4>)go;
    const float4* b4 = reinterpret_cast<const float4*>(buf);
#pragma unroll
    for (int k = 0; k < kColF4; ++k) {
      const int i = tid + k * NT;
      if (i < n4) {
        const float4 v = b4[i + 2 * (i >> 6)];  // float4 i = complex 2i, 2i+1 of row i/2
        stg(g4, (unsigned)i, make_float4(v.x, -v.y, v.z, -v.w));
      }
    }
  }
}

template <bool B, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_colfft(KArgs a, const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), colfft_body<NT>, 0);
}

// The 1024-thread column pass for columns of at most kColMidMax rows (the 2160 x 2560 problems):
// without the 4096-point transforms it needs 64 VGPRs, so eight waves per SIMD, and two
// workgroups share a CU where their LDS fits (ny <= 2213), against one for the full instance.
template <bool B>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_colfft_mid(KArgs a, const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), (colfft_body<1024, kColBlock * kColMidMax>), 0);
}

// ---------------------------------------------------------------------------------------------
// Row inverse pass: per block of kRows rows, for every line: inverse real FFT of the filtered
// half spectrum -> dI_s; then either write dI_s (precondition mode) or accumulate the
// projection of I_s + omega dI_s onto one thickness (solve mode) and write tau.
//   * The block's 4 x 4 tiles of a line are copied verbatim to LDS by direct global->LDS loads;
//     the next line's copy streams in while the current line is transformed (the transform
//     reads its twiddles from LDS, so no other global load waits behind the copy).
//   * The thread's pixels, their thickness and their projection sums stay in registers.
// ---------------------------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void fetch_row_tiles(gptr<const float2> sp, float2* dst, int nblk,
                                                int ny, int y0) {
  // 16-byte chunk q of the block: tile blk = q / 8, row r = (q / 2) % 4, columns 2 (q % 2) + {0,1}
  const int nq = nblk * 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float4* d4 = reinterpret_cast<float4*>(dst);
  for (int base = wave * 64; base < nq; base += NT) {
    const int q = base + lane;
    if (q < nq) {
      const int blk = q >> 3, r = (q >> 1) & 3;
      const int y = min(y0 + r, ny - 1);  // rows past the image repeat the last row
      gptr<const char> src = (gptr<const char>)sp + (unsigned)(((blk * ny + y) * 2 + (q & 1)) * 16);
      __builtin_amdgcn_global_load_lds((const gvoid_t*)src, (lvoid_t*)(d4 + base), 16, 0, 0);
    }
  }
}

// XDEP: x-dependent spectrum, the update and projection constants are read per column.
// BLK (with XDEP): block-wise preconditioner.  Each line has p.nbp filtered spectra, one per
// preconditioner block b (block 0 at p.spec, block b >= 1 in p.spec_blk); the row
// inverse transforms each of them and blends them per column with the interpolation weights
// lambda_b(x) (p.xblk[x] = {b0, t}: lambda_b0 = 1 - t, lambda_(b0+1) = t, 0 otherwise) before
// the update.
template <int NT, bool SOLVE, bool XDEP, bool BLK = false>
__device__ __forceinline__ void rowinv_body(const ProbDesc& p, int local, int) {
  using SC = SizeClass<NT>;
  extern __shared__ float2 buf[];
  const int nx = p.nx, ny = p.ny, M = nx >> 1;
  const int y0 = local * kRows;
  const int L = p.lp.n;
  const int tid = threadIdx.x;
  const int nin = p.nblk * kColBlock * kRows;  // complex values of one line's tiles
  const size_t line_elems = (size_t)p.nblk * ny * kColBlock;
  float2* raw = buf;        // the line's tiles as copied: [block][row][column]
  float2* F = buf + nin;    // transform buffer
  const TwTable tw = load_twiddles(nin + kRows * lds_rows(M), p.row, tid, NT);
  const float2 w1 = G(p.row_tw)[1];
  gptr<const float2> spec = G((const float2*)p.spec);
  fetch_row_tiles<NT>(spec, raw, p.nblk, ny, y0);

  // the thread's pixels: row r, column x = tid + j NT (k = r * kPerRow + j)
  constexpr int kPerRow = SC::kMaxNx / NT;
  // live[j]: the wave has columns of chunk j inside the row (wave-uniform; narrow images in a
  // size class leave whole chunks empty, which are then skipped)
  bool live[kPerRow];
#pragma unroll
  for (int j = 0; j < kPerRow; ++j)
    live[j] = __builtin_amdgcn_readfirstlane((tid & ~63) + j * NT) < nx;
  float tv[SC::kPix], acc[SC::kPix];
#pragma unroll
  for (int k = 0; k < SC::kPix; ++k) {
    const int r = k / kPerRow, x = min(tid + (k % kPerRow) * NT, nx - 1);
    const int y = min(y0 + r, ny - 1);
    tv[k] = 0.f;
    if constexpr (SOLVE)
      if (live[k % kPerRow]) tv[k] = ldg(G((const float*)p.tau), (unsigned)(__mul24(y, nx) + x));
    acc[k] = 0.f;
  }
  const float odd_sign = (tid & 1) ? -1.f : 1.f;  // NT is even: x has the parity of tid
  const RowPix<NT> pix(tid);
  // sum of every update the thread applies: finite exactly when each of them is (the floor
  // of the update would otherwise hide a NaN)
  float chk = 0.f;
  // transform units: one per line, or one per (line, preconditioner block), block fastest
  const int nb = BLK ? p.nbp : 1;
  const int nunit = L * nb;
  float dacc[BLK ? SC::kPix : 1];
#pragma unroll
  for (int k = 0; k < (BLK ? SC::kPix : 1); ++k) dacc[k] = 0.f;

  for (int un = 0; un < nunit; ++un) {
    const int s = BLK ? un / nb : un;
    const int bk = BLK ? un - s * nb : 0;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of unit un have landed
    __syncthreads();                // ... and everyone's; unit un-1 is no longer read
    // Z[k] = E_k + i O_k, E_k = (X_k + conj X_{M-k})/2, O_k = (X_k - conj X_{M-k})/2 W^-k;
    // store conj(Z) so that a forward FFT followed by conjugation inverts it.
    // W_nx^(M-k) = -conj(W_nx^k).
    const int half = M >> 1;
    for (int i = tid; i < (half + 1) * kRows; i += NT) {
      const int k = i / kRows, r = i - k * kRows;
      // tile position of frequency k in row r: (k / 4) * 16 + r * 4 + k % 4
      const float2 xk = raw[((k >> 2) << 4) | (r << 2) | (k & 3)];
      const float2 xm = raw[(((M - k) >> 2) << 4) | (r << 2) | ((M - k) & 3)];
      const float2 wk = half_tw(tw, w1, k);
      {
        const float2 xmc = cconj(xm);
        const float2 E = make_float2(0.5f * (xk.x + xmc.x), 0.5f * (xk.y + xmc.y));
        const float2 D = make_float2(0.5f * (xk.x - xmc.x), 0.5f * (xk.y - xmc.y));
        const float2 O = cmul(D, cconj(wk));
        const float2 Z = make_float2(E.x - O.y, E.y + O.x);
        F[lds_index<kRows>(k, r)] = cconj(Z);
      }
      if (k != 0 && 2 * k != M) {
        const float2 xkc = cconj(xk);
        const float2 E = make_float2(0.5f * (xm.x + xkc.x), 0.5f * (xm.y + xkc.y));
        const float2 D = make_float2(0.5f * (xm.x - xkc.x), 0.5f * (xm.y - xkc.y));
        const float2 O = cmul(D, make_float2(-wk.x, -wk.y));  // conj(W^(M-k)) = -W^k
        const float2 Z = make_float2(E.x - O.y, E.y + O.x);
        F[lds_index<kRows>(M - k, r)] = cconj(Z);
      }
    }
    __syncthreads();  // the tiles are consumed: unit un+1 streams in during the transform
    if (un + 1 < nunit) {
      const int s1 = BLK ? (un + 1) / nb : un + 1, b1 = BLK ? (un + 1) - s1 * nb : 0;
      gptr<const float2> sb = b1 == 0 ? spec : G((const float2*)p.spec_blk) + (size_t)(b1 - 1) * p.spec_set;
      fetch_row_tiles<NT>(sb + (size_t)s1 * line_elems, raw, p.nblk, ny, y0);
    }
    fft_lds<kRows, NT, SC::kRowEmax, SOLVE ? (BLK ? 5 : 3) : 4>(nin, p.row, tw);

    const float* fb = reinterpret_cast<const float*>(F);
    if constexpr (BLK) {
      // blend this block's output into the line's update; the update follows the last block
#pragma unroll
      for (int k = 0; k < SC::kPix; ++k) {
        const int r = k / kPerRow, x = tid + (k % kPerRow) * NT;
        if (live[k % kPerRow] && x < nx) {
          const float2 bt = ldg(G(p.xblk), (unsigned)x);
          const int b0 = (int)bt.x;
          const float lam = bk == b0 ? 1.f - bt.y : (bk == b0 + 1 ? bt.y : 0.f);
          dacc[k] = fmaf(lam, odd_sign * fb[pix.at(r, k % kPerRow)], dacc[k]);
        }
      }
      if (bk + 1 < nb) continue;
    }
    if constexpr (SOLVE) {
      // The projection takes ln(max(I_s + omega dI_s, 1e-6 w_s) / w_s) as
      // ln(max(exp(-a_s tau) + (omega / w_s) dI_s, 1e-6)): the same value, but formed without
      // the product w_s (1 / w_s), whose float32 rounding (about 1e-7, different in every
      // column of an x-dependent spectrum) would otherwise enter every iteration as a thickness
      // offset of that size over mu_s.  exp and ln through the hardware base-2 transcendentals
      // (v_exp_f32 / v_log_f32): the ratio stays a normal number (>= 1e-6), where both are
      // accurate to about one ulp.
      const float la2 = p.lp.a[s] * 1.4426950408889634f;
      const float mws_ln2 = p.lp.mw[s] * 0.69314718055994531f;
      const float om = p.relax, om_w = p.relax * p.lp.inv_w[s];
#pragma unroll
      for (int k = 0; k < SC::kPix; ++k) {
        const int r = k / kPerRow, x = tid + (k % kPerRow) * NT;
        if (live[k % kPerRow] && x < nx) {
          // conj of the transform output: the odd (imaginary) samples change sign
          float dI;
          if constexpr (BLK) {
            dI = dacc[k];
            dacc[k] = 0.f;
          } else {
            dI = odd_sign * fb[pix.at(r, k % kPerRow)];
          }
          chk += dI;
          if constexpr (XDEP) {
            const float4 c = xcol_at(p, x, s), q = xproj_at(p, x, s);
            const float g = __builtin_amdgcn_exp2f(-(c.y * 1.4426950408889634f) * tv[k]);
            const float r = fmaxf(fmaf(om * q.y, dI, g), 1e-6f);
            acc[k] += (q.x * 0.69314718055994531f) * __builtin_amdgcn_logf(r);
          } else {
            const float g = __builtin_amdgcn_exp2f(-la2 * tv[k]);
            const float r = fmaxf(fmaf(om_w, dI, g), 1e-6f);
            acc[k] += mws_ln2 * __builtin_amdgcn_logf(r);
          }
        }
      }
    } else {
      gptr<float> o = G(p.out) + (size_t)s * nx * ny;
#pragma unroll
      for (int k = 0; k < SC::kPix; ++k) {
        const int r = k / kPerRow, x = tid + (k % kPerRow) * NT, y = y0 + r;
        if (live[k % kPerRow] && x < nx && y < ny)
          stg(o, (unsigned)(__mul24(y, nx) + x), odd_sign * fb[pix.at(r, k % kPerRow)]);
      }
    }
  }

  if constexpr (SOLVE) {
    const float inv_den = p.lp.inv_den, pc = p.lp.phase_coef;
    bool bad = !(fabsf(chk) <= 3.40282347e38f);
#pragma unroll
    for (int k = 0; k < SC::kPix; ++k) {
      const int r = k / kPerRow, x = tid + (k % kPerRow) * NT, y = y0 + r;
      if (live[k % kPerRow] && x < nx && y < ny) {
        float id = inv_den;
        if constexpr (XDEP) id = ldg(G(p.xden), (unsigned)x);
        const float t = -acc[k] * id;
        bad = bad || !(fabsf(t) <= 3.40282347e38f);
        stg(G(p.tau), (unsigned)(__mul24(y, nx) + x), t);
        if (p.phase_out) stg(G(p.phase_out), (unsigned)(__mul24(y, nx) + x), pc * t);
      }
    }
    // one vector store per wave that met a non-finite value (every writer stores 1)
    if (__any(bad) && (tid & 63) == 0 && p.status != nullptr) G(p.status)[0] = 1u;
  }
}

// solve and precondition modes are separate kernels: each is register-allocated for its own path
template <bool B, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_rowinv(
    KArgs a, const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), (rowinv_body<NT, true, false>), 0);
}
template <bool B, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_rowinv_x(
    KArgs a, const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), (rowinv_body<NT, true, true>), 0);
}
// x-dependent spectrum with the block-wise preconditioner
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_rowinv_xb(
    KArgs a, const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(false, a, table, xcd_remap(blockIdx.x, gridDim.x),
               (rowinv_body<NT, true, true, true>), 0);
}
template <bool B, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_rowinv_pre(
    KArgs a, const ProbDesc* __restrict__ table) {
  EPR_DISPATCH(B, a, table, xcd_remap(blockIdx.x, gridDim.x), (rowinv_body<NT, false, false>), 0);
}

// the row-pass instances by lines per workgroup, as two-parameter templates for EPR_LAUNCH_SC
template <bool B, int NT> constexpr auto k_rowfft1 = k_rowfft<B, NT, 1>;
template <bool B, int NT> constexpr auto k_rowfft2 = k_rowfft<B, NT, 2>;
template <bool B, int NT> constexpr auto k_rowfft4 = k_rowfft<B, NT, 4>;
template <bool B, int NT> constexpr auto k_rowfft_x1 = k_rowfft_x<B, NT, 1>;
template <bool B, int NT> constexpr auto k_rowfft_x2 = k_rowfft_x<B, NT, 2>;
template <bool B, int NT> constexpr auto k_rowfft_x4 = k_rowfft_x<B, NT, 4>;

#define EPR_LAUNCH_SC(K, a, grid, nt, lds, s)                                                \
  do {                                                                                       \
    if (nt == 512) {                                                                         \
      if ((a).table)                                                                         \
        hipLaunchKernelGGL((K<true, 512>), dim3(grid), dim3(512), lds, s, a, a.table);               \
      else                                                                                   \
        hipLaunchKernelGGL((K<false, 512>), dim3(grid), dim3(512), lds, s, a, a.table);              \
    } else {                                                                                 \
      if ((a).table)                                                                         \
        hipLaunchKernelGGL((K<true, 1024>), dim3(grid), dim3(1024), lds, s, a, a.table);             \
      else                                                                                   \
        hipLaunchKernelGGL((K<false, 1024>), dim3(grid), dim3(1024), lds, s, a, a.table);            \
    }                                                                                        \
  } while (0)

// single-problem kernels (the block-wise row inverse)
#define EPR_LAUNCH_X(K, a, grid, nt, lds, s)                                                  \
  do {                                                                                       \
    if (nt == 512)                                                                           \
      hipLaunchKernelGGL((K<512>), dim3(grid), dim3(512), lds, s, a, a.table);              \
    else                                                                                     \
      hipLaunchKernelGGL((K<1024>), dim3(grid), dim3(1024), lds, s, a, a.table);            \
  } while (0)

hipError_t launch_rowfft(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, int nt) {
  const bool x = a.table ? a.xdep != 0 : a.p.xcol != nullptr;
  const int k = a.table ? a.rl : row_lines(a.p);
  if (x && a.mode != kRowCopyFft) {
    switch (k) {
      case 4: EPR_LAUNCH_SC(k_rowfft_x4, a, total_blocks, nt, lds, s); break;
      case 2: EPR_LAUNCH_SC(k_rowfft_x2, a, total_blocks, nt, lds, s); break;
      default: EPR_LAUNCH_SC(k_rowfft_x1, a, total_blocks, nt, lds, s); break;
    }
  } else {
    switch (k) {
      case 4: EPR_LAUNCH_SC(k_rowfft4, a, total_blocks, nt, lds, s); break;
      case 2: EPR_LAUNCH_SC(k_rowfft2, a, total_blocks, nt, lds, s); break;
      default: EPR_LAUNCH_SC(k_rowfft1, a, total_blocks, nt, lds, s); break;
    }
  }
  return hipGetLastError();
}
hipError_t launch_colfft(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, int nt) {
  const int ny_max = a.table ? a.ny_max : a.p.ny;
  if (nt == 1024 && ny_max > 0 && ny_max <= kColMidMax) {
    if (a.table)
      hipLaunchKernelGGL(k_colfft_mid<true>, dim3(total_blocks), dim3(1024), lds, s, a, a.table);
    else
      hipLaunchKernelGGL(k_colfft_mid<false>, dim3(total_blocks), dim3(1024), lds, s, a, a.table);
    return hipGetLastError();
  }
  EPR_LAUNCH_SC(k_colfft, a, total_blocks, nt, lds, s);
  return hipGetLastError();
}
hipError_t launch_rowinv(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, int nt) {
  const bool x = a.table ? a.xdep != 0 : a.p.xcol != nullptr;
  if (a.mode == kRowInvSolve && !a.table && a.p.xcol && a.p.nbp > 0)
    EPR_LAUNCH_X(k_rowinv_xb, a, total_blocks, nt, lds, s);
  else if (a.mode == kRowInvSolve && x)
    EPR_LAUNCH_SC(k_rowinv_x, a, total_blocks, nt, lds, s);
  else if (a.mode == kRowInvSolve)
    EPR_LAUNCH_SC(k_rowinv, a, total_blocks, nt, lds, s);
  else
    EPR_LAUNCH_SC(k_rowinv_pre, a, total_blocks, nt, lds, s);
  return hipGetLastError();
}

hipError_t set_spectral_attributes() {
  const int mx = 160 * 1024 - 64;
  const void* fns[] = {
#define EPR_ROWFFT_FNS(K)                                                                 \
      (const void*)K<false, 512>, (const void*)K<true, 512>,                                 \
      (const void*)K<false, 1024>, (const void*)K<true, 1024>
      EPR_ROWFFT_FNS(k_rowfft1), EPR_ROWFFT_FNS(k_rowfft2), EPR_ROWFFT_FNS(k_rowfft4),
      EPR_ROWFFT_FNS(k_rowfft_x1), EPR_ROWFFT_FNS(k_rowfft_x2), EPR_ROWFFT_FNS(k_rowfft_x4),
      (const void*)k_colfft<false, 512>, (const void*)k_colfft<true, 512>,
      (const void*)k_colfft<false, 1024>, (const void*)k_colfft<true, 1024>,
      (const void*)k_colfft_mid<false>, (const void*)k_colfft_mid<true>,
      (const void*)k_rowinv<false, 512>, (const void*)k_rowinv<true, 512>,
      (const void*)k_rowinv<false, 1024>, (const void*)k_rowinv<true, 1024>,
      (const void*)k_rowinv_pre<false, 512>, (const void*)k_rowinv_pre<true, 512>,
      (const void*)k_rowinv_pre<false, 1024>, (const void*)k_rowinv_pre<true, 1024>,
      (const void*)k_rowinv_x<false, 512>, (const void*)k_rowinv_x<true, 512>,
      (const void*)k_rowinv_x<false, 1024>, (const void*)k_rowinv_x<true, 1024>,
      (const void*)k_rowinv_xb<512>, (const void*)k_rowinv_xb<1024>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace epr
