// Internal types shared by the gfx950 kernels and the host side of libepr.
//
// Data layout in HBM, per problem (ny x nx detector, L spectral lines):
//   X, Y      [ny][nx] f32   maps the lines are derived from (solve: both are the thickness
//                            tau; forward/adjoint: X = absorption, Y = phase)
//   d         [ny][nx] f32   detector image
//   e         [L][ny][nx]    split detector residuals e_s (or per-line input of the spectral
//                            stages)
//   spec      [L][nblk][ny][kColBlock] complex64: half spectra (kx = 0 .. nx/2) stored in
//                            column blocks of kColBlock frequencies, so that a block holds whole
//                            columns contiguously (the column pass streams 32*ny bytes) and a
//                            group of kRows rows of a block is 128 contiguous bytes (the row
//                            passes write/read full 128-byte lines).
//   maxg      [kMaxgBlocks][3] per-block max |D_x Y|, max |D_y Y| and min X: the splat derives
//                            its halo and its fixed-point scales from them on the device, so
//                            no host round trip is needed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epr {

constexpr int kMaxLines = 16;
constexpr int kMaxStages = 16;
constexpr int kMaxDim = 4096;
constexpr int kColBlock = 4;     // complex columns per half-spectrum block
constexpr int kRows = 4;         // rows per workgroup in the row passes
constexpr int kMaxgBlocks = 256; // workgroups of the max-gradient reduction per problem
constexpr int kSplatThreads = 512;
constexpr int kSplatTileX = 64;  // default splat tile (columns x rows)
constexpr int kSplatTileY = 32;

// One FFT length: radix sequence and twiddle table. tw[j * tw_stride] = exp(-2 pi i j / n).
// The kernels copy the first tw_half(n) entries to LDS (the rest follow by W^(j+n/2) = -W^j).
__host__ __device__ inline int tw_half(int n) { return (n & 1) ? n : n >> 1; }
// FFT work buffers in LDS hold element j of a sequence in row j + (j >> kLdsPadShift): rows
// needed for elements 0..n.
constexpr int kLdsPadShift = 5;
__host__ __device__ inline int lds_rows(int n) { return n + (n >> kLdsPadShift) + 1; }
struct FftPlan {
  int n;
  int nst;
  int tw_stride;
  int radix[kMaxStages];
  const float2* tw;
  int variant;  // radix order of a compile-time length (0: default; see fft_variants)
};

// Radix orders compiled for the lengths with compile-time stage sequences, as a tunable launch
// choice: number of variants of a row (forward real-FFT half length) or column transform length
// (1 for every other length).
__host__ __device__ inline int fft_row_variants(int n) {
  return (n == 512 || n == 1024 || n == 1280) ? 3 : (n == 2048 ? 2 : 1);
}
__host__ __device__ inline int fft_col_variants(int n) {
  return (n == 1024 || n == 2048 || n == 2160) ? 3 : 1;
}

// Per-line constants of one problem (float, derived in double on the host).
//   I_s    = w_s exp(-a_s X)                   (Eq. 7, or absorption scaled to line s)
//   u_s    = b_s D Y          [pixels]         (Eq. 2 in pixel units)
//   WKB1   = q_s = (eps_s/p^2)^2 / 4           (Eq. 1, diffraction-pressure coefficient)
//   filter = 1 / (1 + h_s (fx^2 + fy^2)), h_s = 4 pi^2 alpha_s   (Section 2)
//   projection: tau = -inv_den sum_s mw_s ln(max(I_s + omega dI_s, floor_s) inv_w_s)
struct LineParams {
  int n;
  float w[kMaxLines];
  float a[kMaxLines];
  float b[kMaxLines];
  float q[kMaxLines];
  float h[kMaxLines];
  float mw[kMaxLines];
  float inv_w[kMaxLines];
  float floor_[kMaxLines];
  float a_hi[kMaxLines];  // largest a_s over the columns (x-dependent spectrum; else a_s)
  float b_absmax;     // max_s |b_s|
  float inv_den;      // 1 / sum_s w_s mu_s^2
  float phase_coef;   // phi_ref = phase_coef * tau
  float spec_scale;   // 2 / (nx ny): normalisation of the unnormalised forward/inverse pair
};

struct ProbDesc {
  int ny, nx;
  int nblk;           // ceil((nx/2 + 1) / kColBlock)
  int splat_tx, splat_ty;
  const float* X;
  const float* Y;
  const float* d;
  float* out;         // forward: detector intensity; adjoint/precondition: per-line output
  float* e;           // [L][ny][nx]
  float2* spec;       // [L][nblk][ny][kColBlock]
  float* tau;         // solve state, in/out
  float* phase_out;   // optional
  float* maxg;        // [kMaxgBlocks][3]
  float* resid;       // residual partial sums [splat blocks][2] (may be null)
  unsigned* status;   // set to 1 when an update meets a NaN or an infinity (may be null)
  FftPlan row;        // length nx/2 (twiddles of length nx, stride 2)
  FftPlan col;        // length ny
  float2* row_tw;     // exp(-2 pi i k / nx), k = 0..nx-1 (real-FFT post/pre-processing)
  LineParams lp;
  float relax;
  int os;             // oversampling factor f: ny x nx is the internal grid, d is the detector
                      // image of (ny/f) x (nx/f) pixels, each the mean of f x f internal pixels
  // x-dependent effective spectrum (null: the LineParams constants hold for every column):
  // xcol[(x * L + s) * 2] = {w, a, b, q}, xcol[(x * L + s) * 2 + 1] = {mw, 1/w, floor, 0} of
  // line s at column x, xden[x] = 1 / sum_s w mu^2 there.
  const float4* xcol;
  const float* xden;
  // block-wise preconditioner of an x-dependent spectrum (nbp = 0: the column-mean filter):
  // block 0's filtered spectra are `spec` (filtered in place), block b >= 1's are at
  // spec_blk + (b - 1) spec_set (complex values, same layout as spec); the column pass of
  // block b writes to spec_out (null: in place), and the row inverse blends the nbp blocks'
  // outputs per column with xblk[x] = {b0, t}.
  int nbp;
  int rlpb;           // row pass: lines per workgroup, transformed one after the other (1, 2, 4)
  float2* spec_out;
  float2* spec_blk;
  size_t spec_set;
  const float2* xblk;
};

// Line constants at one column of an x-dependent spectrum.
struct ColConst {
  float w, a, b, q;
};

// Kernel arguments: a single problem by value, or a device table of problems with per-stage
// block prefix sums (starts[i] = first block of problem i, starts[nprob] = total blocks).
struct KArgs {
  ProbDesc p;
  const ProbDesc* table;
  const int* starts;
  int nprob;
  int mode;
  int xdep;   // the problems carry an x-dependent spectrum (xcol / xden): the _x kernels run
  int rl;     // batched row pass: lines per workgroup of the launch's problems
  int ny_max; // batched column pass: largest ny of the launch's problems (0: not known)
};

// Modes
enum SplatMode { kSplatForward = 0, kSplatSplit = 1, kSplatLines = 2 };
enum RowMode { kRowGatherFft = 0, kRowCopyFft = 1, kRowGatherOnly = 2 };
enum RowInvMode { kRowInvSolve = 0, kRowInvPrecond = 1 };
enum LocalMode { kLocalForward = 0, kLocalSplit = 1, kLocalLines = 2 };
// closure order of the local kernel: 1, 2 (Eq. 1), or the diffraction-pressure term added to
// the transported per-line predictions held in e (second-order non-local model)
constexpr int kOrderTransportWkb1 = 3;

// Work decomposition (blocks per problem for each stage), shared by host and device.
__host__ __device__ inline int blocks_maxg(const ProbDesc&) { return kMaxgBlocks; }
__host__ __device__ inline int blocks_splat(const ProbDesc& p) {
  return ((p.ny + p.splat_ty - 1) / p.splat_ty) * ((p.nx + p.splat_tx - 1) / p.splat_tx);
}
__host__ __device__ inline int row_lines(const ProbDesc& p) { return p.rlpb > 1 ? p.rlpb : 1; }
__host__ __device__ inline int blocks_rowfft(const ProbDesc& p) {
  return ((p.ny + kRows - 1) / kRows) * ((p.lp.n + row_lines(p) - 1) / row_lines(p));
}
__host__ __device__ inline int blocks_colfft(const ProbDesc& p) { return p.nblk * p.lp.n; }
__host__ __device__ inline int blocks_rowinv(const ProbDesc& p) {
  return (p.ny + kRows - 1) / kRows;
}
constexpr int kLocalTile = 16;  // local closure: 16 x 16 outputs per workgroup
constexpr int kLocalHalo = 4;
__host__ __device__ inline int blocks_local(const ProbDesc& p) {
  return ((p.ny + kLocalTile - 1) / kLocalTile) * ((p.nx + kLocalTile - 1) / kLocalTile);
}
// detector-level residual on an oversampled grid: one detector pixel per thread, 256 threads
__host__ __device__ inline int blocks_binsplit(const ProbDesc& p) {
  return ((p.ny / p.os) * (p.nx / p.os) + 255) / 256;
}

// LDS bytes of each kernel for a problem
inline size_t lds_splat(const ProbDesc& p) {
  return sizeof(float) * (size_t)p.lp.n * (p.splat_tx + 2) * (p.splat_ty + 2);
}
// (transform buffer of one line, then the LDS twiddle table of the pass's FFT length)
inline size_t lds_rowfft(const ProbDesc& p) {
  return sizeof(float2) * ((size_t)kRows * lds_rows(p.nx / 2) + tw_half(p.nx / 2));
}
inline size_t lds_colfft(const ProbDesc& p) {
  return sizeof(float2) * ((size_t)kColBlock * lds_rows(p.ny) + tw_half(p.ny));
}
// (row inverse: the block's 4 x 4 spectral tiles as copied from HBM, the transform buffer,
// the table)
inline size_t lds_rowinv(const ProbDesc& p) {
  return sizeof(float2) * ((size_t)p.nblk * kColBlock * kRows + (size_t)kRows * lds_rows(p.nx / 2) +
                           tw_half(p.nx / 2));
}
// Threads of the spectral kernels for a problem: 512 up to 2048 x 2048, 1024 beyond.
inline int spectral_threads(const ProbDesc& p) { return (p.nx <= 2048 && p.ny <= 2048) ? 512 : 1024; }
// Longest column of the 1024-thread class's mid column-pass instance (2160-row detectors): built
// without the longer lengths, it fits eight waves per SIMD instead of four.
constexpr int kColMidMax = 2304;

// Launch wrappers (defined next to their kernels). `total_blocks` is the grid size; `lds` the
// dynamic LDS bytes. They return the hipError_t of the launch.
hipError_t launch_maxgrad(const KArgs& a, int total_blocks, hipStream_t s);
hipError_t launch_splat(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, int lines);
hipError_t launch_local(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, int order);
hipError_t launch_rowfft(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, int nt);
hipError_t launch_colfft(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, int nt);
hipError_t launch_rowinv(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, int nt);
hipError_t launch_resid_reduce(const KArgs& a, float* hist_slot, int nb, hipStream_t s);
hipError_t launch_binsplit(const KArgs& a, int total_blocks, hipStream_t s, int lines, int f);
// r [lines][ny/f][nx/f] -> out [lines][ny][nx]: each value over its f x f pixels, times 1/f^2
hipError_t launch_unbin_lines(const float* r, float* out, int ny, int nx, int f, int lines,
                              hipStream_t s);
hipError_t launch_vjp(const KArgs& a, int total_blocks, size_t lds, hipStream_t s, float* gx,
                      float* gy, float* ga);
// local closures (order 1, 2) or the pressure term added to the non-local gradients (order 3);
// work and q: [L][ny][nx] scratch planes (order >= 2).  Both VJP launchers read the line
// constants per column when a.p.xcol is set (x-dependent spectrum, X = Y = thickness).
hipError_t launch_vjp_local(const KArgs& a, int total_blocks, hipStream_t s, int order,
                            float* work, float* q, float* gx, float* gy, float* ga);
// gphase = D_x^T gx + D_y^T gy, or (accumulate != 0) gphase += that
hipError_t launch_vjp_transpose(const KArgs& a, int total_blocks, hipStream_t s,
                                const float* gx, const float* gy, float* gphase,
                                int accumulate);
size_t lds_local(int n_lines);
// Fixed scratch of the allocation-free solve (noalloc.hip): the device address of this GPU's
// copy of the scratch array (`device` must be the current device on the first call for it),
// and a W_n^j table (j < n) written into it by a kernel.
hipError_t noalloc_scratch_address(int device, void** out);
hipError_t launch_twiddle_table(float2* out, int n, hipStream_t s);
hipError_t set_transport_attributes();
hipError_t set_spectral_attributes();
hipError_t set_local_attributes();
hipError_t set_vjp_attributes();

}  // namespace epr
