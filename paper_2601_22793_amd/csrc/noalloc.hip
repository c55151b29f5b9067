// Fixed device scratch of epr_solve_noalloc.
//
// The solver's workspace (split residuals, half spectra, max-gradient and residual partials)
// and its two FFT twiddle tables are placed in one file-scope device array instead of
// hipMalloc'ed buffers, so that entry point allocates nothing.  Every GPU the library runs on
// holds its own copy of the array until the process ends.  In host code the array's name is
// only a host-side stand-in: its device address on each GPU comes from hipGetSymbolAddress,
// taken once per device at handle creation (with that device current), and only that address
// is ever passed to kernels or used in copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "epr.h"
#include "epr_internal.h"

namespace epr {

namespace {

__device__ __align__(256) unsigned char scratch[EPR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// W_n^j = exp(-2 pi i j / n), j < n, rounded from double to float.
__global__ __launch_bounds__(256) void k_twiddle_table(float2* out, int n) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < n) {
    double s, c;
    sincospi(-2.0 * (double)j / (double)n, &s, &c);
    out[j] = make_float2((float)c, (float)s);
  }
}

}  // namespace

hipError_t noalloc_scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_twiddle_table(float2* out, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddle_table, dim3((n + 255) / 256), dim3(256), 0, s, out, n);
  return hipGetLastError();
}

}  // namespace epr
