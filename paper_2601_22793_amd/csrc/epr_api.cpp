// Host side of libepr: the C ABI of include/epr.h.
//
// Validation, per-line constants (in double, rounded once to float), FFT plans, workspace,
// the launch sequence of one EPR iteration (Methods 4.4), the batched solver with its HIP
// graph cache, diagnostics and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <functional>
#include <map>
#include <tuple>
#include <memory>
#include <string>
#include <vector>

#include "../../include/epr.h"
#include "epr_internal.h"
#include "regime.h"

using namespace epr;

namespace {

constexpr double kHcEvM = 1.239841984e-6;  // h c [eV m]
constexpr double kPi = 3.14159265358979323846;
constexpr int kStatusWords = 1024;      // non-finite flags held without growing the buffer
constexpr size_t kSolveGraphCap = 64;   // cached single-problem solve graphs per handle

void key_append(std::vector<uint8_t>& k, const void* p, size_t n) {
  const uint8_t* b = static_cast<const uint8_t*>(p);
  k.insert(k.end(), b, b + n);
}

thread_local std::string g_create_error;

// --------------------------------------------------------------------------------------------
// FFT plans
// --------------------------------------------------------------------------------------------

// Radix sequence for n (product of 2, 3, 5): radix 16 first, then the rest of the power of
// two as 8 / 4 / 2, then 5s and 3s.  Returns the number of stages, or -1.
int factorize(int n, int* radix, int cap) {
  if (n < 1) return -1;
  int m = n, k = 0;
  int p2 = 0;
  while (m % 2 == 0) { m /= 2; ++p2; }
  int c5 = 0, c3 = 0;
  while (m % 5 == 0) { m /= 5; ++c5; }
  while (m % 3 == 0) { m /= 3; ++c3; }
  if (m != 1) return -1;
  auto push = [&](int r) { if (k < cap) radix[k] = r; ++k; };
  while (p2 >= 4) { push(16); p2 -= 4; }
  if (p2 == 3) push(8);
  if (p2 == 2) push(4);
  if (p2 == 1) push(2);
  for (int i = 0; i < c5; ++i) push(5);
  for (int i = 0; i < c3; ++i) push(3);
  if (n == 1) return 0;
  return k <= cap ? k : -1;
}

bool smooth235(int n) {
  int r[kMaxStages * 2];
  return factorize(n, r, kMaxStages * 2) >= 0;
}

struct Twiddles {
  float2* dev = nullptr;
  int n = 0;
};

// --------------------------------------------------------------------------------------------
// Device buffers
// --------------------------------------------------------------------------------------------
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace

// Prepared batched launch sequence: the device problem table, sorted into groups of one
// spectral size class each (one launch per stage and group), with per-stage block prefix sums.
struct BatchGroup {
  ProbDesc* table = nullptr;   // first problem of the group in the device table
  int* starts = nullptr;       // [ns][n + 1] prefix sums of this group
  int n = 0;
  int nt = 512;                // spectral threads of the group
  int lpb = 1;                 // row-pass lines per workgroup of the group
  int total[8] = {};
  size_t lds_sp = 0, lds_rf = 0, lds_cf = 0, lds_ri = 0;
};
struct BatchPlan {
  std::vector<ProbDesc> descs;  // host copy of the device table (diagnostics)
  BatchGroup grp[2];
  int ngroups = 0;
  int L = 0, ns = 0, n_iter = 0, order = 2, os = 1;
  bool nonlocal = true;         // a transport model (the max-gradient partials are valid)
  bool xdep = false;            // x-dependent spectra (the problems carry per-column tables)
  std::vector<int> stages;      // BatchStage of each launch of an iteration, in order
  unsigned* status = nullptr;   // per-problem non-finite flags, caller's order
  int n = 0;
  bool want_resid = false;      // residual history of the caller's problem 0
  ProbDesc resid_desc{};        // that problem (its resid partials are written by the split)
  int resid_group = 0;          // the size-class group that holds it
};

struct epr_ctx {
  int device = 0;
  BatchPlan batch;
  std::string last_error;
  std::map<int, Twiddles> tw;           // length -> W_n table
  DevBuf ws;                            // single-problem workspace
  DevBuf hist;                          // residual history (256 floats)
  DevBuf batch_ws;                      // batched workspace
  DevBuf batch_table;                   // device ProbDesc table + stage starts
  DevBuf batch_xtab;                    // per-column tables of a batched x-dependent solve
  DevBuf sel;                           // model selection: Paganin thickness + counts
  DevBuf xtab;                          // per-column constants of an x-dependent spectrum
  DevBuf status;                        // per-problem non-finite flags of the last solve
  void* scratch = nullptr;              // this device's fixed scratch array (epr_solve_noalloc)
  std::vector<float> blk_h;             // block-wise preconditioner: h of block b, line s at [b L + s]
  hipStream_t cap_stream = nullptr;     // capture stream for graphs
  hipStream_t cap_stream2 = nullptr;    // second branch of a batched graph (size class 1)
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;  // fork / join of that branch
  // batched graph cache
  std::vector<uint8_t> graph_key;
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t batch_stream = nullptr;   // stream of the last batched replay
  // single-problem solve graphs, least recently used evicted first
  struct SolveGraph {
    std::vector<uint8_t> key;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t used;
  };
  std::vector<SolveGraph> solve_graphs;
  uint64_t graph_clock = 0;
  // diagnostics
  hipStream_t last_stream = nullptr;
  int last_n_iter = 0;
  int last_nprob = 0;
  bool last_resid = false;
  bool last_nonlocal = false;  // the max-gradient partials are valid only after a non-local solve
  int last_model = 0;
  int last_status_n = 0;       // flags of the last solve (caller's order) in `status`
  std::vector<ProbDesc> last_descs;
  // tuned launch shape
  int splat_tx = kSplatTileX, splat_ty = kSplatTileY;
  std::map<int, int> fft_row_var, fft_col_var;  // tuned radix order per transform length
  int row_lines = 1;                            // tuned lines per row-pass workgroup (1 or 2)
  uint32_t tune_gen = 0;                        // bumped whenever a tuned choice changes
  DevBuf tune_ws, tune_tau;                     // autotuner workspace and warm thickness
  // stage timing
  struct EvPair {
    hipEvent_t a, b;
    int stage;
    int cls;   // size class of the launch's problems (0: up to 2048 x 2048, 1: larger)
  };
  bool timing = false;
  std::vector<EvPair> pending;   // plain launches not folded yet
  std::vector<hipEvent_t> pool;
  double tms[EPR_N_STAGES] = {};
  int64_t tcount[EPR_N_STAGES] = {};
  double tms_cls[EPR_N_STAGES][2] = {};
  int64_t tcount_cls[EPR_N_STAGES][2] = {};

  int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error = buf;
    return code;
  }
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

#define HIP_TRY(h, expr)                                                                    \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return (h)->fail(EPR_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

int ensure(epr_ctx* h, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes) return EPR_OK;
  if (b.ptr) {
    (void)hipDeviceSynchronize();
    (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return h->fail(EPR_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  }
  b.bytes = bytes;
  return EPR_OK;
}

hipEvent_t take_event(epr_ctx* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Add the elapsed times of recorded event pairs to the totals (events must be complete).
int fold_events(epr_ctx* h, std::vector<epr_ctx::EvPair>& v, bool recycle) {
  for (auto& ev : v) {
    float ms = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&ms, ev.a, ev.b));
    h->tms[ev.stage] += ms;
    h->tcount[ev.stage] += 1;
    h->tms_cls[ev.stage][ev.cls] += ms;
    h->tcount_cls[ev.stage][ev.cls] += 1;
    if (recycle) {
      h->pool.push_back(ev.a);
      h->pool.push_back(ev.b);
    }
  }
  if (recycle) v.clear();
  return EPR_OK;
}

// Launch one stage on `st`; in timing mode bracket it with events (appended to `sink`).
template <class F>
int run_stage(epr_ctx* h, int stage, hipStream_t st, std::vector<epr_ctx::EvPair>* sink,
              F launch, int cls = 0) {
  epr_ctx::EvPair ev{nullptr, nullptr, stage, cls};
  if (h->timing) {
    ev.a = take_event(h);
    ev.b = take_event(h);
    if (!ev.a || !ev.b) return h->fail(EPR_ERR_HIP, "hipEventCreate failed");
    HIP_TRY(h, hipEventRecord(ev.a, st));
  }
  hipError_t e = launch();
  if (e != hipSuccess) return h->fail(EPR_ERR_HIP, "kernel launch (stage %d): %s", stage,
                                      hipGetErrorString(e));
  if (h->timing) {
    HIP_TRY(h, hipEventRecord(ev.b, st));
    sink->push_back(ev);
    if (sink == &h->pending && h->pending.size() > 4096) {
      HIP_TRY(h, hipStreamSynchronize(st));
      return fold_events(h, h->pending, true);
    }
  }
  return EPR_OK;
}

enum Stage { kStMaxg = 0, kStSplat = 1, kStLocal = 2, kStRowFft = 3, kStColFft = 4,
             kStRowInv = 5, kStVjp = 6, kStBinSplit = 7 };

// Launches of a batched iteration.
enum BatchStage { kBsMaxg, kBsSplatSplit, kBsSplatLines, kBsLocalSplit, kBsLocalLines,
                  kBsWkb1Split, kBsWkb1Lines, kBsBinSplit, kBsRowGather, kBsRowCopy, kBsColFft,
                  kBsRowInv };

const float2* twiddles(epr_ctx* h, int n, int* status) {
  auto it = h->tw.find(n);
  if (it != h->tw.end()) return it->second.dev;
  std::vector<float2> t(n);
  for (int j = 0; j < n; ++j) {
    const double ang = -2.0 * kPi * (double)j / (double)n;
    t[j] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  Twiddles tw;
  tw.n = n;
  hipError_t e = hipMalloc(&tw.dev, sizeof(float2) * n);
  if (e == hipSuccess) e = hipMemcpy(tw.dev, t.data(), sizeof(float2) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    *status = h->fail(EPR_ERR_HIP, "twiddle table %d: %s", n, hipGetErrorString(e));
    return nullptr;
  }
  h->tw[n] = tw;
  return tw.dev;
}

// `table`: a W_table_n table the caller provides (else the handle's cached one).
int make_plan(epr_ctx* h, int n, int table_n, int stride, FftPlan* out,
              const float2* table = nullptr) {
  out->n = n;
  out->tw_stride = stride;
  out->nst = factorize(n, out->radix, kMaxStages);
  if (out->nst < 0) return h->fail(EPR_ERR_SHAPE, "FFT length %d is not a product of 2, 3, 5", n);
  int st = EPR_OK;
  out->tw = table ? table : twiddles(h, table_n, &st);
  return st;
}

// --------------------------------------------------------------------------------------------
// Validation
// --------------------------------------------------------------------------------------------
int check_geometry(epr_ctx* h, const epr_geometry* g) {
  if (!g) return h->fail(EPR_ERR_INVALID_ARG, "geometry is NULL");
  if (g->ny < 8 || g->nx < 8 || g->ny > kMaxDim || g->nx > kMaxDim)
    return h->fail(EPR_ERR_SHAPE, "image %dx%d outside 8..%d", g->ny, g->nx, kMaxDim);
  if (g->nx % 2 != 0) return h->fail(EPR_ERR_SHAPE, "nx = %d must be even", g->nx);
  if (!smooth235(g->ny) || !smooth235(g->nx))
    return h->fail(EPR_ERR_SHAPE, "image %dx%d: sizes must be products of 2, 3 and 5", g->ny,
                   g->nx);
  if (!(g->pixel_m > 0.0) || !std::isfinite(g->pixel_m))
    return h->fail(EPR_ERR_INVALID_ARG, "pixel size must be positive and finite");
  if (!(g->distance_m >= 0.0) || !std::isfinite(g->distance_m))
    return h->fail(EPR_ERR_INVALID_ARG, "distance must be >= 0 and finite");
  return EPR_OK;
}

// n_lines, reference energy and exponents (the line arrays are checked by check_spectrum)
int check_spectrum_header(epr_ctx* h, const epr_spectrum* s) {
  if (!s) return h->fail(EPR_ERR_INVALID_ARG, "spectrum is NULL");
  if (s->n_lines < 1 || s->n_lines > kMaxLines)
    return h->fail(EPR_ERR_INVALID_ARG, "n_lines = %d outside 1..%d", s->n_lines, kMaxLines);
  if (!(s->energy_ref_kev > 0.0) || !std::isfinite(s->energy_ref_kev))
    return h->fail(EPR_ERR_INVALID_ARG, "reference energy must be positive");
  if (!std::isfinite(s->delta_exponent) || !std::isfinite(s->beta_exponent))
    return h->fail(EPR_ERR_INVALID_ARG, "exponents must be finite");
  return EPR_OK;
}

int check_spectrum(epr_ctx* h, const epr_spectrum* s) {
  if (!s) return h->fail(EPR_ERR_INVALID_ARG, "spectrum is NULL");
  if (s->n_lines < 1 || s->n_lines > kMaxLines)
    return h->fail(EPR_ERR_INVALID_ARG, "n_lines = %d outside 1..%d", s->n_lines, kMaxLines);
  if (!s->energy_kev || !s->weight) return h->fail(EPR_ERR_INVALID_ARG, "spectrum arrays NULL");
  double sw = 0.0;
  for (int i = 0; i < s->n_lines; ++i) {
    if (!(s->energy_kev[i] > 0.0) || !std::isfinite(s->energy_kev[i]))
      return h->fail(EPR_ERR_INVALID_ARG, "energy[%d] must be positive", i);
    if (!(s->weight[i] > 0.0) || !std::isfinite(s->weight[i]))
      return h->fail(EPR_ERR_INVALID_ARG, "weight[%d] must be positive", i);
    sw += s->weight[i];
  }
  if (std::fabs(sw - 1.0) > 1e-6)
    return h->fail(EPR_ERR_INVALID_ARG, "weights sum to %.9g, not 1", sw);
  if (!(s->energy_ref_kev > 0.0) || !std::isfinite(s->energy_ref_kev))
    return h->fail(EPR_ERR_INVALID_ARG, "reference energy must be positive");
  if (!std::isfinite(s->delta_exponent) || !std::isfinite(s->beta_exponent))
    return h->fail(EPR_ERR_INVALID_ARG, "exponents must be finite");
  return EPR_OK;
}

int check_profile(epr_ctx* h, const epr_spectrum_profile* pr, int n_lines) {
  if (!pr) return h->fail(EPR_ERR_INVALID_ARG, "profile is NULL");
  if (pr->n_blocks < 1 || pr->n_blocks > 4096)
    return h->fail(EPR_ERR_INVALID_ARG, "n_blocks = %d outside 1..4096", pr->n_blocks);
  if (!pr->block_x || !pr->energy_kev || !pr->weight)
    return h->fail(EPR_ERR_INVALID_ARG, "profile arrays NULL");
  for (int b = 0; b < pr->n_blocks; ++b) {
    if (!std::isfinite(pr->block_x[b]) || (b > 0 && !(pr->block_x[b] > pr->block_x[b - 1])))
      return h->fail(EPR_ERR_INVALID_ARG, "block_x must be finite and increasing");
    double sw = 0.0;
    for (int i = 0; i < n_lines; ++i) {
      const double e = pr->energy_kev[b * n_lines + i], w = pr->weight[b * n_lines + i];
      if (!(e > 0.0) || !std::isfinite(e))
        return h->fail(EPR_ERR_INVALID_ARG, "block %d energy[%d] must be positive", b, i);
      if (!(w > 0.0) || !std::isfinite(w))
        return h->fail(EPR_ERR_INVALID_ARG, "block %d weight[%d] must be positive", b, i);
      sw += w;
    }
    if (std::fabs(sw - 1.0) > 1e-6)
      return h->fail(EPR_ERR_INVALID_ARG, "block %d weights sum to %.9g, not 1", b, sw);
  }
  return EPR_OK;
}

int check_material(epr_ctx* h, const epr_material* m) {
  if (!m) return h->fail(EPR_ERR_INVALID_ARG, "material is NULL");
  if (!(m->delta_ref > 0.0) || !(m->beta_ref > 0.0) || !std::isfinite(m->delta_ref) ||
      !std::isfinite(m->beta_ref))
    return h->fail(EPR_ERR_INVALID_ARG, "delta_ref and beta_ref must be positive");
  return EPR_OK;
}

int check_model(epr_ctx* h, int model) {
  if (model != EPR_LOCAL_L1 && model != EPR_LOCAL_L2 && model != EPR_NONLOCAL &&
      model != EPR_NONLOCAL_L2)
    return h->fail(EPR_ERR_INVALID_ARG, "unknown model %d", model);
  return EPR_OK;
}

int check_opts(epr_ctx* h, const epr_opts* o, bool allow_auto, bool allow_block = false) {
  if (!o) return h->fail(EPR_ERR_INVALID_ARG, "opts is NULL");
  if (o->model == EPR_AUTO) {
    if (!allow_auto)
      return h->fail(EPR_ERR_UNSUPPORTED, "EPR_AUTO is accepted by epr_solve only");
  } else {
    int st = check_model(h, o->model);
    if (st) return st;
  }
  if (o->n_iter < 0) return h->fail(EPR_ERR_INVALID_ARG, "n_iter must be >= 0");
  if (!(o->relaxation > 0.0 && o->relaxation <= 2.0))
    return h->fail(EPR_ERR_INVALID_ARG, "relaxation must lie in (0, 2]");
  if (o->flags & ~(EPR_FLAG_RESIDUALS | EPR_FLAG_BLOCK_PRECOND))
    return h->fail(EPR_ERR_INVALID_ARG, "unknown flags");
  if ((o->flags & EPR_FLAG_BLOCK_PRECOND) && !allow_block)
    return h->fail(EPR_ERR_UNSUPPORTED, "EPR_FLAG_BLOCK_PRECOND is accepted by epr_solve_xspec only");
  if (o->oversample != 0 && o->oversample != 1 && o->oversample != 2 && o->oversample != 4)
    return h->fail(EPR_ERR_INVALID_ARG, "oversample = %d: use 1, 2 or 4", o->oversample);
  return EPR_OK;
}

// Internal grid of an oversampled solve: f times the pixels per axis, pixel p / f.
epr_geometry internal_geometry(const epr_geometry& g, int f) {
  epr_geometry gf = g;
  gf.ny = g.ny * f;
  gf.nx = g.nx * f;
  gf.pixel_m = g.pixel_m / f;
  return gf;
}

int check_internal(epr_ctx* h, const epr_geometry* g, const epr_opts* o) {
  if (!o || o->oversample <= 1) return EPR_OK;
  const epr_geometry gf = internal_geometry(*g, o->oversample);
  const int st = check_geometry(h, &gf);
  if (st) {
    const std::string m = h->last_error;
    return h->fail(st, "internal grid of oversample %d: %s", o->oversample, m.c_str());
  }
  return EPR_OK;
}

// --------------------------------------------------------------------------------------------
// Per-line constants
// --------------------------------------------------------------------------------------------
struct LineDouble {
  double w, k, delta, beta, mu, eps_px, alpha_px, phase_scale, absorb_scale;
};

std::vector<LineDouble> lines_double(const epr_geometry& g, const epr_spectrum& s, double dref,
                                     double bref) {
  std::vector<LineDouble> out(s.n_lines);
  const double eref = s.energy_ref_kev * 1e3;
  const double kref = 2.0 * kPi * eref / kHcEvM;
  for (int i = 0; i < s.n_lines; ++i) {
    LineDouble& l = out[i];
    const double e = s.energy_kev[i] * 1e3;
    l.w = s.weight[i];
    l.k = 2.0 * kPi * e / kHcEvM;
    const double ratio = eref / e;
    l.delta = dref * std::pow(ratio, s.delta_exponent);
    l.beta = bref * std::pow(ratio, s.beta_exponent);
    l.mu = 2.0 * l.k * l.beta;
    l.eps_px = g.distance_m / l.k / (g.pixel_m * g.pixel_m);
    l.alpha_px = l.eps_px * l.delta / (2.0 * l.beta);
    l.phase_scale = (l.k * l.delta) / (kref * dref);
    l.absorb_scale = l.mu / (2.0 * kref * bref);
  }
  return out;
}

enum class Kind { Solve, Maps };

// Solve: X = Y = tau, I_s = w exp(-mu_s tau), u_s = -(L delta_s / p^2) D tau.
// Maps (forward/adjoint/vjp): X = absorption, Y = phase at E_ref,
//   I_s = w exp(-(mu_s/mu_ref) A), u_s = eps_s phase_scale_s D phase.
LineParams line_params(const epr_geometry& g, const epr_spectrum& s, const epr_material* m,
                       Kind kind, double relax_unused = 0.0) {
  (void)relax_unused;
  const double dref = m ? m->delta_ref : 1.0, bref = m ? m->beta_ref : 1.0;
  std::vector<LineDouble> ld = lines_double(g, s, dref, bref);
  LineParams lp;
  std::memset(&lp, 0, sizeof lp);
  lp.n = s.n_lines;
  double den = 0.0, bmax = 0.0;
  for (int i = 0; i < s.n_lines; ++i) {
    const LineDouble& l = ld[i];
    double a, b;
    if (kind == Kind::Solve) {
      a = l.mu;
      b = -l.eps_px * l.k * l.delta;  // = -L delta_s / p^2
    } else {
      a = l.absorb_scale;
      b = l.eps_px * l.phase_scale;
    }
    lp.w[i] = (float)l.w;
    lp.a[i] = (float)a;
    lp.b[i] = (float)b;
    lp.q[i] = (float)(0.25 * l.eps_px * l.eps_px);
    lp.h[i] = (float)(4.0 * kPi * kPi * l.alpha_px);
    lp.mw[i] = (float)(l.w * l.mu);
    lp.inv_w[i] = (float)(1.0 / l.w);
    lp.floor_[i] = (float)(1e-6 * l.w);
    den += l.w * l.mu * l.mu;
    bmax = std::max(bmax, std::fabs((double)lp.b[i]));
  }
  lp.b_absmax = (float)bmax;
  for (int i = 0; i < s.n_lines; ++i) lp.a_hi[i] = lp.a[i];
  lp.inv_den = (float)(1.0 / den);
  const double kref = 2.0 * kPi * s.energy_ref_kev * 1e3 / kHcEvM;
  lp.phase_coef = (float)(-kref * dref);
  lp.spec_scale = (float)(2.0 / ((double)g.nx * (double)g.ny));
  return lp;
}

// Per-column constants of an x-dependent spectrum (ProbDesc::xcol / xden layout) and the
// LineParams that go with them: w, a (smallest over the columns) and a_hi bound the line
// intensities for the splat's fixed-point scales, b_absmax bounds the shifts, and h is the
// column-mean preconditioner.  Energy and weight of every line are interpolated linearly
// between the block centres (held constant beyond the outer ones); all constants follow from
// them as in lines_double.
struct XTable {
  std::vector<float4> col;
  std::vector<float> den;
  std::vector<float2> blk;    // per column {b0, t}: interpolation position between centres
  std::vector<float> blk_h;   // [block][line] 4 pi^2 alpha_s at the block's energies
  LineParams lp;
};

// g is the grid the solver works on; with oversampling by f its column x sits at detector
// coordinate (x + 1/2) / f - 1/2, where the profile (given in detector columns) is read.
XTable xspec_table(const epr_geometry& g, const epr_spectrum& s, const epr_spectrum_profile& pr,
                   const epr_material& m, int f) {
  const int L = s.n_lines, nx = g.nx, B = pr.n_blocks;
  XTable t;
  t.col.resize((size_t)nx * L * 2);
  t.den.resize(nx);
  t.blk.resize(nx);
  t.blk_h.resize((size_t)B * L);
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < L; ++i) {
      // alpha_s = eps_s delta_s / (2 beta_s) at block b's energy of line s (internal pixel)
      const double e = pr.energy_kev[b * L + i] * 1e3;
      const double k = 2.0 * kPi * e / kHcEvM;
      const double ratio = s.energy_ref_kev * 1e3 / e;
      const double delta = m.delta_ref * std::pow(ratio, s.delta_exponent);
      const double beta = m.beta_ref * std::pow(ratio, s.beta_exponent);
      const double eps = g.distance_m / k / (g.pixel_m * g.pixel_m);
      t.blk_h[(size_t)b * L + i] = (float)(4.0 * kPi * kPi * eps * delta / (2.0 * beta));
    }
  LineParams& lp = t.lp;
  std::memset(&lp, 0, sizeof lp);
  lp.n = L;
  std::vector<double> amean(L, 0.0), wmax(L, 0.0), amin(L, HUGE_VAL), amax(L, 0.0);
  double bmax = 0.0;
  const double eref = s.energy_ref_kev * 1e3, p2 = g.pixel_m * g.pixel_m;
  const double* bx = pr.block_x;
  for (int x = 0; x < nx; ++x) {
    const double xd = f > 1 ? (x + 0.5) / f - 0.5 : (double)x;
    int j = 0;
    double u = 0.0;  // position between centres j and j + 1
    if (xd >= bx[B - 1]) {
      j = B - 1;
    } else if (xd > bx[0]) {
      while (bx[j + 1] < xd) ++j;
      u = (xd - bx[j]) / (bx[j + 1] - bx[j]);
    }
    t.blk[x] = make_float2((float)j, (float)u);
    double den = 0.0;
    for (int i = 0; i < L; ++i) {
      double ek = pr.energy_kev[j * L + i], w = pr.weight[j * L + i];
      if (u > 0.0) {
        ek += u * (pr.energy_kev[(j + 1) * L + i] - ek);
        w += u * (pr.weight[(j + 1) * L + i] - w);
      }
      const double e = ek * 1e3;
      const double k = 2.0 * kPi * e / kHcEvM;
      const double ratio = eref / e;
      const double delta = m.delta_ref * std::pow(ratio, s.delta_exponent);
      const double beta = m.beta_ref * std::pow(ratio, s.beta_exponent);
      const double mu = 2.0 * k * beta;
      const double eps = g.distance_m / k / p2;
      const double b = -eps * k * delta;
      t.col[((size_t)x * L + i) * 2] =
          make_float4((float)w, (float)mu, (float)b, (float)(0.25 * eps * eps));
      t.col[((size_t)x * L + i) * 2 + 1] =
          make_float4((float)(w * mu), (float)(1.0 / w), (float)(1e-6 * w), 0.f);
      den += w * mu * mu;
      amean[i] += eps * delta / (2.0 * beta);
      wmax[i] = std::max(wmax[i], w);
      amin[i] = std::min(amin[i], mu);
      amax[i] = std::max(amax[i], mu);
      bmax = std::max(bmax, std::fabs((double)(float)b));
    }
    t.den[x] = (float)(1.0 / den);
  }
  for (int i = 0; i < L; ++i) {
    lp.w[i] = (float)wmax[i];
    lp.a[i] = (float)amin[i];
    lp.a_hi[i] = (float)amax[i];
    lp.h[i] = (float)(4.0 * kPi * kPi * amean[i] / nx);
    lp.inv_w[i] = 1.f;
  }
  lp.b_absmax = (float)bmax;
  lp.inv_den = 1.f;
  const double kref = 2.0 * kPi * eref / kHcEvM;
  lp.phase_coef = (float)(-kref * m.delta_ref);
  lp.spec_scale = (float)(2.0 / ((double)g.nx * (double)g.ny));
  return t;
}

// Sizes of the per-problem workspace pieces (bytes, 256-aligned).
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
struct WsLayout {
  size_t e, spec, maxg, resid, total;
};
WsLayout ws_layout(int ny, int nx, int L, int tx, int ty) {
  WsLayout w;
  const int nblk = (nx / 2 + 1 + kColBlock - 1) / kColBlock;
  w.e = align256(sizeof(float) * (size_t)L * ny * nx);
  w.spec = align256(sizeof(float2) * (size_t)L * nblk * ny * kColBlock);
  w.maxg = align256(sizeof(float) * 3 * kMaxgBlocks);
  const size_t nb = (size_t)((ny + ty - 1) / ty) * ((nx + tx - 1) / tx);
  w.resid = align256(sizeof(float) * 2 * std::max(nb, (size_t)((ny + 15) / 16) * ((nx + 15) / 16)));
  w.total = w.e + w.spec + w.maxg + w.resid;
  return w;
}

// Copy an x-dependent table to the handle's device copy (the columns' constants, then 1/den,
// then the block positions).  Earlier calls on this handle may still read the old table: they
// are let finish first.
int upload_xtable(epr_ctx* h, const XTable& t, hipStream_t st, const float4** col,
                  const float** den, const float2** blk) {
  const size_t cb = align256(sizeof(float4) * t.col.size());
  const size_t db = align256(sizeof(float) * t.den.size());
  const int e = ensure(h, h->xtab, cb + db + sizeof(float2) * t.blk.size());
  if (e != EPR_OK) return e;
  HIP_TRY(h, hipStreamSynchronize(st));
  char* base = static_cast<char*>(h->xtab.ptr);
  HIP_TRY(h, hipMemcpy(base, t.col.data(), sizeof(float4) * t.col.size(), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(base + cb, t.den.data(), sizeof(float) * t.den.size(),
                       hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(base + cb + db, t.blk.data(), sizeof(float2) * t.blk.size(),
                       hipMemcpyHostToDevice));
  *col = reinterpret_cast<const float4*>(base);
  *den = reinterpret_cast<const float*>(base + cb);
  *blk = reinterpret_cast<const float2*>(base + cb + db);
  return EPR_OK;
}

// row_tab / col_tab: W_nx and W_ny tables the caller provides (else the handle's cached ones).
int fill_desc(epr_ctx* h, const epr_geometry& g, const LineParams& lp, char* base, ProbDesc* p,
              const float2* row_tab = nullptr, const float2* col_tab = nullptr) {
  std::memset(p, 0, sizeof *p);
  p->ny = g.ny;
  p->nx = g.nx;
  p->nblk = (g.nx / 2 + 1 + kColBlock - 1) / kColBlock;
  p->splat_tx = h->splat_tx;
  p->splat_ty = h->splat_ty;
  p->lp = lp;
  p->os = 1;
  WsLayout w = ws_layout(g.ny, g.nx, lp.n, h->splat_tx, h->splat_ty);
  if (base) {
    p->e = reinterpret_cast<float*>(base);
    p->spec = reinterpret_cast<float2*>(base + w.e);
    p->maxg = reinterpret_cast<float*>(base + w.e + w.spec);
    p->resid = reinterpret_cast<float*>(base + w.e + w.spec + w.maxg);
  }
  int st = make_plan(h, g.nx / 2, g.nx, 2, &p->row, row_tab);
  if (st) return st;
  st = make_plan(h, g.ny, g.ny, 1, &p->col, col_tab);
  if (st) return st;
  auto rv = h->fft_row_var.find(g.nx / 2), cv = h->fft_col_var.find(g.ny);
  p->row.variant = rv == h->fft_row_var.end() ? 0 : rv->second;
  p->col.variant = cv == h->fft_col_var.end() ? 0 : cv->second;
  p->row_tw = const_cast<float2*>(p->row.tw);
  return EPR_OK;
}

// The solves' row pass takes the tuned lines per workgroup where it applies (rows up to 2048
// pixels, the 512-thread class; not the x-dependent kernels).
void apply_row_lines(const epr_ctx* h, ProbDesc* p) {
  p->rlpb = (h->row_lines == 2 && spectral_threads(*p) == 512 && p->xcol == nullptr) ? 2 : 1;
}

KArgs single(const ProbDesc& p, int mode) {
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.p = p;
  a.mode = mode;
  return a;
}

bool transport_model(int model) { return model == EPR_NONLOCAL || model == EPR_NONLOCAL_L2; }

// Max-gradient partials and every line's transported prediction M_s[I_s] into e.
int launch_transport_lines(epr_ctx* h, const ProbDesc& p, hipStream_t st, int cls) {
  auto* sink = &h->pending;
  int rc = run_stage(h, kStMaxg, st, sink,
                     [&] { return launch_maxgrad(single(p, 0), blocks_maxg(p), st); }, cls);
  if (rc) return rc;
  return run_stage(h, kStSplat, st, sink, [&] {
    return launch_splat(single(p, kSplatLines), blocks_splat(p), lds_splat(p), st, p.lp.n);
  }, cls);
}

// Predictions on an oversampled internal grid: every line's P_s into e, then the detector-level
// sum, residual and split, replicated back onto the internal grid.
int launch_lines_binsplit(epr_ctx* h, const ProbDesc& p, int model, hipStream_t st,
                          float* hist_slot, int cls) {
  auto* sink = &h->pending;
  int rc;
  if (model == EPR_NONLOCAL) {
    rc = launch_transport_lines(h, p, st, cls);
  } else if (model == EPR_NONLOCAL_L2) {
    rc = launch_transport_lines(h, p, st, cls);
    if (rc) return rc;
    rc = run_stage(h, kStLocal, st, sink, [&] {
      return launch_local(single(p, kLocalLines), blocks_local(p), lds_local(p.lp.n), st,
                          kOrderTransportWkb1);
    }, cls);
  } else {
    rc = run_stage(h, kStLocal, st, sink, [&] {
      return launch_local(single(p, kLocalLines), blocks_local(p), lds_local(p.lp.n), st,
                          model == EPR_LOCAL_L1 ? 1 : 2);
    }, cls);
  }
  if (rc) return rc;
  rc = run_stage(h, kStBinSplit, st, sink, [&] {
    return launch_binsplit(single(p, 0), blocks_binsplit(p), st, p.lp.n, p.os);
  }, cls);
  if (rc) return rc;
  if (hist_slot) HIP_TRY(h, launch_resid_reduce(single(p, 0), hist_slot, blocks_binsplit(p), st));
  return EPR_OK;
}

// One EPR iteration of a single problem (plain path: one launch per stage).
int launch_iteration(epr_ctx* h, const ProbDesc& p, int model, hipStream_t st, float* hist_slot) {
  const int cls = spectral_threads(p) == 1024 ? 1 : 0;
  auto* sink = &h->pending;
  int rc;
  if (p.os > 1) {
    rc = launch_lines_binsplit(h, p, model, st, hist_slot, cls);
    if (rc) return rc;
    rc = run_stage(h, kStRowFft, st, sink, [&] {
      return launch_rowfft(single(p, transport_model(model) ? kRowGatherFft : kRowCopyFft),
                           blocks_rowfft(p), lds_rowfft(p), st, spectral_threads(p));
    }, cls);
    if (rc) return rc;
  } else if (model == EPR_NONLOCAL_L2) {
    rc = launch_transport_lines(h, p, st, cls);
    if (rc) return rc;
    rc = run_stage(h, kStLocal, st, sink, [&] {
      return launch_local(single(p, kLocalSplit), blocks_local(p), lds_local(p.lp.n), st,
                          kOrderTransportWkb1);
    }, cls);
    if (rc) return rc;
    if (hist_slot) HIP_TRY(h, launch_resid_reduce(single(p, 0), hist_slot, blocks_local(p), st));
    rc = run_stage(h, kStRowFft, st, sink, [&] {
      return launch_rowfft(single(p, kRowGatherFft), blocks_rowfft(p), lds_rowfft(p), st, spectral_threads(p));
    }, cls);
    if (rc) return rc;
  } else if (model == EPR_NONLOCAL) {
    rc = run_stage(h, kStMaxg, st, sink,
                   [&] { return launch_maxgrad(single(p, 0), blocks_maxg(p), st); }, cls);
    if (rc) return rc;
    rc = run_stage(h, kStSplat, st, sink, [&] {
      return launch_splat(single(p, kSplatSplit), blocks_splat(p), lds_splat(p), st, p.lp.n);
    }, cls);
    if (rc) return rc;
    if (hist_slot) HIP_TRY(h, launch_resid_reduce(single(p, 0), hist_slot, blocks_splat(p), st));
    rc = run_stage(h, kStRowFft, st, sink, [&] {
      return launch_rowfft(single(p, kRowGatherFft), blocks_rowfft(p), lds_rowfft(p), st, spectral_threads(p));
    }, cls);
    if (rc) return rc;
  } else {
    rc = run_stage(h, kStLocal, st, sink, [&] {
      return launch_local(single(p, kLocalSplit), blocks_local(p), lds_local(p.lp.n), st,
                          model == EPR_LOCAL_L1 ? 1 : 2);
    }, cls);
    if (rc) return rc;
    if (hist_slot) HIP_TRY(h, launch_resid_reduce(single(p, 0), hist_slot, blocks_local(p), st));
    rc = run_stage(h, kStRowFft, st, sink, [&] {
      return launch_rowfft(single(p, kRowCopyFft), blocks_rowfft(p), lds_rowfft(p), st, spectral_threads(p));
    }, cls);
    if (rc) return rc;
  }
  if (p.nbp > 0) {
    // block-wise preconditioner: blocks 1.. filter the forward spectra into their own copies,
    // block 0 last, in place
    for (int b = p.nbp - 1; b >= 0 && rc == EPR_OK; --b) {
      ProbDesc q = p;
      for (int i = 0; i < p.lp.n; ++i) q.lp.h[i] = h->blk_h[(size_t)b * p.lp.n + i];
      q.spec_out = b == 0 ? nullptr : p.spec_blk + (size_t)(b - 1) * p.spec_set;
      rc = run_stage(h, kStColFft, st, sink, [&] {
        return launch_colfft(single(q, 0), blocks_colfft(q), lds_colfft(q), st, spectral_threads(q));
      }, cls);
    }
  } else {
    rc = run_stage(h, kStColFft, st, sink,
                   [&] { return launch_colfft(single(p, 0), blocks_colfft(p), lds_colfft(p), st, spectral_threads(p)); }, cls);
  }
  if (rc) return rc;
  return run_stage(h, kStRowInv, st, sink, [&] {
    return launch_rowinv(single(p, kRowInvSolve), blocks_rowinv(p), lds_rowinv(p), st, spectral_threads(p));
  }, cls);
}

#define CHECK(expr)          \
  do {                       \
    int st_ = (expr);        \
    if (st_ != EPR_OK) return st_; \
  } while (0)

bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

int check_ptr(epr_ctx* h, const void* p, const char* name) {
  if (!p) return h->fail(EPR_ERR_INVALID_ARG, "%s is NULL", name);
  if (!aligned4(p)) return h->fail(EPR_ERR_INVALID_ARG, "%s is not 4-byte aligned", name);
  return EPR_OK;
}

// Enqueue a launch sequence on `st` through a cached HIP graph.  `key` holds everything that
// shapes the launches (kernel arguments with their pointers, grids, iteration count); a graph
// with the same key is replayed, otherwise enqueue(stream) is captured on the handle's capture
// stream, instantiated, cached and launched.  The least recently used graph is evicted past
// kSolveGraphCap entries, after the stream of earlier calls has drained.
template <class F>
int run_graph(epr_ctx* h, std::vector<uint8_t>& key, hipStream_t st, F enqueue) {
  for (auto& g : h->solve_graphs) {
    if (g.key == key) {
      g.used = ++h->graph_clock;
      HIP_TRY(h, hipGraphLaunch(g.exec, st));
      return EPR_OK;
    }
  }
  HIP_TRY(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue(h->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
  if (rc != EPR_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess)
    return h->fail(EPR_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return h->fail(EPR_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  }
  if (h->solve_graphs.size() >= kSolveGraphCap) {
    auto lru = std::min_element(h->solve_graphs.begin(), h->solve_graphs.end(),
                                [](const epr_ctx::SolveGraph& a, const epr_ctx::SolveGraph& b) {
                                  return a.used < b.used;
                                });
    HIP_TRY(h, hipStreamSynchronize(h->last_stream));
    HIP_TRY(h, hipStreamSynchronize(st));
    (void)hipGraphExecDestroy(lru->exec);
    (void)hipGraphDestroy(lru->graph);
    h->solve_graphs.erase(lru);
  }
  h->solve_graphs.push_back({key, graph, exec, ++h->graph_clock});
  HIP_TRY(h, hipGraphLaunch(exec, st));
  return EPR_OK;
}

// The iterations of a single-problem solve on `st`: the problem's non-finite flag is cleared
// first (by a kernel: no memset node in a graph), then opts->n_iter iterations; the last one
// writes phase_out.  Replayed from a cached graph unless stage timing is on.
int enqueue_solve(epr_ctx* h, const ProbDesc& p, int model, int n_iter, bool want_resid,
                  float* phase_out, hipStream_t st) {
  auto enqueue = [&](hipStream_t cs) -> int {
    HIP_TRY(h, launch_fill_u32(p.status, 1, cs));
    ProbDesc q = p;
    for (int it = 0; it < n_iter; ++it) {
      q.phase_out = (it == n_iter - 1) ? phase_out : nullptr;
      float* slot = want_resid ? static_cast<float*>(h->hist.ptr) + it : nullptr;
      const int rc = launch_iteration(h, q, model, cs, slot);
      if (rc != EPR_OK) return rc;
    }
    return EPR_OK;
  };
  if (h->timing || n_iter == 0) return enqueue(st);
  std::vector<uint8_t> key;
  const int wr = want_resid ? 1 : 0;
  key_append(key, &model, sizeof model);
  key_append(key, &n_iter, sizeof n_iter);
  key_append(key, &wr, sizeof wr);
  key_append(key, &phase_out, sizeof phase_out);
  key_append(key, &h->hist.ptr, sizeof h->hist.ptr);
  key_append(key, &p, sizeof p);
  return run_graph(h, key, st, enqueue);
}

// Regime histogram of one thickness map: c_s = L delta_s / p^2 = eps_px k_s delta_s.
int regime_impl(epr_ctx* h, const epr_geometry& g, const epr_spectrum& s, const epr_material& m,
                const float* tau, int n_bins, double eta_max, unsigned* counts, hipStream_t st) {
  RegimeParams rp;
  std::memset(&rp, 0, sizeof rp);
  rp.n_lines = s.n_lines;
  rp.n_bins = n_bins;
  rp.scale = (float)n_bins / (float)eta_max;  // the bin decision is taken in float
  const std::vector<LineDouble> ld = lines_double(g, s, m.delta_ref, m.beta_ref);
  for (int i = 0; i < s.n_lines; ++i) rp.c[i] = (float)std::fabs(ld[i].eps_px * ld[i].k * ld[i].delta);
  HIP_TRY(h, launch_regime(tau, g.ny, g.nx, rp, counts, st));
  return EPR_OK;
}

// Automatic model choice: Paganin retrieval (one local first-order iteration from tau = 0 with
// relaxation 1), then the count of pixels with eta_s >= 1 per line.  Synchronous.
int select_impl(epr_ctx* h, const epr_geometry& g, const epr_spectrum& s, const epr_material& m,
                const float* intensity, double max_fraction, int* model, uint32_t* over,
                hipStream_t st) {
  const LineParams lp = line_params(g, s, &m, Kind::Solve);
  const WsLayout w = ws_layout(g.ny, g.nx, lp.n, h->splat_tx, h->splat_ty);
  CHECK(ensure(h, h->ws, w.total));
  const size_t npix = (size_t)g.ny * g.nx;
  const size_t tau_bytes = align256(sizeof(float) * npix);
  CHECK(ensure(h, h->sel, tau_bytes + sizeof(unsigned) * 2 * kMaxLines));
  float* tau = static_cast<float*>(h->sel.ptr);
  unsigned* cnt = reinterpret_cast<unsigned*>(static_cast<char*>(h->sel.ptr) + tau_bytes);
  HIP_TRY(h, launch_fill_u32(reinterpret_cast<unsigned*>(tau), (int)npix, st));
  ProbDesc p;
  CHECK(fill_desc(h, g, lp, static_cast<char*>(h->ws.ptr), &p));
  p.X = tau;
  p.Y = tau;
  p.d = intensity;
  p.tau = tau;
  p.relax = 1.f;
  p.resid = nullptr;
  p.phase_out = nullptr;
  CHECK(launch_iteration(h, p, EPR_LOCAL_L1, st, nullptr));
  CHECK(regime_impl(h, g, s, m, tau, 1, 1.0, cnt, st));
  std::vector<unsigned> hc(2 * (size_t)s.n_lines);
  HIP_TRY(h, hipMemcpyAsync(hc.data(), cnt, sizeof(unsigned) * hc.size(), hipMemcpyDeviceToHost, st));
  HIP_TRY(h, hipStreamSynchronize(st));
  bool local = true;
  for (int i = 0; i < s.n_lines; ++i) {
    const unsigned n_over = hc[2 * i + 1];
    if ((double)n_over > max_fraction * (double)npix) local = false;
    if (over) over[i] = n_over;
  }
  *model = local ? EPR_LOCAL_L2 : EPR_NONLOCAL;
  return EPR_OK;
}

}  // namespace

// ==============================================================================================
// C ABI
// ==============================================================================================
extern "C" {

const char* epr_status_string(int status) {
  switch (status) {
    case EPR_OK: return "success";
    case EPR_ERR_INVALID_ARG: return "invalid argument";
    case EPR_ERR_SHAPE: return "unsupported image shape";
    case EPR_ERR_NO_DEVICE: return "no HIP device";
    case EPR_ERR_HIP: return "HIP runtime error";
    case EPR_ERR_OOM: return "out of device memory";
    case EPR_ERR_UNSUPPORTED: return "unsupported device or model";
    case EPR_ERR_NONFINITE: return "non-finite value in the update";
    default: return "unknown status";
  }
}

const char* epr_last_error(epr_handle h) {
  if (!h) return g_create_error.c_str();
  return h->last_error.c_str();
}

int epr_fft_plan(int32_t n, int32_t* radices, int32_t capacity) {
  if (n < 1 || capacity < 0 || (capacity > 0 && !radices)) return EPR_ERR_INVALID_ARG;
  int tmp[64];
  const int k = factorize(n, tmp, 64);
  if (k < 0) return EPR_ERR_SHAPE;
  for (int i = 0; i < std::min(k, (int)capacity); ++i) radices[i] = tmp[i];
  return k;
}

int epr_check_problem(const epr_geometry* geom, const epr_spectrum* spec,
                      const epr_material* mat, const epr_opts* opts, char* msg, size_t msg_len) {
  epr_ctx tmp;
  int st = check_geometry(&tmp, geom);
  if (!st) st = check_spectrum(&tmp, spec);
  if (!st && mat) st = check_material(&tmp, mat);
  if (!st && opts) st = check_opts(&tmp, opts, true);
  if (!st && opts) st = check_internal(&tmp, geom, opts);
  if (msg && msg_len) {
    std::snprintf(msg, msg_len, "%s", tmp.last_error.c_str());
  }
  return st;
}

int epr_create(epr_handle* out, int device) {
  if (!out) {
    g_create_error = "out is NULL";
    return EPR_ERR_INVALID_ARG;
  }
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    g_create_error = "no HIP device visible";
    return EPR_ERR_NO_DEVICE;
  }
  if (device < 0 || device >= count) {
    g_create_error = "device index out of range";
    return EPR_ERR_NO_DEVICE;
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    g_create_error = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e);
    return EPR_ERR_HIP;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_create_error = std::string("device is ") + prop.gcnArchName + ", library is built for gfx950";
    return EPR_ERR_UNSUPPORTED;
  }
  std::unique_ptr<epr_ctx> h(new epr_ctx);
  h->device = device;
  DeviceGuard guard(device);
  // Opt the kernels into the large dynamic LDS they may need.  A runtime that does not
  // support the attribute leaves the default; a launch needing more then fails and reports.
  (void)set_transport_attributes();
  (void)set_spectral_attributes();
  (void)set_local_attributes();
  (void)set_vjp_attributes();
  (void)set_regime_attributes();
  (void)hipGetLastError();
  if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&h->cap_stream2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming) != hipSuccess) {
    g_create_error = "hipStreamCreate / hipEventCreate failed";
    return EPR_ERR_HIP;
  }
  e = noalloc_scratch_address(device, &h->scratch);
  if (e != hipSuccess) {
    g_create_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return EPR_ERR_HIP;
  }
  if (ensure(h.get(), h->hist, sizeof(float) * 256) != EPR_OK ||
      ensure(h.get(), h->status, sizeof(unsigned) * kStatusWords) != EPR_OK) {
    g_create_error = h->last_error;
    return EPR_ERR_OOM;
  }
  *out = h.release();
  return EPR_OK;
}

int epr_destroy(epr_handle h) {
  if (!h) return EPR_ERR_INVALID_ARG;
  {
    DeviceGuard guard(h->device);
    (void)hipDeviceSynchronize();
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    for (auto& g : h->solve_graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    for (auto& ev : h->pending) {
      (void)hipEventDestroy(ev.a);
      (void)hipEventDestroy(ev.b);
    }
    for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
    for (auto& kv : h->tw) (void)hipFree(kv.second.dev);
    for (DevBuf* b : {&h->ws, &h->hist, &h->batch_ws, &h->batch_table, &h->sel, &h->xtab,
                      &h->status, &h->tune_ws, &h->tune_tau, &h->batch_xtab})
      if (b->ptr) (void)hipFree(b->ptr);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->cap_stream2) (void)hipStreamDestroy(h->cap_stream2);
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    if (h->join_ev) (void)hipEventDestroy(h->join_ev);
  }
  delete h;
  return EPR_OK;
}

int epr_forward(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec, int model,
                const float* phase, const float* absorb, float* intensity, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_model(h, model));
  CHECK(check_ptr(h, phase, "phase"));
  CHECK(check_ptr(h, absorb, "absorb"));
  CHECK(check_ptr(h, intensity, "intensity"));
  if (intensity == phase || intensity == absorb)
    return h->fail(EPR_ERR_INVALID_ARG, "intensity must not alias the inputs");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const LineParams lp = line_params(*geom, *spec, nullptr, Kind::Maps);
  const WsLayout w = ws_layout(geom->ny, geom->nx, lp.n, h->splat_tx, h->splat_ty);
  CHECK(ensure(h, h->ws, w.total));
  ProbDesc p;
  CHECK(fill_desc(h, *geom, lp, static_cast<char*>(h->ws.ptr), &p));
  p.X = absorb;
  p.Y = phase;
  p.out = intensity;
  const int cls = spectral_threads(p) == 1024 ? 1 : 0;
  if (model == EPR_NONLOCAL) {
    CHECK(run_stage(h, kStMaxg, st, &h->pending,
                    [&] { return launch_maxgrad(single(p, 0), blocks_maxg(p), st); }, cls));
    CHECK(run_stage(h, kStSplat, st, &h->pending, [&] {
      return launch_splat(single(p, kSplatForward), blocks_splat(p), lds_splat(p), st, p.lp.n);
    }, cls));
  } else if (model == EPR_NONLOCAL_L2) {
    CHECK(launch_transport_lines(h, p, st, cls));
    CHECK(run_stage(h, kStLocal, st, &h->pending, [&] {
      return launch_local(single(p, kLocalForward), blocks_local(p), lds_local(lp.n), st,
                          kOrderTransportWkb1);
    }, cls));
  } else {
    CHECK(run_stage(h, kStLocal, st, &h->pending, [&] {
      return launch_local(single(p, kLocalForward), blocks_local(p), lds_local(lp.n), st,
                          model == EPR_LOCAL_L1 ? 1 : 2);
    }, cls));
  }
  h->last_stream = st;
  return EPR_OK;
}

int epr_adjoint(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec, int model,
                const float* phase, const float* resid_lines, float* obj_lines, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_model(h, model));
  CHECK(check_ptr(h, phase, "phase"));
  CHECK(check_ptr(h, resid_lines, "resid_lines"));
  CHECK(check_ptr(h, obj_lines, "obj_lines"));
  if (resid_lines == obj_lines) return h->fail(EPR_ERR_INVALID_ARG, "outputs must not alias");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t bytes = sizeof(float) * (size_t)spec->n_lines * geom->ny * geom->nx;
  if (!transport_model(model)) {
    HIP_TRY(h, hipMemcpyAsync(obj_lines, resid_lines, bytes, hipMemcpyDeviceToDevice, st));
    return EPR_OK;
  }
  const LineParams lp = line_params(*geom, *spec, nullptr, Kind::Maps);
  ProbDesc p;
  CHECK(fill_desc(h, *geom, lp, nullptr, &p));
  p.Y = phase;
  p.e = const_cast<float*>(resid_lines);
  p.out = obj_lines;
  const int cls = spectral_threads(p) == 1024 ? 1 : 0;
  CHECK(run_stage(h, kStRowFft, st, &h->pending, [&] {
    return launch_rowfft(single(p, kRowGatherOnly), blocks_rowfft(p), lds_rowfft(p), st, spectral_threads(p));
  }, cls));
  h->last_stream = st;
  return EPR_OK;
}

int epr_precondition(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                     const epr_material* mat, const float* in_lines, float* out_lines,
                     void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_material(h, mat));
  CHECK(check_ptr(h, in_lines, "in_lines"));
  CHECK(check_ptr(h, out_lines, "out_lines"));
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const LineParams lp = line_params(*geom, *spec, mat, Kind::Solve);
  const WsLayout w = ws_layout(geom->ny, geom->nx, lp.n, h->splat_tx, h->splat_ty);
  CHECK(ensure(h, h->ws, w.total));
  ProbDesc p;
  CHECK(fill_desc(h, *geom, lp, static_cast<char*>(h->ws.ptr), &p));
  p.e = const_cast<float*>(in_lines);  // the row pass reads its input from e
  p.out = out_lines;
  const int cls = spectral_threads(p) == 1024 ? 1 : 0;
  CHECK(run_stage(h, kStRowFft, st, &h->pending, [&] {
    return launch_rowfft(single(p, kRowCopyFft), blocks_rowfft(p), lds_rowfft(p), st, spectral_threads(p));
  }, cls));
  CHECK(run_stage(h, kStColFft, st, &h->pending, [&] {
    return launch_colfft(single(p, 0), blocks_colfft(p), lds_colfft(p), st, spectral_threads(p));
  }, cls));
  CHECK(run_stage(h, kStRowInv, st, &h->pending, [&] {
    return launch_rowinv(single(p, kRowInvPrecond), blocks_rowinv(p), lds_rowinv(p), st, spectral_threads(p));
  }, cls));
  h->last_stream = st;
  return EPR_OK;
}

int epr_regime(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
               const epr_material* mat, const float* thickness, int32_t n_bins, double eta_max,
               uint32_t* counts, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_material(h, mat));
  CHECK(check_ptr(h, thickness, "thickness"));
  CHECK(check_ptr(h, counts, "counts"));
  if (n_bins < 1 || n_bins > kMaxBins)
    return h->fail(EPR_ERR_INVALID_ARG, "n_bins = %d outside 1..%d", n_bins, kMaxBins);
  if (!(eta_max > 0.0) || !std::isfinite(eta_max) || !std::isfinite((float)eta_max))
    return h->fail(EPR_ERR_INVALID_ARG, "eta_max must be positive and finite");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  CHECK(regime_impl(h, *geom, *spec, *mat, thickness, n_bins, eta_max, counts, st));
  h->last_stream = st;
  return EPR_OK;
}

int epr_select_model(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                     const epr_material* mat, const float* intensity, double max_fraction,
                     int32_t* model_out, uint32_t* over_counts, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_material(h, mat));
  CHECK(check_ptr(h, intensity, "intensity"));
  if (!model_out) return h->fail(EPR_ERR_INVALID_ARG, "model_out is NULL");
  if (!(max_fraction >= 0.0 && max_fraction <= 1.0))
    return h->fail(EPR_ERR_INVALID_ARG, "max_fraction must lie in [0, 1]");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  int model = 0;
  CHECK(select_impl(h, *geom, *spec, *mat, intensity, max_fraction, &model, over_counts, st));
  *model_out = model;
  h->last_stream = st;
  return EPR_OK;
}

int epr_solve(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
              const epr_material* mat, const epr_opts* opts, const float* intensity,
              float* thickness, float* phase_out, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_material(h, mat));
  CHECK(check_opts(h, opts, true));
  CHECK(check_internal(h, geom, opts));
  CHECK(check_ptr(h, intensity, "intensity"));
  CHECK(check_ptr(h, thickness, "thickness"));
  if (phase_out && !aligned4(phase_out))
    return h->fail(EPR_ERR_INVALID_ARG, "phase_out is not 4-byte aligned");
  if (opts->n_iter > 256 && (opts->flags & EPR_FLAG_RESIDUALS))
    return h->fail(EPR_ERR_INVALID_ARG, "residual history holds at most 256 iterations");
  if ((const void*)intensity == (const void*)thickness)
    return h->fail(EPR_ERR_INVALID_ARG, "thickness must not alias intensity");
  if (opts->n_iter == 0 && phase_out)
    return h->fail(EPR_ERR_INVALID_ARG, "phase_out needs n_iter >= 1");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int f = opts->oversample > 1 ? opts->oversample : 1;
  const epr_geometry gi = internal_geometry(*geom, f);  // the detector grid when f = 1
  const LineParams lp = line_params(gi, *spec, mat, Kind::Solve);
  const WsLayout w = ws_layout(gi.ny, gi.nx, lp.n, h->splat_tx, h->splat_ty);
  CHECK(ensure(h, h->ws, w.total));
  ProbDesc p;
  CHECK(fill_desc(h, gi, lp, static_cast<char*>(h->ws.ptr), &p));
  p.X = thickness;
  p.Y = thickness;
  p.d = intensity;
  p.tau = thickness;
  p.relax = (float)opts->relaxation;
  p.os = f;
  const bool want_resid = (opts->flags & EPR_FLAG_RESIDUALS) != 0;
  if (!want_resid) p.resid = nullptr;
  p.status = static_cast<unsigned*>(h->status.ptr);
  apply_row_lines(h, &p);
  int model = opts->model;
  if (model == EPR_AUTO)
    CHECK(select_impl(h, *geom, *spec, *mat, intensity, EPR_AUTO_MAX_FRACTION, &model, nullptr, st));
  CHECK(enqueue_solve(h, p, model, opts->n_iter, want_resid, phase_out, st));
  h->last_status_n = 1;
  h->last_stream = st;
  h->last_n_iter = opts->n_iter;
  h->last_nprob = 1;
  h->last_resid = want_resid;
  h->last_descs.assign(1, p);
  h->last_nonlocal = transport_model(model);
  h->last_model = model;
  return EPR_OK;
}

int epr_solve_noalloc(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                      const epr_material* mat, const epr_opts* opts, const float* intensity,
                      float* thickness, float* phase_out, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_material(h, mat));
  CHECK(check_opts(h, opts, false));
  CHECK(check_internal(h, geom, opts));
  CHECK(check_ptr(h, intensity, "intensity"));
  CHECK(check_ptr(h, thickness, "thickness"));
  if (phase_out && !aligned4(phase_out))
    return h->fail(EPR_ERR_INVALID_ARG, "phase_out is not 4-byte aligned");
  if (opts->n_iter > 256 && (opts->flags & EPR_FLAG_RESIDUALS))
    return h->fail(EPR_ERR_INVALID_ARG, "residual history holds at most 256 iterations");
  if ((const void*)intensity == (const void*)thickness)
    return h->fail(EPR_ERR_INVALID_ARG, "thickness must not alias intensity");
  if (opts->n_iter == 0 && phase_out)
    return h->fail(EPR_ERR_INVALID_ARG, "phase_out needs n_iter >= 1");
  if (!h->scratch) return h->fail(EPR_ERR_HIP, "the fixed scratch array has no device address");
  const int f = opts->oversample > 1 ? opts->oversample : 1;
  const epr_geometry gi = internal_geometry(*geom, f);
  const LineParams lp = line_params(gi, *spec, mat, Kind::Solve);
  // scratch layout: W_nx table, W_ny table, then the workspace of epr_solve
  const size_t row_tab = align256(sizeof(float2) * (size_t)gi.nx);
  const size_t col_tab = align256(sizeof(float2) * (size_t)gi.ny);
  const WsLayout w = ws_layout(gi.ny, gi.nx, lp.n, h->splat_tx, h->splat_ty);
  const size_t need = row_tab + col_tab + w.total;
  if (need > EPR_NOALLOC_SCRATCH_BYTES)
    return h->fail(EPR_ERR_UNSUPPORTED,
                   "%d x %d internal pixels with %d lines need %zu bytes of workspace; the "
                   "fixed scratch of epr_solve_noalloc holds %zu", gi.ny, gi.nx, lp.n, need,
                   (size_t)EPR_NOALLOC_SCRATCH_BYTES);
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(h->scratch);
  float2* rt = reinterpret_cast<float2*>(base);
  float2* ct = reinterpret_cast<float2*>(base + row_tab);
  // nothing in the scratch has to start at zero: every iteration overwrites the residuals,
  // spectra and partials before reading them; only the tables are written up front
  HIP_TRY(h, launch_twiddle_table(rt, gi.nx, st));
  HIP_TRY(h, launch_twiddle_table(ct, gi.ny, st));
  ProbDesc p;
  CHECK(fill_desc(h, gi, lp, base + row_tab + col_tab, &p, rt, ct));
  p.X = thickness;
  p.Y = thickness;
  p.d = intensity;
  p.tau = thickness;
  p.relax = (float)opts->relaxation;
  p.os = f;
  const bool want_resid = (opts->flags & EPR_FLAG_RESIDUALS) != 0;
  if (!want_resid) p.resid = nullptr;
  p.status = static_cast<unsigned*>(h->status.ptr);
  apply_row_lines(h, &p);
  // every launch enqueued directly (no graph, no timing events)
  const bool saved = h->timing;
  h->timing = false;
  int rc = EPR_OK;
  if (launch_fill_u32(p.status, 1, st) != hipSuccess)
    rc = h->fail(EPR_ERR_HIP, "status clear: %s", hipGetErrorString(hipGetLastError()));
  ProbDesc q = p;
  for (int it = 0; it < opts->n_iter && rc == EPR_OK; ++it) {
    q.phase_out = (it == opts->n_iter - 1) ? phase_out : nullptr;
    float* slot = want_resid ? static_cast<float*>(h->hist.ptr) + it : nullptr;
    rc = launch_iteration(h, q, opts->model, st, slot);
  }
  h->timing = saved;
  if (rc != EPR_OK) return rc;
  h->last_status_n = 1;
  h->last_stream = st;
  h->last_n_iter = opts->n_iter;
  h->last_nprob = 1;
  h->last_resid = want_resid;
  h->last_descs.assign(1, p);
  h->last_nonlocal = transport_model(opts->model);
  h->last_model = opts->model;
  return EPR_OK;
}

int epr_solve_xspec(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                    const epr_spectrum_profile* profile, const epr_material* mat,
                    const epr_opts* opts, const float* intensity, float* thickness,
                    float* phase_out, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum_header(h, spec));
  CHECK(check_profile(h, profile, spec->n_lines));
  CHECK(check_material(h, mat));
  CHECK(check_opts(h, opts, false, true));
  CHECK(check_internal(h, geom, opts));
  CHECK(check_ptr(h, intensity, "intensity"));
  CHECK(check_ptr(h, thickness, "thickness"));
  if (phase_out && !aligned4(phase_out))
    return h->fail(EPR_ERR_INVALID_ARG, "phase_out is not 4-byte aligned");
  if (opts->n_iter > 256 && (opts->flags & EPR_FLAG_RESIDUALS))
    return h->fail(EPR_ERR_INVALID_ARG, "residual history holds at most 256 iterations");
  if ((const void*)intensity == (const void*)thickness)
    return h->fail(EPR_ERR_INVALID_ARG, "thickness must not alias intensity");
  if (opts->n_iter == 0 && phase_out)
    return h->fail(EPR_ERR_INVALID_ARG, "phase_out needs n_iter >= 1");
  const bool block = (opts->flags & EPR_FLAG_BLOCK_PRECOND) != 0;
  if (block && profile->n_blocks > EPR_MAX_PRECOND_BLOCKS)
    return h->fail(EPR_ERR_UNSUPPORTED, "the block-wise preconditioner takes at most %d blocks, "
                   "the profile has %d", EPR_MAX_PRECOND_BLOCKS, profile->n_blocks);
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int f = opts->oversample > 1 ? opts->oversample : 1;
  const epr_geometry gi = internal_geometry(*geom, f);  // the detector grid when f = 1
  const XTable t = xspec_table(gi, *spec, *profile, *mat, f);
  const int nbp = block ? profile->n_blocks : 0;
  const float4* xcol = nullptr;
  const float* den = nullptr;
  const float2* xblk = nullptr;
  CHECK(upload_xtable(h, t, st, &xcol, &den, &xblk));
  const WsLayout w = ws_layout(gi.ny, gi.nx, t.lp.n, h->splat_tx, h->splat_ty);
  // the block-wise preconditioner keeps one set of spectra per block: block 0 in the standard
  // workspace (filtered in place), blocks 1.. after it
  const size_t set_bytes = w.spec;
  const size_t extra = nbp > 1 ? (size_t)(nbp - 1) * set_bytes : 0;
  CHECK(ensure(h, h->ws, w.total + extra));
  ProbDesc p;
  CHECK(fill_desc(h, gi, t.lp, static_cast<char*>(h->ws.ptr), &p));
  if (nbp > 0) {
    p.nbp = nbp;
    p.xblk = xblk;
    p.spec_blk = reinterpret_cast<float2*>(static_cast<char*>(h->ws.ptr) + w.total);
    p.spec_set = set_bytes / sizeof(float2);
    h->blk_h = t.blk_h;
  }
  p.X = thickness;
  p.Y = thickness;
  p.d = intensity;
  p.tau = thickness;
  p.relax = (float)opts->relaxation;
  p.os = f;
  p.xcol = xcol;
  p.xden = den;
  const bool want_resid = (opts->flags & EPR_FLAG_RESIDUALS) != 0;
  if (!want_resid) p.resid = nullptr;
  p.status = static_cast<unsigned*>(h->status.ptr);
  CHECK(enqueue_solve(h, p, opts->model, opts->n_iter, want_resid, phase_out, st));
  h->last_status_n = 1;
  h->last_stream = st;
  h->last_n_iter = opts->n_iter;
  h->last_nprob = 1;
  h->last_resid = want_resid;
  h->last_descs.assign(1, p);
  h->last_nonlocal = transport_model(opts->model);
  h->last_model = opts->model;
  return EPR_OK;
}

// Shared checks and set-up of epr_forward_xspec and epr_adjoint_xspec: the per-column table on
// the device and a problem descriptor whose maps are the thickness (X = Y = tau).
int xspec_maps_setup(epr_ctx* h, const epr_geometry* geom, const epr_spectrum* spec,
                     const epr_spectrum_profile* profile, const epr_material* mat, int model,
                     const float* thickness, hipStream_t st, char* ws_base, ProbDesc* p) {
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum_header(h, spec));
  CHECK(check_profile(h, profile, spec->n_lines));
  CHECK(check_material(h, mat));
  CHECK(check_model(h, model));
  if (model == EPR_AUTO)
    return h->fail(EPR_ERR_UNSUPPORTED, "the x-dependent forward model needs an explicit model");
  CHECK(check_ptr(h, thickness, "thickness"));
  const XTable t = xspec_table(*geom, *spec, *profile, *mat, 1);
  const float4* xcol = nullptr;
  const float* den = nullptr;
  const float2* xblk = nullptr;
  CHECK(upload_xtable(h, t, st, &xcol, &den, &xblk));
  CHECK(fill_desc(h, *geom, t.lp, ws_base, p));
  p->X = thickness;
  p->Y = thickness;
  p->xcol = xcol;
  p->xden = den;
  return EPR_OK;
}

int epr_forward_xspec(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                      const epr_spectrum_profile* profile, const epr_material* mat, int model,
                      const float* thickness, float* intensity, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_ptr(h, intensity, "intensity"));
  if ((const void*)intensity == (const void*)thickness)
    return h->fail(EPR_ERR_INVALID_ARG, "intensity must not alias the thickness");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  CHECK(check_geometry(h, geom));   // (sizes the workspace before the full set-up)
  CHECK(check_spectrum_header(h, spec));
  const WsLayout w = ws_layout(geom->ny, geom->nx, spec->n_lines, h->splat_tx, h->splat_ty);
  CHECK(ensure(h, h->ws, w.total));
  ProbDesc p;
  CHECK(xspec_maps_setup(h, geom, spec, profile, mat, model, thickness, st,
                         static_cast<char*>(h->ws.ptr), &p));
  p.out = intensity;
  const int cls = spectral_threads(p) == 1024 ? 1 : 0;
  const int L = p.lp.n;
  if (model == EPR_NONLOCAL) {
    CHECK(run_stage(h, kStMaxg, st, &h->pending,
                    [&] { return launch_maxgrad(single(p, 0), blocks_maxg(p), st); }, cls));
    CHECK(run_stage(h, kStSplat, st, &h->pending, [&] {
      return launch_splat(single(p, kSplatForward), blocks_splat(p), lds_splat(p), st, L);
    }, cls));
  } else if (model == EPR_NONLOCAL_L2) {
    CHECK(launch_transport_lines(h, p, st, cls));
    CHECK(run_stage(h, kStLocal, st, &h->pending, [&] {
      return launch_local(single(p, kLocalForward), blocks_local(p), lds_local(L), st,
                          kOrderTransportWkb1);
    }, cls));
  } else {
    CHECK(run_stage(h, kStLocal, st, &h->pending, [&] {
      return launch_local(single(p, kLocalForward), blocks_local(p), lds_local(L), st,
                          model == EPR_LOCAL_L1 ? 1 : 2);
    }, cls));
  }
  h->last_stream = st;
  return EPR_OK;
}

int epr_adjoint_xspec(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                      const epr_spectrum_profile* profile, const epr_material* mat, int model,
                      const float* thickness, const float* resid_lines, float* obj_lines,
                      void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_ptr(h, resid_lines, "resid_lines"));
  CHECK(check_ptr(h, obj_lines, "obj_lines"));
  if (resid_lines == obj_lines) return h->fail(EPR_ERR_INVALID_ARG, "outputs must not alias");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  ProbDesc p;
  CHECK(xspec_maps_setup(h, geom, spec, profile, mat, model, thickness, st, nullptr, &p));
  if (!transport_model(model)) {
    const size_t bytes = sizeof(float) * (size_t)spec->n_lines * geom->ny * geom->nx;
    HIP_TRY(h, hipMemcpyAsync(obj_lines, resid_lines, bytes, hipMemcpyDeviceToDevice, st));
    h->last_stream = st;
    return EPR_OK;
  }
  p.e = const_cast<float*>(resid_lines);
  p.out = obj_lines;
  const int cls = spectral_threads(p) == 1024 ? 1 : 0;
  CHECK(run_stage(h, kStRowFft, st, &h->pending, [&] {
    return launch_rowfft(single(p, kRowGatherOnly), blocks_rowfft(p), lds_rowfft(p), st,
                         spectral_threads(p));
  }, cls));
  h->last_stream = st;
  return EPR_OK;
}

int epr_forward_vjp(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec, int model,
                    const float* phase, const float* absorb, const float* grad_intensity,
                    float* grad_phase, float* grad_absorb, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_model(h, model));
  if (model == EPR_AUTO)
    return h->fail(EPR_ERR_UNSUPPORTED, "the vector-Jacobian product needs an explicit model");
  CHECK(check_ptr(h, phase, "phase"));
  CHECK(check_ptr(h, absorb, "absorb"));
  CHECK(check_ptr(h, grad_intensity, "grad_intensity"));
  CHECK(check_ptr(h, grad_phase, "grad_phase"));
  CHECK(check_ptr(h, grad_absorb, "grad_absorb"));
  if (grad_phase == grad_absorb) return h->fail(EPR_ERR_INVALID_ARG, "outputs must not alias");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const LineParams lp = line_params(*geom, *spec, nullptr, Kind::Maps);
  const WsLayout w = ws_layout(geom->ny, geom->nx, lp.n, h->splat_tx, h->splat_ty);
  // G_x, G_y, and for the second-order models two sets of per-line planes
  const size_t plane = (size_t)geom->ny * geom->nx;
  const size_t need = std::max(w.total, align256(sizeof(float) * (2 + 2 * (size_t)lp.n) * plane));
  CHECK(ensure(h, h->ws, need));
  ProbDesc p;
  CHECK(fill_desc(h, *geom, lp, nullptr, &p));
  p.X = absorb;
  p.Y = phase;
  p.d = grad_intensity;
  float* gx = static_cast<float*>(h->ws.ptr);
  float* gy = gx + plane;
  float* work = gy + plane;
  float* qpl = work + lp.n * plane;
  const int nb = (geom->ny * geom->nx + 255) / 256;
  CHECK(run_stage(h, kStVjp, st, &h->pending, [&] {
    hipError_t e = hipSuccess;
    if (model == EPR_NONLOCAL || model == EPR_NONLOCAL_L2)
      e = launch_vjp(single(p, 0), nb, 0, st, gx, gy, grad_absorb);
    if (e == hipSuccess && model != EPR_NONLOCAL) {
      const int order = model == EPR_LOCAL_L1 ? 1 : model == EPR_LOCAL_L2 ? 2 : 3;
      e = launch_vjp_local(single(p, 0), nb, st, order, work, qpl, gx, gy, grad_absorb);
    }
    if (e != hipSuccess) return e;
    return launch_vjp_transpose(single(p, 0), nb, st, gx, gy, grad_phase);
  }));
  h->last_stream = st;
  return EPR_OK;
}

int epr_get_diagnostics(epr_handle h, epr_diagnostics* out) {
  if (!h || !out) return EPR_ERR_INVALID_ARG;
  DeviceGuard guard(h->device);
  std::memset(out, 0, sizeof *out);
  HIP_TRY(h, hipStreamSynchronize(h->last_stream));
  out->n_iter = h->last_n_iter;
  out->n_problems = h->last_nprob;
  out->model = h->last_model;
  if (h->last_resid && h->last_n_iter > 0) {
    HIP_TRY(h, hipMemcpy(out->residual, h->hist.ptr, sizeof(float) * std::min(h->last_n_iter, 256),
                         hipMemcpyDeviceToHost));
  }
  float ms = 0.f;
  for (const ProbDesc& p : h->last_descs) {
    if (!p.maxg || !h->last_nonlocal) continue;
    std::vector<float> g(3 * kMaxgBlocks);
    HIP_TRY(h, hipMemcpy(g.data(), p.maxg, sizeof(float) * g.size(), hipMemcpyDeviceToHost));
    float gx = 0.f, gy = 0.f;
    for (int i = 0; i < kMaxgBlocks; ++i) {
      gx = std::max(gx, g[3 * i]);
      gy = std::max(gy, g[3 * i + 1]);
    }
    ms = std::max(ms, p.lp.b_absmax * std::sqrt(gx * gx + gy * gy));
  }
  out->max_shift_px = ms;
  out->nonfinite = 0;
  out->first_nonfinite = -1;
  if (h->last_status_n > 0) {
    std::vector<unsigned> flags(h->last_status_n);
    HIP_TRY(h, hipMemcpy(flags.data(), h->status.ptr, sizeof(unsigned) * flags.size(),
                         hipMemcpyDeviceToHost));
    for (int i = 0; i < h->last_status_n; ++i) {
      if (!flags[i]) continue;
      if (out->first_nonfinite < 0) out->first_nonfinite = i;
      ++out->nonfinite;
    }
  }
  if (out->nonfinite)
    return h->fail(EPR_ERR_NONFINITE, "%d problem(s) met a NaN or an infinity in the update "
                   "(first: problem %d)", out->nonfinite, out->first_nonfinite);
  return EPR_OK;
}

// ----------------------------------------------------------------------------------------------
// Batched solve
// ----------------------------------------------------------------------------------------------
}  // extern "C"

namespace {

// The launches of one batched iteration for a model and an oversampling factor, in order.
std::vector<int> batch_stages(int model, int f) {
  std::vector<int> v;
  const bool transport = model == EPR_NONLOCAL || model == EPR_NONLOCAL_L2;
  if (transport) {
    v.push_back(kBsMaxg);
    v.push_back(model == EPR_NONLOCAL && f == 1 ? kBsSplatSplit : kBsSplatLines);
    if (model == EPR_NONLOCAL_L2) v.push_back(f == 1 ? kBsWkb1Split : kBsWkb1Lines);
  } else {
    v.push_back(f == 1 ? kBsLocalSplit : kBsLocalLines);
  }
  if (f > 1) v.push_back(kBsBinSplit);
  v.push_back(transport ? kBsRowGather : kBsRowCopy);
  v.push_back(kBsColFft);
  v.push_back(kBsRowInv);
  return v;
}

int stage_blocks(int stage, const ProbDesc& p) {
  switch (stage) {
    case kBsMaxg: return blocks_maxg(p);
    case kBsSplatSplit:
    case kBsSplatLines: return blocks_splat(p);
    case kBsLocalSplit:
    case kBsLocalLines:
    case kBsWkb1Split:
    case kBsWkb1Lines: return blocks_local(p);
    case kBsBinSplit: return blocks_binsplit(p);
    case kBsRowGather:
    case kBsRowCopy: return blocks_rowfft(p);
    case kBsColFft: return blocks_colfft(p);
    default: return blocks_rowinv(p);
  }
}



// Launch sequence of a prepared batch: opts.n_iter iterations, one launch per stage covering
// every problem of a size-class group.  The groups share no data, so each group's whole
// sequence is enqueued on its own stream: `cs` for group 0 and `cs2` (when given) for group 1,
// forked from and joined back into `cs` with events.  Captured into a graph, the two chains are
// parallel branches whose launches can overlap each other's ramp-up and tail.  sink != nullptr
// and timing on: one stream, events around each stage.
int enqueue_batched(epr_ctx* h, hipStream_t cs, std::vector<epr_ctx::EvPair>* sink,
                    hipStream_t cs2 = nullptr) {
  const BatchPlan& bp = h->batch;
  std::vector<epr_ctx::EvPair> dummy;
  auto* sk = sink ? sink : &dummy;
  const bool saved = h->timing;
  if (!sink) h->timing = false;
  int rc = EPR_OK;
  if (launch_fill_u32(bp.status, bp.n, cs) != hipSuccess)
    rc = h->fail(EPR_ERR_HIP, "status clear: %s", hipGetErrorString(hipGetLastError()));
  const bool fork = cs2 != nullptr && bp.ngroups == 2 && rc == EPR_OK;
  if (fork) {
    if (hipEventRecord(h->fork_ev, cs) != hipSuccess ||
        hipStreamWaitEvent(cs2, h->fork_ev, 0) != hipSuccess)
      rc = h->fail(EPR_ERR_HIP, "batched fork: %s", hipGetErrorString(hipGetLastError()));
  }
  for (int g = 0; g < bp.ngroups && rc == EPR_OK; ++g) {
    const BatchGroup& G = bp.grp[g];
    hipStream_t gs = (fork && g == 1) ? cs2 : cs;
    const int cls = G.nt == 1024 ? 1 : 0;
    for (int it = 0; it < bp.n_iter && rc == EPR_OK; ++it) {
      for (int st_i = 0; st_i < bp.ns && rc == EPR_OK; ++st_i) {
        KArgs a;
        std::memset(&a, 0, sizeof a);
        a.table = G.table;
        a.starts = G.starts + (size_t)st_i * (G.n + 1);
        a.nprob = G.n;
        a.xdep = bp.xdep ? 1 : 0;
        a.lpb = G.lpb;
        const int grid = G.total[st_i];
        switch (bp.stages[st_i]) {
          case kBsMaxg:
            rc = run_stage(h, kStMaxg, gs, sk, [&] { return launch_maxgrad(a, grid, gs); }, cls);
            break;
          case kBsSplatSplit:
          case kBsSplatLines:
            a.mode = bp.stages[st_i] == kBsSplatSplit ? kSplatSplit : kSplatLines;
            rc = run_stage(h, kStSplat, gs, sk,
                           [&] { return launch_splat(a, grid, G.lds_sp, gs, bp.L); }, cls);
            break;
          case kBsLocalSplit:
          case kBsLocalLines:
          case kBsWkb1Split:
          case kBsWkb1Lines: {
            const int k = bp.stages[st_i];
            a.mode = (k == kBsLocalSplit || k == kBsWkb1Split) ? kLocalSplit : kLocalLines;
            const int order = (k == kBsWkb1Split || k == kBsWkb1Lines) ? kOrderTransportWkb1
                                                                        : bp.order;
            rc = run_stage(h, kStLocal, gs, sk, [&] {
              return launch_local(a, grid, lds_local(bp.L), gs, order);
            }, cls);
            break;
          }
          case kBsBinSplit:
            rc = run_stage(h, kStBinSplit, gs, sk,
                           [&] { return launch_binsplit(a, grid, gs, bp.L, bp.os); }, cls);
            break;
          case kBsRowGather:
          case kBsRowCopy:
            a.mode = bp.stages[st_i] == kBsRowGather ? kRowGatherFft : kRowCopyFft;
            rc = run_stage(h, kStRowFft, gs, sk,
                           [&] { return launch_rowfft(a, grid, G.lds_rf, gs, G.nt); }, cls);
            break;
          case kBsColFft:
            rc = run_stage(h, kStColFft, gs, sk,
                           [&] { return launch_colfft(a, grid, G.lds_cf, gs, G.nt); }, cls);
            break;
          default:
            a.mode = kRowInvSolve;
            rc = run_stage(h, kStRowInv, gs, sk,
                           [&] { return launch_rowinv(a, grid, G.lds_ri, gs, G.nt); }, cls);
        }
        const int k = bp.stages[st_i];
        if (rc == EPR_OK && bp.want_resid && g == bp.resid_group && it < 256 &&
            (k == kBsSplatSplit || k == kBsLocalSplit || k == kBsWkb1Split || k == kBsBinSplit)) {
          // the stage that formed the residual: reduce problem 0's partials into its slot
          const hipError_t e = launch_resid_reduce(single(bp.resid_desc, 0),
                                                   static_cast<float*>(h->hist.ptr) + it,
                                                   stage_blocks(k, bp.resid_desc), gs);
          if (e != hipSuccess)
            rc = h->fail(EPR_ERR_HIP, "residual reduction: %s", hipGetErrorString(e));
        }
      }
    }
  }
  if (fork) {
    // join even after an error, so that the capture ends with every stream rejoined
    const hipError_t e1 = hipEventRecord(h->join_ev, cs2);
    const hipError_t e2 = hipStreamWaitEvent(cs, h->join_ev, 0);
    if (rc == EPR_OK && (e1 != hipSuccess || e2 != hipSuccess))
      rc = h->fail(EPR_ERR_HIP, "batched join: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  h->timing = saved;
  return rc;
}

}  // namespace




namespace {

// Batched solve; profiles (may be null): an x-dependent spectrum per problem.
int solve_batched_impl(epr_ctx* h, int32_t n, const epr_problem* problems,
                       const epr_spectrum_profile* profiles, const epr_opts* opts, void* stream) {
  if (n < 1 || !problems) return h->fail(EPR_ERR_INVALID_ARG, "need n >= 1 problems");
  CHECK(check_opts(h, opts, false));
  if (opts->n_iter > 256 && (opts->flags & EPR_FLAG_RESIDUALS))
    return h->fail(EPR_ERR_INVALID_ARG, "residual history holds at most 256 iterations");
  const int L = problems[0].spec.n_lines;
  for (int i = 0; i < n; ++i) {
    const epr_problem& q = problems[i];
    CHECK(check_geometry(h, &q.geom));
    if (profiles) {
      CHECK(check_spectrum_header(h, &q.spec));
      CHECK(check_profile(h, &profiles[i], q.spec.n_lines));
    } else {
      CHECK(check_spectrum(h, &q.spec));
    }
    CHECK(check_material(h, &q.mat));
    CHECK(check_internal(h, &q.geom, opts));
    CHECK(check_ptr(h, q.intensity, "intensity"));
    CHECK(check_ptr(h, q.thickness, "thickness"));
    if (q.spec.n_lines != L)
      return h->fail(EPR_ERR_INVALID_ARG, "problem %d has %d lines, problem 0 has %d", i,
                     q.spec.n_lines, L);
  }
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  CHECK(ensure(h, h->status, sizeof(unsigned) * std::max(n, kStatusWords)));

  // cache key: everything that shapes the launches
  std::vector<uint8_t> key;
  key_append(key, &h->status.ptr, sizeof h->status.ptr);
  key_append(key, opts, sizeof *opts);
  key_append(key, &h->splat_tx, sizeof h->splat_tx);
  key_append(key, &h->splat_ty, sizeof h->splat_ty);
  key_append(key, &h->tune_gen, sizeof h->tune_gen);
  for (int i = 0; i < n; ++i) {
    const epr_problem& q = problems[i];
    key_append(key, &q.geom, sizeof q.geom);
    key_append(key, &q.mat, sizeof q.mat);
    key_append(key, &q.intensity, sizeof q.intensity);
    key_append(key, &q.thickness, sizeof q.thickness);
    if (profiles) {
      const epr_spectrum_profile& pr = profiles[i];
      key_append(key, &pr.n_blocks, sizeof pr.n_blocks);
      key_append(key, pr.block_x, sizeof(double) * pr.n_blocks);
      key_append(key, pr.energy_kev, sizeof(double) * pr.n_blocks * L);
      key_append(key, pr.weight, sizeof(double) * pr.n_blocks * L);
    } else {
      key_append(key, q.spec.energy_kev, sizeof(double) * L);
      key_append(key, q.spec.weight, sizeof(double) * L);
    }
    key_append(key, &q.spec.energy_ref_kev, 3 * sizeof(double));
  }
  const int xflag = profiles ? 1 : 0;
  key_append(key, &xflag, sizeof xflag);

  BatchPlan& bp = h->batch;
  if (key != h->graph_key) {
    // an earlier replay may still read the device problem table and the workspace that are
    // about to be replaced
    if (h->batch_stream != st) HIP_TRY(h, hipStreamSynchronize(h->batch_stream));
    HIP_TRY(h, hipStreamSynchronize(st));
    if (h->graph_exec) {
      (void)hipGraphExecDestroy(h->graph_exec);
      h->graph_exec = nullptr;
    }
    if (h->graph) {
      (void)hipGraphDestroy(h->graph);
      h->graph = nullptr;
    }
    h->graph_key.clear();
    const int f = opts->oversample > 1 ? opts->oversample : 1;
    std::vector<size_t> off(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      const epr_geometry gi = internal_geometry(problems[i].geom, f);
      const WsLayout w = ws_layout(gi.ny, gi.nx, L, h->splat_tx, h->splat_ty);
      off[i + 1] = off[i] + w.total;
    }
    CHECK(ensure(h, h->batch_ws, off[n]));
    std::vector<ProbDesc> descs(n);
    // x-dependent spectra: every problem's per-column tables, {col, den} after each other
    std::vector<XTable> xt(profiles ? n : 0);
    std::vector<size_t> xoff(n + 1, 0);
    for (int i = 0; profiles && i < n; ++i) {
      const epr_geometry gi = internal_geometry(problems[i].geom, f);
      xt[i] = xspec_table(gi, problems[i].spec, profiles[i], problems[i].mat, f);
      xoff[i + 1] = xoff[i] + align256(sizeof(float4) * xt[i].col.size()) +
                    align256(sizeof(float) * xt[i].den.size());
    }
    if (profiles) CHECK(ensure(h, h->batch_xtab, xoff[n]));
    for (int i = 0; i < n; ++i) {
      const epr_problem& q = problems[i];
      const epr_geometry gi = internal_geometry(q.geom, f);
      const LineParams lp = profiles ? xt[i].lp : line_params(gi, q.spec, &q.mat, Kind::Solve);
      CHECK(fill_desc(h, gi, lp, static_cast<char*>(h->batch_ws.ptr) + off[i], &descs[i]));
      if (profiles) {
        char* xb = static_cast<char*>(h->batch_xtab.ptr) + xoff[i];
        const size_t cb = align256(sizeof(float4) * xt[i].col.size());
        HIP_TRY(h, hipMemcpy(xb, xt[i].col.data(), sizeof(float4) * xt[i].col.size(),
                             hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(xb + cb, xt[i].den.data(), sizeof(float) * xt[i].den.size(),
                             hipMemcpyHostToDevice));
        descs[i].xcol = reinterpret_cast<const float4*>(xb);
        descs[i].xden = reinterpret_cast<const float*>(xb + cb);
      }
      descs[i].os = f;
      descs[i].X = q.thickness;
      descs[i].Y = q.thickness;
      descs[i].d = q.intensity;
      descs[i].tau = q.thickness;
      descs[i].relax = (float)opts->relaxation;
      descs[i].status = static_cast<unsigned*>(h->status.ptr) + i;
      apply_row_lines(h, &descs[i]);
      // only the caller's problem 0 keeps its residual partials (the history records it)
      if (i != 0 || !(opts->flags & EPR_FLAG_RESIDUALS)) descs[i].resid = nullptr;
    }
    bp.want_resid = (opts->flags & EPR_FLAG_RESIDUALS) != 0;
    bp.xdep = profiles != nullptr;
    bp.resid_desc = descs[0];
    bp.status = static_cast<unsigned*>(h->status.ptr);
    bp.n = n;
    bp.nonlocal = transport_model(opts->model);
    bp.order = opts->model == EPR_LOCAL_L1 ? 1 : 2;
    bp.os = f;
    bp.stages = batch_stages(opts->model, f);
    bp.L = L;
    bp.n_iter = opts->n_iter;
    // group by spectral size class (512-thread problems first)
    std::stable_sort(descs.begin(), descs.end(), [](const ProbDesc& a, const ProbDesc& b) {
      return spectral_threads(a) < spectral_threads(b);
    });
    bp.ns = (int)bp.stages.size();
    std::vector<std::pair<int, int>> ranges;  // [first, count) per group
    for (int i = 0; i < n;) {
      int j = i;
      while (j < n && spectral_threads(descs[j]) == spectral_threads(descs[i])) ++j;
      ranges.push_back({i, j - i});
      i = j;
    }
    bp.ngroups = (int)ranges.size();
    bp.resid_group = (bp.ngroups == 2 && spectral_threads(bp.resid_desc) == 1024) ? 1 : 0;
    std::vector<int> starts;
    std::vector<size_t> start_off(bp.ngroups);
    for (int g = 0; g < bp.ngroups; ++g) {
      BatchGroup& G = bp.grp[g];
      const int first = ranges[g].first, cnt = ranges[g].second;
      G.n = cnt;
      G.nt = spectral_threads(descs[first]);
      G.lpb = row_lines(descs[first]);
      start_off[g] = starts.size();
      for (int st_i = 0; st_i < bp.ns; ++st_i) {
        int acc = 0;
        for (int i = 0; i < cnt; ++i) {
          starts.push_back(acc);
          acc += stage_blocks(bp.stages[st_i], descs[first + i]);
        }
        starts.push_back(acc);
        G.total[st_i] = acc;
      }
      G.lds_sp = G.lds_rf = G.lds_cf = G.lds_ri = 0;
      for (int i = 0; i < cnt; ++i) {
        const ProbDesc& p = descs[first + i];
        G.lds_sp = std::max(G.lds_sp, lds_splat(p));
        G.lds_rf = std::max(G.lds_rf, lds_rowfft(p));
        G.lds_cf = std::max(G.lds_cf, lds_colfft(p));
        G.lds_ri = std::max(G.lds_ri, lds_rowinv(p));
      }
    }
    const size_t table_bytes = align256(sizeof(ProbDesc) * n);
    CHECK(ensure(h, h->batch_table, table_bytes + sizeof(int) * starts.size()));
    ProbDesc* dtable = static_cast<ProbDesc*>(h->batch_table.ptr);
    int* dstarts = reinterpret_cast<int*>(static_cast<char*>(h->batch_table.ptr) + table_bytes);
    HIP_TRY(h, hipMemcpy(dtable, descs.data(), sizeof(ProbDesc) * n, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(dstarts, starts.data(), sizeof(int) * starts.size(),
                         hipMemcpyHostToDevice));
    for (int g = 0; g < bp.ngroups; ++g) {
      bp.grp[g].table = dtable + ranges[g].first;
      bp.grp[g].starts = dstarts + start_off[g];
    }
    h->graph_key = key;
    bp.descs = descs;
  }

  if (h->timing) {
    // HIP events captured into a graph cannot be timed: enqueue the identical launch
    // sequence directly on the caller's stream with events around each stage.
    CHECK(enqueue_batched(h, st, &h->pending));
  } else {
    if (!h->graph_exec) {
      HIP_TRY(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
      const int rc = enqueue_batched(h, h->cap_stream, nullptr, h->cap_stream2);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(h->cap_stream, &g);
      if (rc != EPR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (ec != hipSuccess)
        return h->fail(EPR_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
      h->graph = g;
      HIP_TRY(h, hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0));
    }
    HIP_TRY(h, hipGraphLaunch(h->graph_exec, st));
  }
  h->batch_stream = st;
  h->last_stream = st;
  h->last_n_iter = opts->n_iter;
  h->last_nprob = n;
  h->last_resid = bp.want_resid;
  h->last_status_n = n;
  h->last_descs = bp.descs;
  h->last_nonlocal = bp.nonlocal;
  h->last_model = opts->model;
  return EPR_OK;
}

}  // namespace

extern "C" {

int epr_solve_batched(epr_handle h, int32_t n, const epr_problem* problems, const epr_opts* opts,
                      void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  return solve_batched_impl(h, n, problems, nullptr, opts, stream);
}

int epr_solve_batched_xspec(epr_handle h, int32_t n, const epr_problem* problems,
                            const epr_spectrum_profile* profiles, const epr_opts* opts,
                            void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  if (!profiles) return h->fail(EPR_ERR_INVALID_ARG, "profiles is NULL");
  return solve_batched_impl(h, n, problems, profiles, opts, stream);
}


int epr_set_timing(epr_handle h, int enabled) {
  if (!h) return EPR_ERR_INVALID_ARG;
  DeviceGuard guard(h->device);
  if (!h->pending.empty()) {
    HIP_TRY(h, hipStreamSynchronize(h->last_stream));
    for (auto& ev : h->pending) {
      h->pool.push_back(ev.a);
      h->pool.push_back(ev.b);
    }
    h->pending.clear();
  }
  h->timing = enabled != 0;
  for (int i = 0; i < EPR_N_STAGES; ++i) {
    h->tms[i] = 0.0;
    h->tcount[i] = 0;
    for (int c = 0; c < 2; ++c) {
      h->tms_cls[i][c] = 0.0;
      h->tcount_cls[i][c] = 0;
    }
  }
  return EPR_OK;
}

int epr_get_timing(epr_handle h, epr_timing* out) {
  if (!h || !out) return EPR_ERR_INVALID_ARG;
  DeviceGuard guard(h->device);
  HIP_TRY(h, hipStreamSynchronize(h->last_stream));
  CHECK(fold_events(h, h->pending, true));
  for (int i = 0; i < EPR_N_STAGES; ++i) {
    out->ms[i] = h->tms[i];
    out->launches[i] = h->tcount[i];
    for (int c = 0; c < 2; ++c) {
      out->ms_class[i][c] = h->tms_cls[i][c];
      out->launches_class[i][c] = h->tcount_cls[i][c];
    }
  }
  return EPR_OK;
}

// ----------------------------------------------------------------------------------------------
// Autotuner: splat tile shape (on a warm state) and the radix order of every compiled transform
// length, timed on the caller's problems.
// ----------------------------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr int kTuneWarmIters = 2;
constexpr int kTuneReps = 3;
// a candidate replaces the value in use only when it is at least this much faster: differences
// below it are within the run-to-run spread of a timing and would pick noise
constexpr float kTuneMargin = 0.01f;
const int kSplatCand[][2] = {{64, 32}, {32, 32}, {64, 16}, {32, 64}, {128, 16}, {64, 64},
                             {128, 32}, {32, 16}};
constexpr size_t kLdsLimit = 160 * 1024 - 64;

// Is a splat tile usable for problems of L lines (LDS of the bordered per-line accumulators)?
bool splat_tile_ok(int tx, int ty, int L) {
  if (tx < 8 || ty < 8 || tx > 256 || ty > 256 || tx * ty > 4096) return false;
  return sizeof(float) * (size_t)L * (tx + 2) * (ty + 2) <= kLdsLimit;
}

// The tuning cache: one flat JSON object of integers, {"splat_tx": 64, "splat_ty": 32,
// "row_1024": 0, "col_2048": 1, ...} (row_<n>: radix order of the length-n row transform,
// col_<n>: of the length-n column transform).  Returns false if the file is absent or
// malformed.
bool read_tune_cache(const char* path, std::map<std::string, int>* kv) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  std::string txt;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, got);
  std::fclose(f);
  size_t i = txt.find('{');
  if (i == std::string::npos) return false;
  ++i;
  for (;;) {
    while (i < txt.size() && std::isspace((unsigned char)txt[i])) ++i;
    if (i < txt.size() && txt[i] == '}') return !kv->empty();
    if (i >= txt.size() || txt[i] != '"') return false;
    const size_t q = txt.find('"', i + 1);
    if (q == std::string::npos) return false;
    const std::string key = txt.substr(i + 1, q - i - 1);
    i = txt.find(':', q);
    if (i == std::string::npos) return false;
    char* endp = nullptr;
    const double v = std::strtod(txt.c_str() + i + 1, &endp);
    if (endp == txt.c_str() + i + 1) return false;
    (*kv)[key] = (int)v;
    i = (size_t)(endp - txt.c_str());
    while (i < txt.size() && std::isspace((unsigned char)txt[i])) ++i;
    if (i < txt.size() && txt[i] == ',') ++i;
  }
}

struct TuneProblem {
  ProbDesc p;
  int model;
};

// Summed duration (ms) of `reps` runs of fn() on stream st, after one untimed run.
template <class F>
int time_ms(epr_ctx* h, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps, F fn, float* out) {
  int rc = fn();
  if (rc) return rc;
  HIP_TRY(h, hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) {
    rc = fn();
    if (rc) return rc;
  }
  HIP_TRY(h, hipEventRecord(e1, st));
  HIP_TRY(h, hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(h, hipEventElapsedTime(&ms, e0, e1));
  *out = ms;
  return EPR_OK;
}

}  // namespace

extern "C" {

int epr_autotune(epr_handle h, int32_t n, const epr_problem* problems, const epr_opts* opts,
                 const char* cache_json) {
  if (!h) return EPR_ERR_INVALID_ARG;
  if (n < 1 || !problems) return h->fail(EPR_ERR_INVALID_ARG, "need n >= 1 problems");
  CHECK(check_opts(h, opts, false));
  int Lmax = 0;
  for (int i = 0; i < n; ++i) {
    const epr_problem& q = problems[i];
    CHECK(check_geometry(h, &q.geom));
    CHECK(check_spectrum(h, &q.spec));
    CHECK(check_material(h, &q.mat));
    CHECK(check_internal(h, &q.geom, opts));
    CHECK(check_ptr(h, q.intensity, "intensity"));
    CHECK(check_ptr(h, q.thickness, "thickness"));
    Lmax = std::max(Lmax, (int)q.spec.n_lines);
  }
  const int f = opts->oversample > 1 ? opts->oversample : 1;
  // the transform lengths of these problems (internal grid)
  std::vector<int> rows, cols;
  for (int i = 0; i < n; ++i) {
    const epr_geometry gi = internal_geometry(problems[i].geom, f);
    if (std::find(rows.begin(), rows.end(), gi.nx / 2) == rows.end()) rows.push_back(gi.nx / 2);
    if (std::find(cols.begin(), cols.end(), gi.ny) == cols.end()) cols.push_back(gi.ny);
  }
  const bool transport = transport_model(opts->model);

  if (cache_json) {
    std::map<std::string, int> kv;
    if (read_tune_cache(cache_json, &kv)) {
      // a cached choice is used only if every entry is valid for these problems; otherwise
      // the file is ignored, the choices are timed again and the file is rewritten
      bool ok = true;
      int tx = h->splat_tx, ty = h->splat_ty;
      if (kv.count("splat_tx") || kv.count("splat_ty")) {
        tx = kv.count("splat_tx") ? kv["splat_tx"] : -1;
        ty = kv.count("splat_ty") ? kv["splat_ty"] : -1;
        ok = splat_tile_ok(tx, ty, Lmax);
      }
      std::map<int, int> rv = h->fft_row_var, cv = h->fft_col_var;
      int lines = h->row_lines;
      if (kv.count("row_lines")) {
        lines = kv["row_lines"];
        ok = ok && (lines == 1 || lines == 2);
      }
      for (const auto& e : kv) {
        int len = 0;
        if (std::sscanf(e.first.c_str(), "row_%d", &len) == 1) {
          ok = ok && e.second >= 0 && e.second < fft_row_variants(len);
          rv[len] = e.second;
        } else if (std::sscanf(e.first.c_str(), "col_%d", &len) == 1) {
          ok = ok && e.second >= 0 && e.second < fft_col_variants(len);
          cv[len] = e.second;
        }
      }
      if (ok) {
        h->splat_tx = tx;
        h->splat_ty = ty;
        h->fft_row_var = rv;
        h->fft_col_var = cv;
        h->row_lines = lines;
        ++h->tune_gen;
        return EPR_OK;
      }
    }
  }

  DeviceGuard guard(h->device);
  HIP_TRY(h, hipDeviceSynchronize());  // the caller's data is complete
  hipStream_t st = h->cap_stream;
  // workspace for the largest problem with the widest candidate residual partials, and one
  // warm thickness per problem
  size_t ws_bytes = 0, tau_bytes = 0;
  std::vector<size_t> tau_off(n);
  for (int i = 0; i < n; ++i) {
    const epr_geometry gi = internal_geometry(problems[i].geom, f);
    for (const auto& c : kSplatCand)
      ws_bytes = std::max(ws_bytes, ws_layout(gi.ny, gi.nx, problems[i].spec.n_lines, c[0], c[1]).total);
    tau_off[i] = tau_bytes;
    tau_bytes += align256(sizeof(float) * (size_t)gi.ny * gi.nx);
  }
  CHECK(ensure(h, h->tune_ws, ws_bytes));
  CHECK(ensure(h, h->tune_tau, tau_bytes));
  const bool saved_timing = h->timing;
  h->timing = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = EPR_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = h->fail(EPR_ERR_HIP, "hipEventCreate failed");

  // descriptor of problem i on the tuning workspace, thickness = its warm copy
  auto desc = [&](int i, ProbDesc* p) -> int {
    const epr_problem& q = problems[i];
    const epr_geometry gi = internal_geometry(q.geom, f);
    const LineParams lp = line_params(gi, q.spec, &q.mat, Kind::Solve);
    int r = fill_desc(h, gi, lp, static_cast<char*>(h->tune_ws.ptr), p);
    if (r) return r;
    float* tau = reinterpret_cast<float*>(static_cast<char*>(h->tune_tau.ptr) + tau_off[i]);
    p->X = p->Y = p->tau = tau;
    p->d = q.intensity;
    p->relax = (float)opts->relaxation;
    p->os = f;
    p->resid = nullptr;
    p->status = nullptr;
    apply_row_lines(h, p);
    return EPR_OK;
  };

  // warm state: kTuneWarmIters iterations from each problem's own start, on the copies
  for (int i = 0; i < n && rc == EPR_OK; ++i) {
    const epr_geometry gi = internal_geometry(problems[i].geom, f);
    ProbDesc p;
    rc = desc(i, &p);
    if (rc) break;
    if (hipMemcpyAsync(p.tau, problems[i].thickness, sizeof(float) * (size_t)gi.ny * gi.nx,
                       hipMemcpyDeviceToDevice, st) != hipSuccess) {
      rc = h->fail(EPR_ERR_HIP, "warm copy: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    for (int it = 0; it < kTuneWarmIters && rc == EPR_OK; ++it)
      rc = launch_iteration(h, p, opts->model, st, nullptr);
  }

  // Every choice is timed on what the solvers run: one iteration of the batched solve of all
  // the given problems (a batch of one for a single problem), replayed from its graph, on the
  // warm copies.  The dimensions are tuned one after the other, each with the others at their
  // best so far: splat tile, lines per row-pass workgroup, then the radix order of each row and
  // column length.
  std::vector<epr_problem> tp(problems, problems + n);
  for (int i = 0; i < n; ++i)
    tp[i].thickness = reinterpret_cast<float*>(static_cast<char*>(h->tune_tau.ptr) + tau_off[i]);
  epr_opts to = *opts;
  to.n_iter = 1;
  to.flags = 0;
  // the tuner's batched runs replace the handle's cached batched graph and the state
  // epr_get_diagnostics reports on; the latter is restored at the end
  const auto saved_diag = std::make_tuple(h->last_stream, h->last_n_iter, h->last_nprob,
                                          h->last_resid, h->last_nonlocal, h->last_model,
                                          h->last_status_n, h->last_descs);
  auto measure = [&](float* out) -> int {
    int r = solve_batched_impl(h, n, tp.data(), nullptr, &to, st);  // capture (untimed)
    if (r) return r;
    return time_ms(h, st, e0, e1, kTuneReps, [&]() -> int {
      return solve_batched_impl(h, n, tp.data(), nullptr, &to, st);
    }, out);
  };
  float best = 1e30f;
  if (rc == EPR_OK) rc = measure(&best);
  // one dimension: try each value with set(v), keep the fastest (the current value first)
  auto tune = [&](const std::vector<int>& values, const std::function<void(int)>& set,
                  int current) {
    int bv = current;
    for (int v : values) {
      if (rc != EPR_OK) return;
      if (v == current) continue;
      set(v);
      ++h->tune_gen;
      float ms = 0.f;
      rc = measure(&ms);
      if (rc == EPR_OK && ms < best * (1.f - kTuneMargin)) {
        best = ms;
        bv = v;
      }
    }
    set(bv);
    ++h->tune_gen;
  };
  if (transport) {
    std::vector<int> tiles;
    for (int c = 0; c < (int)(sizeof kSplatCand / sizeof kSplatCand[0]); ++c)
      if (splat_tile_ok(kSplatCand[c][0], kSplatCand[c][1], Lmax)) tiles.push_back(c);
    int cur = -1;
    for (int c : tiles)
      if (kSplatCand[c][0] == h->splat_tx && kSplatCand[c][1] == h->splat_ty) cur = c;
    tune(tiles, [&](int c) { h->splat_tx = kSplatCand[c][0]; h->splat_ty = kSplatCand[c][1]; },
         cur);
  }
  bool any512 = false;
  for (int i = 0; i < n; ++i) {
    const epr_geometry gi = internal_geometry(problems[i].geom, f);
    any512 = any512 || (gi.nx <= 2048 && gi.ny <= 2048);
  }
  if (any512) tune({1, 2}, [&](int v) { h->row_lines = v; }, h->row_lines);
  for (int len : rows) {
    const int nv = fft_row_variants(len);
    std::vector<int> vs;
    for (int v = 0; v < nv; ++v) vs.push_back(v);
    if (nv > 1) tune(vs, [&](int v) { h->fft_row_var[len] = v; }, h->fft_row_var[len]);
  }
  for (int len : cols) {
    const int nv = fft_col_variants(len);
    std::vector<int> vs;
    for (int v = 0; v < nv; ++v) vs.push_back(v);
    if (nv > 1) tune(vs, [&](int v) { h->fft_col_var[len] = v; }, h->fft_col_var[len]);
  }
  const float best_ms = best;
  std::tie(h->last_stream, h->last_n_iter, h->last_nprob, h->last_resid, h->last_nonlocal,
           h->last_model, h->last_status_n, h->last_descs) = saved_diag;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  h->timing = saved_timing;
  ++h->tune_gen;
  if (rc) return rc;
  if (cache_json) {
    FILE* fo = std::fopen(cache_json, "w");
    if (fo) {
      std::fprintf(fo, "{\"splat_tx\": %d, \"splat_ty\": %d, \"row_lines\": %d", h->splat_tx,
                   h->splat_ty, h->row_lines);
      for (const auto& e : h->fft_row_var) std::fprintf(fo, ", \"row_%d\": %d", e.first, e.second);
      for (const auto& e : h->fft_col_var) std::fprintf(fo, ", \"col_%d\": %d", e.first, e.second);
      std::fprintf(fo, ", \"iteration_ms\": %.6f", best_ms);
      std::fprintf(fo, "}\n");
      std::fclose(fo);
    }
  }
  return EPR_OK;
}

}  // extern "C"
