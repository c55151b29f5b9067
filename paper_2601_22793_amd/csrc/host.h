// Host side of libepr, shared by its translation units (host_core.cpp, api_ops.cpp,
// api_solve.cpp, api_batch.cpp, api_tune.cpp): the handle (struct epr_ctx) with its device
// buffers, graph caches and tuned launch shapes, and the helpers every entry point uses
// (validation, per-line constants in double rounded once to float, FFT plans, workspace
// layout, the launch sequence of one EPR iteration, stage timing, graph capture).  Internal:
// nothing here is part of the C ABI (the library exports the epr_* functions only, libepr.map).
#pragma once

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

namespace epr {
namespace host {

constexpr double kHcEvM = 1.239841984e-6;  // h c [eV m]
constexpr double kPi = 3.14159265358979323846;
constexpr int kStatusWords = 1024;      // non-finite flags held without growing the buffer
constexpr size_t kSolveGraphCap = 64;   // cached single-problem solve graphs per handle

inline void key_append(std::vector<uint8_t>& k, const void* p, size_t n) {
  const uint8_t* b = static_cast<const uint8_t*>(p);
  k.insert(k.end(), b, b + n);
}

// error message of the last failed epr_create on this thread
extern thread_local std::string g_create_error;

// Radix sequence for n (product of 2, 3, 5): radix 16 first, then the rest of the power of
// two as 8 / 4 / 2, then 5s and 3s.  Returns the number of stages, or -1.
int factorize(int n, int* radix, int cap);
bool smooth235(int n);

struct Twiddles {
  float2* dev = nullptr;
  int n = 0;
};

// Device buffers
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Prepared batched launch sequence: the device problem table, sorted into groups of one
// spectral size class each (one launch per stage and group), with per-stage block prefix sums.
struct BatchGroup {
  ProbDesc* table = nullptr;   // first problem of the group in the device table
  int* starts = nullptr;       // [ns][n + 1] prefix sums of this group
  int n = 0;
  int nt = 512;                // spectral threads of the group
  int rl = 1;                  // row-pass lines per workgroup of the group
  int ny_max = 0;              // largest ny of the group (column-pass instance)
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

}  // namespace host
}  // namespace epr

// The handle of the C ABI.
struct epr_ctx {
  using DevBuf = epr::host::DevBuf;
  using Twiddles = epr::host::Twiddles;
  using BatchPlan = epr::host::BatchPlan;
  using ProbDesc = epr::ProbDesc;
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
  int splat_tx = epr::kSplatTileX, splat_ty = epr::kSplatTileY;
  std::map<int, int> fft_row_var, fft_col_var;  // tuned radix order per transform length
  int row_lines = 2;                            // tuned lines per row-pass workgroup (1, 2, 4)
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

namespace epr {
namespace host {

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

#define CHECK(expr)          \
  do {                       \
    int st_ = (expr);        \
    if (st_ != EPR_OK) return st_; \
  } while (0)

enum Stage { kStMaxg = 0, kStSplat = 1, kStLocal = 2, kStRowFft = 3, kStColFft = 4,
             kStRowInv = 5, kStVjp = 6, kStBinSplit = 7 };

// Launches of a batched iteration.
enum BatchStage { kBsMaxg, kBsSplatSplit, kBsSplatLines, kBsLocalSplit, kBsLocalLines,
                  kBsWkb1Split, kBsWkb1Lines, kBsBinSplit, kBsRowGather, kBsRowCopy, kBsColFft,
                  kBsRowInv };

enum class Kind { Solve, Maps };

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

// Sizes of the per-problem workspace pieces (bytes, 256-aligned).
inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
struct WsLayout {
  size_t e, spec, maxg, resid, total;
};

inline bool transport_model(int model) { return model == EPR_NONLOCAL || model == EPR_NONLOCAL_L2; }

inline bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

// helpers defined in host_core.cpp
int ensure(epr_ctx* h, DevBuf& b, size_t bytes);
hipEvent_t take_event(epr_ctx* h);
int fold_events(epr_ctx* h, std::vector<epr_ctx::EvPair>& v, bool recycle);
const float2* twiddles(epr_ctx* h, int n, int* status);
int make_plan(epr_ctx* h, int n, int table_n, int stride, FftPlan* out,
              const float2* table = nullptr);
int check_geometry(epr_ctx* h, const epr_geometry* g);
int check_spectrum_header(epr_ctx* h, const epr_spectrum* s);
int check_spectrum(epr_ctx* h, const epr_spectrum* s);
int check_profile(epr_ctx* h, const epr_spectrum_profile* pr, int n_lines);
int check_material(epr_ctx* h, const epr_material* m);
int check_model(epr_ctx* h, int model);
int check_opts(epr_ctx* h, const epr_opts* o, bool allow_auto, bool allow_block = false);
epr_geometry internal_geometry(const epr_geometry& g, int f);
int check_internal(epr_ctx* h, const epr_geometry* g, const epr_opts* o);
LineParams line_params(const epr_geometry& g, const epr_spectrum& s, const epr_material* m,
                       Kind kind, double relax_unused = 0.0);
XTable xspec_table(const epr_geometry& g, const epr_spectrum& s, const epr_spectrum_profile& pr,
                   const epr_material& m, int f);
WsLayout ws_layout(int ny, int nx, int L, int tx, int ty);
int upload_xtable(epr_ctx* h, const XTable& t, hipStream_t st, const float4** col,
                  const float** den, const float2** blk);
int fill_desc(epr_ctx* h, const epr_geometry& g, const LineParams& lp, char* base, ProbDesc* p,
              const float2* row_tab = nullptr, const float2* col_tab = nullptr);
void apply_row_lines(const epr_ctx* h, ProbDesc* p);
KArgs single(const ProbDesc& p, int mode);
int launch_transport_lines(epr_ctx* h, const ProbDesc& p, hipStream_t st, int cls);
int launch_lines_binsplit(epr_ctx* h, const ProbDesc& p, int model, hipStream_t st,
                          float* hist_slot, int cls);
int launch_iteration(epr_ctx* h, const ProbDesc& p, int model, hipStream_t st, float* hist_slot);
int check_ptr(epr_ctx* h, const void* p, const char* name);
int enqueue_solve(epr_ctx* h, const ProbDesc& p, int model, int n_iter, bool want_resid,
                  float* phase_out, hipStream_t st);
int regime_impl(epr_ctx* h, const epr_geometry& g, const epr_spectrum& s, const epr_material& m,
                const float* tau, int n_bins, double eta_max, unsigned* counts, hipStream_t st);
int select_impl(epr_ctx* h, const epr_geometry& g, const epr_spectrum& s, const epr_material& m,
                const float* intensity, double max_fraction, int* model, uint32_t* over,
                hipStream_t st);

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

// Batched solve (api_batch.cpp); profiles (may be null): an x-dependent spectrum per problem.
int solve_batched_impl(epr_ctx* h, int32_t n, const epr_problem* problems,
                       const epr_spectrum_profile* profiles, const epr_opts* opts, void* stream);

}  // namespace host
}  // namespace epr
