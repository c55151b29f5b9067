// Autotuner of the launch choices: splat tile, row-pass lines per workgroup and the radix
// order of every compiled transform length, timed on whole batched iterations of the caller's
// problems, with a JSON cache.
#include "host.h"

using namespace epr;
using namespace epr::host;

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
        ok = ok && (lines == 1 || lines == 2 || lines == 4);
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
  if (Lmax > 1) tune({1, 2, 4}, [&](int v) { h->row_lines = v; }, h->row_lines);
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
