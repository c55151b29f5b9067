// Batched solver: every problem of a batch in one launch per stage and spectral size class,
// the iterations captured into a cached HIP graph with the two size classes as parallel
// branches.
#include "host.h"

using namespace epr;
using namespace epr::host;

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
        a.rl = G.rl;
        a.ny_max = G.ny_max;
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

namespace epr {
namespace host {

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
      G.rl = row_lines(descs[first]);
      G.ny_max = 0;
      for (int i = 0; i < cnt; ++i) G.ny_max = std::max(G.ny_max, descs[first + i].ny);
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

}  // namespace host
}  // namespace epr

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

}  // extern "C"
