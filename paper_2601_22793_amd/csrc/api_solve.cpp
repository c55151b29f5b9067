// Entry points of the single-problem solves (Methods 4.4): plain, allocation-free, and with
// an x-dependent spectrum (Methods 4.3 remark).
#include "host.h"

using namespace epr;
using namespace epr::host;

extern "C" {

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
  apply_row_lines(h, &p);
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

}  // extern "C"
