// Entry points of the operators: the forward model (Eq. 5 with the closures of Eq. 1 or the
// transport of Eq. 3), the per-line back-transport (Eq. 4), the Paganin-type preconditioner
// (Section 2), the regime diagnostics and model choice (Section 2), their x-dependent
// versions (Methods 4.3 remark) and the vector-Jacobian products of both forward models.
#include "host.h"

using namespace epr;
using namespace epr::host;

namespace {

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

// Workspace bytes of the vector-Jacobian product: G_x, G_y, and for the second-order models
// two sets of per-line planes.
size_t vjp_workspace(const epr_ctx* h, int ny, int nx, int n_lines) {
  const WsLayout w = ws_layout(ny, nx, n_lines, h->splat_tx, h->splat_ty);
  const size_t plane = (size_t)ny * nx;
  return std::max(w.total, align256(sizeof(float) * (2 + 2 * (size_t)n_lines) * plane));
}

// The VJP kernels of `model` for p (X, Y and d = dL/dP set): grad_a = sum_s -a_s I_s dI_s,
// then grad_y = D_x^T G_x + D_y^T G_y, or with `accumulate` (grad_y == grad_a, an x-dependent
// spectrum over one thickness map) that sum added to grad_a.  The workspace is h->ws.
int vjp_stages(epr_ctx* h, const ProbDesc& p, int model, hipStream_t st, float* grad_y,
               float* grad_a, bool accumulate) {
  const size_t plane = (size_t)p.ny * p.nx;
  float* gx = static_cast<float*>(h->ws.ptr);
  float* gy = gx + plane;
  float* work = gy + plane;
  float* qpl = work + p.lp.n * plane;
  const int nb = (int)((plane + 255) / 256);
  return run_stage(h, kStVjp, st, &h->pending, [&] {
    hipError_t e = hipSuccess;
    if (model == EPR_NONLOCAL || model == EPR_NONLOCAL_L2)
      e = launch_vjp(single(p, 0), nb, 0, st, gx, gy, grad_a);
    if (e == hipSuccess && model != EPR_NONLOCAL) {
      const int order = model == EPR_LOCAL_L1 ? 1 : model == EPR_LOCAL_L2 ? 2 : 3;
      e = launch_vjp_local(single(p, 0), nb, st, order, work, qpl, gx, gy, grad_a);
    }
    if (e != hipSuccess) return e;
    return launch_vjp_transpose(single(p, 0), nb, st, gx, gy, grad_y, accumulate ? 1 : 0);
  });
}

}  // namespace

extern "C" {

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

int epr_forward_oversampled(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                            int model, int32_t oversample, const float* phase,
                            const float* absorb, float* intensity, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_model(h, model));
  if (oversample != 1 && oversample != 2 && oversample != 4)
    return h->fail(EPR_ERR_INVALID_ARG, "oversample = %d: 1, 2 or 4", oversample);
  epr_opts o{};
  o.oversample = oversample;
  CHECK(check_internal(h, geom, &o));
  if (oversample == 1) return epr_forward(h, geom, spec, model, phase, absorb, intensity, stream);
  CHECK(check_ptr(h, phase, "phase"));
  CHECK(check_ptr(h, absorb, "absorb"));
  CHECK(check_ptr(h, intensity, "intensity"));
  if (intensity == phase || intensity == absorb)
    return h->fail(EPR_ERR_INVALID_ARG, "intensity must not alias the inputs");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const epr_geometry gi = internal_geometry(*geom, oversample);
  const LineParams lp = line_params(gi, *spec, nullptr, Kind::Maps);
  const WsLayout w = ws_layout(gi.ny, gi.nx, lp.n, h->splat_tx, h->splat_ty);
  CHECK(ensure(h, h->ws, w.total));
  ProbDesc p;
  CHECK(fill_desc(h, gi, lp, static_cast<char*>(h->ws.ptr), &p));
  p.X = absorb;
  p.Y = phase;
  p.os = oversample;
  p.d = nullptr;         // the bin-split pass writes the binned prediction to out
  p.out = intensity;
  p.resid = nullptr;
  const int cls = spectral_threads(p) == 1024 ? 1 : 0;
  CHECK(launch_lines_binsplit(h, p, model, st, nullptr, cls));
  h->last_stream = st;
  return EPR_OK;
}

int epr_adjoint_oversampled(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                            int model, int32_t oversample, const float* phase,
                            const float* resid_lines, float* obj_lines, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_model(h, model));
  if (oversample != 1 && oversample != 2 && oversample != 4)
    return h->fail(EPR_ERR_INVALID_ARG, "oversample = %d: 1, 2 or 4", oversample);
  epr_opts o{};
  o.oversample = oversample;
  CHECK(check_internal(h, geom, &o));
  if (oversample == 1)
    return epr_adjoint(h, geom, spec, model, phase, resid_lines, obj_lines, stream);
  CHECK(check_ptr(h, phase, "phase"));
  CHECK(check_ptr(h, resid_lines, "resid_lines"));
  CHECK(check_ptr(h, obj_lines, "obj_lines"));
  if (resid_lines == obj_lines) return h->fail(EPR_ERR_INVALID_ARG, "outputs must not alias");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const epr_geometry gi = internal_geometry(*geom, oversample);
  if (!transport_model(model)) {
    HIP_TRY(h, launch_unbin_lines(resid_lines, obj_lines, gi.ny, gi.nx, oversample,
                                  spec->n_lines, st));
    h->last_stream = st;
    return EPR_OK;
  }
  const LineParams lp = line_params(gi, *spec, nullptr, Kind::Maps);
  const WsLayout w = ws_layout(gi.ny, gi.nx, lp.n, h->splat_tx, h->splat_ty);
  CHECK(ensure(h, h->ws, w.total));
  ProbDesc p;
  CHECK(fill_desc(h, gi, lp, static_cast<char*>(h->ws.ptr), &p));
  p.Y = phase;
  p.out = obj_lines;
  HIP_TRY(h, launch_unbin_lines(resid_lines, p.e, gi.ny, gi.nx, oversample, lp.n, st));
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
  CHECK(check_ptr(h, phase, "phase"));
  CHECK(check_ptr(h, absorb, "absorb"));
  CHECK(check_ptr(h, grad_intensity, "grad_intensity"));
  CHECK(check_ptr(h, grad_phase, "grad_phase"));
  CHECK(check_ptr(h, grad_absorb, "grad_absorb"));
  if (grad_phase == grad_absorb) return h->fail(EPR_ERR_INVALID_ARG, "outputs must not alias");
  for (const float* in : {phase, absorb, grad_intensity})
    if (in == grad_phase || in == grad_absorb)
      return h->fail(EPR_ERR_INVALID_ARG, "the gradients must not alias the inputs");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const LineParams lp = line_params(*geom, *spec, nullptr, Kind::Maps);
  CHECK(ensure(h, h->ws, vjp_workspace(h, geom->ny, geom->nx, lp.n)));
  ProbDesc p;
  CHECK(fill_desc(h, *geom, lp, nullptr, &p));
  p.X = absorb;
  p.Y = phase;
  p.d = grad_intensity;
  CHECK(vjp_stages(h, p, model, st, grad_phase, grad_absorb, false));
  h->last_stream = st;
  return EPR_OK;
}

int epr_forward_vjp_oversampled(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                                int model, int32_t oversample, const float* phase,
                                const float* absorb, const float* grad_intensity,
                                float* grad_phase, float* grad_absorb, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_geometry(h, geom));
  CHECK(check_spectrum(h, spec));
  CHECK(check_model(h, model));
  if (oversample != 1 && oversample != 2 && oversample != 4)
    return h->fail(EPR_ERR_INVALID_ARG, "oversample = %d: 1, 2 or 4", oversample);
  epr_opts o{};
  o.oversample = oversample;
  CHECK(check_internal(h, geom, &o));
  if (oversample == 1)
    return epr_forward_vjp(h, geom, spec, model, phase, absorb, grad_intensity, grad_phase,
                           grad_absorb, stream);
  CHECK(check_ptr(h, phase, "phase"));
  CHECK(check_ptr(h, absorb, "absorb"));
  CHECK(check_ptr(h, grad_intensity, "grad_intensity"));
  CHECK(check_ptr(h, grad_phase, "grad_phase"));
  CHECK(check_ptr(h, grad_absorb, "grad_absorb"));
  if (grad_phase == grad_absorb) return h->fail(EPR_ERR_INVALID_ARG, "outputs must not alias");
  for (const float* in : {phase, absorb, grad_intensity})
    if (in == grad_phase || in == grad_absorb)
      return h->fail(EPR_ERR_INVALID_ARG, "the gradients must not alias the inputs");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const epr_geometry gi = internal_geometry(*geom, oversample);
  const LineParams lp = line_params(gi, *spec, nullptr, Kind::Maps);
  // the VJP's planes, then the detector gradient spread over the internal grid
  const size_t base = align256(vjp_workspace(h, gi.ny, gi.nx, lp.n));
  const size_t plane = (size_t)gi.ny * gi.nx;
  CHECK(ensure(h, h->ws, base + sizeof(float) * plane));
  float* g_int = reinterpret_cast<float*>(static_cast<char*>(h->ws.ptr) + base);
  HIP_TRY(h, launch_unbin_lines(grad_intensity, g_int, gi.ny, gi.nx, oversample, 1, st));
  ProbDesc p;
  CHECK(fill_desc(h, gi, lp, nullptr, &p));
  p.X = absorb;
  p.Y = phase;
  p.d = g_int;
  CHECK(vjp_stages(h, p, model, st, grad_phase, grad_absorb, false));
  h->last_stream = st;
  return EPR_OK;
}

int epr_forward_xspec_vjp(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                          const epr_spectrum_profile* profile, const epr_material* mat,
                          int model, const float* thickness, const float* grad_intensity,
                          float* grad_thickness, void* stream) {
  if (!h) return EPR_ERR_INVALID_ARG;
  CHECK(check_ptr(h, grad_intensity, "grad_intensity"));
  CHECK(check_ptr(h, grad_thickness, "grad_thickness"));
  if ((const float*)grad_thickness == thickness || (const float*)grad_thickness == grad_intensity)
    return h->fail(EPR_ERR_INVALID_ARG, "grad_thickness must not alias the inputs");
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  ProbDesc p;
  CHECK(xspec_maps_setup(h, geom, spec, profile, mat, model, thickness, st, nullptr, &p));
  CHECK(ensure(h, h->ws, vjp_workspace(h, geom->ny, geom->nx, p.lp.n)));
  p.d = grad_intensity;
  CHECK(vjp_stages(h, p, model, st, grad_thickness, grad_thickness, true));
  h->last_stream = st;
  return EPR_OK;
}

}  // extern "C"
