// Host side of libepr: the handle's life cycle, validation, per-line constants, FFT plans,
// workspace layout, the launch sequence of one EPR iteration (Methods 4.4), graph capture of
// the single-problem solves, diagnostics and stage timing.  The other entry points of the C
// ABI (include/epr.h) are in api_ops.cpp, api_solve.cpp, api_batch.cpp and api_tune.cpp.
#include "host.h"

using namespace epr;
using namespace epr::host;

namespace epr {
namespace host {

thread_local std::string g_create_error;

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
              const float2* table) {
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
  if (model == EPR_AUTO)
    return h->fail(EPR_ERR_UNSUPPORTED, "EPR_AUTO is accepted by epr_solve only: this call "
                   "needs an explicit model");
  if (model != EPR_LOCAL_L1 && model != EPR_LOCAL_L2 && model != EPR_NONLOCAL &&
      model != EPR_NONLOCAL_L2)
    return h->fail(EPR_ERR_INVALID_ARG, "unknown model %d", model);
  return EPR_OK;
}

int check_opts(epr_ctx* h, const epr_opts* o, bool allow_auto, bool allow_block) {
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


// Solve: X = Y = tau, I_s = w exp(-mu_s tau), u_s = -(L delta_s / p^2) D tau.
// Maps (forward/adjoint/vjp): X = absorption, Y = phase at E_ref,
//   I_s = w exp(-(mu_s/mu_ref) A), u_s = eps_s phase_scale_s D phase.
LineParams line_params(const epr_geometry& g, const epr_spectrum& s, const epr_material* m,
                       Kind kind, double relax_unused) {
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
              const float2* row_tab, const float2* col_tab) {
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

// The solves' row pass takes the tuned lines per workgroup.
void apply_row_lines(const epr_ctx* h, ProbDesc* p) { p->rlpb = h->row_lines; }

KArgs single(const ProbDesc& p, int mode) {
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.p = p;
  a.mode = mode;
  return a;
}


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



int check_ptr(epr_ctx* h, const void* p, const char* name) {
  if (!p) return h->fail(EPR_ERR_INVALID_ARG, "%s is NULL", name);
  if (!aligned4(p)) return h->fail(EPR_ERR_INVALID_ARG, "%s is not 4-byte aligned", name);
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

}  // namespace host
}  // namespace epr

// ==============================================================================================
// C ABI: life cycle, host-only helpers, diagnostics, timing
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

}  // extern "C"
