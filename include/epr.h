/*
 * epr.h -- C ABI of the MI355X (gfx950) fast eikonal phase-retrieval library (libepr.so).
 *
 * The method is Mirone et al., "Fast Eikonal Phase Retrieval for High-Throughput Beamlines"
 * (arXiv:2601.22793).  One iteration predicts the detector image of every spectral line
 * (local O(L^2) closure, Eq. 1, or the non-local ray-map transport, Eqs. 2-3 and the bilinear
 * redistribution that follows Eq. 3), sums the lines (Eq. 5), splits the detector residual
 * over the lines, carries it back to the object plane with the exact adjoint (Eq. 4), applies
 * the FFT-diagonal Paganin-type preconditioner (Section 2) and projects the updated lines onto
 * one thickness map (Eq. 7, Methods 4.4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Image arrays are DEVICE pointers owned by the caller: float32, contiguous, row-major
 *    [ny][nx] (x fastest); per-line stacks are [n_lines][ny][nx].  4-byte alignment is
 *    required, 256-byte alignment is recommended.
 *  - Struct arguments and the arrays they point to (energies, weights) are HOST memory, read
 *    during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default stream).  Every call
 *    except epr_get_diagnostics and epr_autotune only enqueues work on `stream` and returns;
 *    outputs are ready when the stream reaches that point.
 *  - Arguments are validated on the host before anything is enqueued.  Errors return a
 *    negative EPR_ERR_* code, nothing is launched, and epr_last_error() gives a message.
 *  - A handle owns device workspace (split residuals, half spectra, FFT tables, graphs).  Calls
 *    on one handle must be ordered on one stream; concurrent calls on one handle from
 *    different streams race on that workspace.  Use one handle per stream.
 *  - Sizes: 8 <= ny, nx <= 4096, nx even, and both ny and nx products of 2, 3 and 5 only
 *    (the preconditioner is a periodic FFT without padding); 1 <= n_lines <= 16.
 *
 * Units: pixel and distance in metres, energies in keV, phase in radians, absorption as
 * optical depth (A = mu * tau), thickness in metres.
 */
#ifndef EPR_H_
#define EPR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  Negative = error (nothing enqueued), 0 = success. */
#define EPR_OK 0
#define EPR_ERR_INVALID_ARG (-1) /* null pointer, non-finite or out-of-range scalar          */
#define EPR_ERR_SHAPE (-2)       /* ny/nx outside limits, odd nx, not {2,3,5}-smooth          */
#define EPR_ERR_NO_DEVICE (-3)   /* no HIP device, or device index out of range             */
#define EPR_ERR_HIP (-4)         /* a HIP runtime call failed (message has the HIP error)     */
#define EPR_ERR_OOM (-5)         /* workspace allocation failed                               */
#define EPR_ERR_UNSUPPORTED (-6) /* device is not gfx950, or model not available for the call */
#define EPR_ERR_NONFINITE (-7)   /* epr_get_diagnostics: an update of the last solve met a NaN  */
                                 /* or an infinity (its outputs are then unspecified)           */

#define EPR_MAX_LINES 16
#define EPR_MAX_DIM 4096

/* Forward models (Eq. 5): the local closure truncated at order 1 or 2 (Eq. 1), or the
 * non-local explicit ray-map transport M_s (Eq. 3, discretised by bilinear redistribution).
 * EPR_NONLOCAL_L2 is the second-order non-local model: M_s[I_s] plus the diffraction-pressure
 * (WKB1) term of Eq. 1, -eps_s^2/4 div(I_s grad Q_s) with Q_s = lap(sqrt I_s) / sqrt I_s,
 * evaluated on the object grid; its residuals go back through M_s^* like EPR_NONLOCAL's.
 * EPR_AUTO (epr_solve only) picks EPR_LOCAL_L2 or EPR_NONLOCAL with epr_select_model at
 * max_fraction = EPR_AUTO_MAX_FRACTION before iterating. */
typedef enum {
  EPR_AUTO = 0,
  EPR_LOCAL_L1 = 1,
  EPR_LOCAL_L2 = 2,
  EPR_NONLOCAL = 3,
  EPR_NONLOCAL_L2 = 4
} epr_model;
#define EPR_AUTO_MAX_FRACTION 0.01
#define EPR_MAX_BINS 1023

typedef struct epr_ctx* epr_handle;

/* Detector geometry: image size, (internal) pixel size p and propagation distance L. */
typedef struct {
  int32_t ny, nx;
  double pixel_m;
  double distance_m;
} epr_geometry;

/* Discrete spectrum (Methods 4.3): n_lines lines of energy E_s and weight w_s (sum 1), plus
 * the power laws delta_s = delta_ref (E_ref/E_s)^delta_exponent and
 * beta_s = beta_ref (E_ref/E_s)^beta_exponent used to carry material constants and object
 * maps from the reference energy to each line. */
typedef struct {
  int32_t n_lines;
  const double* energy_kev; /* host, n_lines entries, > 0      */
  const double* weight;     /* host, n_lines entries, > 0, sum 1 (within 1e-6)  */
  double energy_ref_kev;
  double delta_exponent;
  double beta_exponent;
} epr_spectrum;

/* Single material assumed by the inversion (Eqs. 6-7), at the reference energy. */
typedef struct {
  double delta_ref;
  double beta_ref;
} epr_material;

/* Solver options. */
typedef struct {
  int32_t model;      /* epr_model                                                         */
  int32_t n_iter;     /* >= 0 iterations                                                   */
  double relaxation;  /* omega in (0, 2]: I_s <- I_s + omega * preconditioned residual     */
  uint32_t flags;     /* EPR_FLAG_* */
  int32_t oversample; /* internal grid factor f: 0 or 1 (none), 2 or 4 (Section 3.2)       */
} epr_opts;

/* Record ||d - P|| / ||d|| of every iteration (read back by epr_get_diagnostics). */
#define EPR_FLAG_RESIDUALS 1u
/* epr_solve_xspec only: the block-wise interpolated preconditioner (see there) instead of the
 * column-mean Paganin filter; the profile may then have at most EPR_MAX_PRECOND_BLOCKS blocks. */
#define EPR_FLAG_BLOCK_PRECOND 2u
#define EPR_MAX_PRECOND_BLOCKS 8

/* One problem of a batched solve. */
typedef struct {
  epr_geometry geom;
  epr_spectrum spec;
  epr_material mat;
  const float* intensity; /* device [ny][nx]: flat-field-corrected detector image d        */
  float* thickness;       /* device [ny][nx] ([f ny][f nx] when oversampling by f):         */
                          /* in = start (zeros = cold start), out = tau                     */
} epr_problem;

/* Create a handle on HIP device `device`.  Fails with EPR_ERR_NO_DEVICE when no device is
 * visible and EPR_ERR_UNSUPPORTED when the device is not gfx950.  *out is NULL on failure. */
int epr_create(epr_handle* out, int device);

/* Release the handle and all its device workspace (synchronises the device first). */
int epr_destroy(epr_handle h);

/* Static description of a status code (never NULL). */
const char* epr_status_string(int status);

/* Last error message of `h` ("" if none); with h == NULL the last error of epr_create. */
const char* epr_last_error(epr_handle h);

/* Detector intensity of Eq. 5 for object maps given at the reference energy:
 *   phi_s = phase * (k_s delta_s)/(k_ref delta_ref),  I_s = w_s exp(-absorb * mu_s / mu_ref),
 *   intensity = sum_s F_s[I_s]   (F_s = P_{m,s} of Eq. 1, or M_s of Eq. 3).
 * phase, absorb, intensity: device [ny][nx].  `intensity` must not alias the inputs.
 * The operators below (forward, adjoint and their variants, the vector-Jacobian products) take
 * an explicit model: EPR_AUTO gives EPR_ERR_UNSUPPORTED, any other unknown value
 * EPR_ERR_INVALID_ARG. */
int epr_forward(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec, int model,
                const float* phase, const float* absorb, float* intensity, void* stream);

/* Per-line back-transport of detector residuals (Methods 4.4): identity for the local models,
 * the exact adjoint M_s^* of the splat (Eq. 4: bilinear interpolation at the mapped points,
 * zero off the grid) for EPR_NONLOCAL.  The ray map comes from `phase` as in epr_forward.
 * resid_lines, obj_lines: device [n_lines][ny][nx], must not alias. */
int epr_adjoint(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec, int model,
                const float* phase, const float* resid_lines, float* obj_lines, void* stream);

/* epr_forward for maps given on an oversampled internal grid (Section 3.2): phase and absorb
 * are [f ny][f nx] at pixel size p / f (geom is the detector: ny, nx, p, L); the forward model
 * runs on that grid and each detector pixel of `intensity` ([ny][nx]) records the mean of its
 * f x f internal pixels.  oversample = f is 1 (plain epr_forward), 2 or 4, and the internal grid
 * must satisfy the size rules.  Every model but EPR_AUTO (EPR_ERR_UNSUPPORTED).  Uses the
 * handle's workspace. */
int epr_forward_oversampled(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                            int model, int32_t oversample, const float* phase,
                            const float* absorb, float* intensity, void* stream);

/* Exact adjoint of epr_forward_oversampled's per-line operators: each line's detector residual
 * ([n_lines][ny][nx]) goes to its f x f internal pixels divided by f^2 (the transpose of the
 * detector mean), then through the back-transport of epr_adjoint on the internal grid (phase
 * [f ny][f nx]; identity for the local models).  obj_lines: [n_lines][f ny][f nx].  (The
 * solvers' residual path copies the detector residual without the 1/f^2 instead: there it is
 * the right inverse of the binning, Section 3.2.) */
int epr_adjoint_oversampled(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                            int model, int32_t oversample, const float* phase,
                            const float* resid_lines, float* obj_lines, void* stream);

/* Per-line Paganin-type preconditioner P_{1,s}^-1 (Section 2): each line is filtered by
 * 1 / (1 + 4 pi^2 alpha_s (fx^2 + fy^2)) with alpha_s = L delta_s / (mu_s p^2) [pixel^2] and
 * fx, fy in cycles per pixel (periodic boundary).  in_lines, out_lines: device
 * [n_lines][ny][nx]; in-place (in_lines == out_lines) is allowed. */
int epr_precondition(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                     const epr_material* mat, const float* in_lines, float* out_lines,
                     void* stream);

/* Shift-to-pixel ratio histogram of every line (Section 2; Section 3.1 shows the same
 * per-line distribution for the strong-shift bamboo test).  For the thickness map tau and line
 * s, eta_s = ||Delta_s|| / p with Delta_s = (L / k_s) grad phi_s and phi_s = -k_s delta_s tau,
 * so eta_s = c_s ||D tau|| with c_s = L delta_s / p^2 and D the pixel-unit derivative
 * (central difference inside, one-sided on the first and last sample of each axis).
 * thickness: device [ny][nx].  counts: device uint32 [n_lines][n_bins + 1], overwritten: bin
 * i < n_bins holds the pixels with i <= eta_s n_bins / eta_max < i + 1, bin n_bins those with
 * eta_s >= eta_max.  The bin of a pixel is decided in float32, every operation rounded on its
 * own: g = sqrt(Dx*Dx + Dy*Dy), v = ((float)c_s * g) * ((float)n_bins / (float)eta_max),
 * bin = min(floor(v), n_bins).  Counts are exact integers (independent of the order).
 * 1 <= n_bins <= EPR_MAX_BINS; eta_max > 0 and finite. */
int epr_regime(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
               const epr_material* mat, const float* thickness, int32_t n_bins, double eta_max,
               uint32_t* counts, void* stream);

/* Automatic local / non-local choice (Section 2: the local O(L^2) closure needs eta < 1 over
 * most of the field of view).  The regime is measured on the Paganin retrieval of `intensity`
 * (device [ny][nx]): one iteration from tau = 0 with relaxation 1, where every model gives the
 * same update.  *model_out = EPR_LOCAL_L2 when, for every line, at most max_fraction * ny * nx
 * pixels have eta_s >= 1 (epr_regime with one bin of width 1), else EPR_NONLOCAL.
 * over_counts: optional host array of n_lines receiving those pixel counts (NULL to skip).
 * max_fraction in [0, 1].  Uses the handle's workspace and synchronises `stream`. */
int epr_select_model(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                     const epr_material* mat, const float* intensity, double max_fraction,
                     int32_t* model_out, uint32_t* over_counts, void* stream);

/* Full EPR solve (Methods 4.4) of one projection.  intensity: device [ny][nx] detector image.
 * thickness: device [ny][nx], in/out -- the start (zeros for a cold start, so the first
 * iteration is a Paganin retrieval) and the result tau after opts->n_iter iterations; calling
 * again continues the iteration (resume).  phase_out: optional device [ny][nx] (NULL to skip)
 * receiving phi_ref = -k_ref delta_ref tau.  Each iteration, per line s:
 *   I_s = w_s exp(-mu_s tau), phi_s = -k_s delta_s tau, P_s = F_s[I_s];
 *   e = d - sum_s P_s, e_s = e max(P_s,0) / sum_s' max(P_s',0) (w_s e where that sum is 0);
 *   r_s = e_s (local) or M_s^* e_s (non-local); dI_s = P_{1,s}^-1 r_s;
 *   tau = -sum_s w_s mu_s ln(max(I_s + omega dI_s, 1e-6 w_s) / w_s) / sum_s w_s mu_s^2. */
int epr_solve(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
              const epr_material* mat, const epr_opts* opts, const float* intensity,
              float* thickness, float* phase_out, void* stream);
/* (opts->model = EPR_AUTO first runs epr_select_model on `intensity`, which synchronises the
 * stream once; epr_get_diagnostics reports the model used.)
 * Oversampling (opts->oversample = f of 2 or 4, Section 3.2): the solver works on an internal
 * grid of (f ny) x (f nx) pixels of size p / f; the detector pixel records the mean of its
 * f x f internal pixels.  `intensity` stays the detector image [ny][nx]; `thickness` and
 * `phase_out` are on the internal grid, [f ny][f nx].  Each iteration predicts every line on
 * the internal grid, bins the predictions to the detector, splits the detector residual there
 * and copies each line's share back to its f x f internal pixels before the back-transport and
 * the preconditioner (at the internal pixel size).  The internal grid must satisfy the size
 * rules (so f nx <= 4096, products of 2, 3, 5). */

/* x-dependent effective spectrum (Methods 4.3, remark on spatially varying spectra: the
 * effective spectrum, and with it f_s, gamma_s and db_s = delta_s / beta_s of Eq. 6, may vary
 * slowly across the detector columns x).  It is tabulated on n_blocks column blocks: block b is
 * centred on detector column block_x[b] (increasing, in pixels) and gives line s the energy
 * energy_kev[b * n_lines + s] and the weight weight[b * n_lines + s] (each block's weights
 * sum to 1).  Column x uses, per line, the energy and the weight interpolated linearly between
 * the two nearest centres (held constant beyond the outer ones); every per-line constant
 * follows from them through the power laws of epr_spectrum.  All arrays are host memory. */
typedef struct {
  int32_t n_blocks;          /* 1 .. 4096 */
  const double* block_x;     /* [n_blocks] */
  const double* energy_kev;  /* [n_blocks][n_lines], > 0 */
  const double* weight;      /* [n_blocks][n_lines], > 0, each block sums to 1 (within 1e-6) */
} epr_spectrum_profile;

/* epr_solve with an x-dependent spectrum (every model but EPR_AUTO; oversampling allowed).
 * spec gives n_lines, energy_ref_kev and the exponents (its energy and weight arrays are not
 * read); profile the spectrum per column.  With oversampling by f the constants are taken per
 * internal column, whose centre lies at detector column (x + 1/2) / f - 1/2, and the split
 * fallback of a detector pixel is the line weight averaged over its f internal columns.  Per column x and line s the
 * iteration uses I_s = w_s(x) exp(-mu_s(x) tau), the shift u_s = -(L delta_s(x) / p^2) D tau
 * (the thickness gradient alone moves the rays), the split fallback w_s(x) and the projection
 * weights w_s(x) mu_s(x).  The preconditioner of line s is the Paganin filter at the column mean
 * of alpha_s: it stays FFT-diagonal, and the fixed point does not depend on it.  With
 * opts->flags & EPR_FLAG_BLOCK_PRECOND it is block-wise instead (the remark's block-wise
 * filtering with interpolation): block b filters the residual with the Paganin filter of
 * alpha_s at its own energies, and column x blends those outputs with the spectrum's
 * interpolation weights (1 - t for the centre at or before x, t for the next one), which costs
 * one column pass and one row-inverse transform per block and line.  The call
 * synchronises `stream` once, before it replaces the handle's per-column table; otherwise as
 * epr_solve (arguments, ownership, errors; EPR_AUTO gives EPR_ERR_UNSUPPORTED). */
int epr_solve_xspec(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                    const epr_spectrum_profile* profile, const epr_material* mat,
                    const epr_opts* opts, const float* intensity, float* thickness,
                    float* phase_out, void* stream);

/* epr_solve for callers that cannot allocate device memory (code recorded under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The same iteration, kernels
 * and results as epr_solve, but the workspace (split residuals, half spectra, max-gradient and
 * residual partials) and the FFT twiddle tables live in one fixed device array of
 * EPR_NOALLOC_SCRATCH_BYTES per GPU, reserved when the library is loaded and held until the
 * process ends; the call makes no hipMalloc, hipFree or graph instantiation and enqueues every
 * launch directly on `stream` (stage timing is not recorded).  The caller still passes the
 * inputs and outputs.  The array needs about 8 * n_lines bytes per (internal) pixel plus
 * 8 (ny + nx) bytes of tables: a larger problem returns EPR_ERR_UNSUPPORTED with the sizes in
 * the message, as does EPR_AUTO (its model selection needs its own buffers).  Every call on a
 * GPU shares that GPU's array, whatever the handle or stream, and nothing in it has to start
 * at zero: calls that overlap in time on one GPU race on it, so order them on one stream.
 * epr_get_diagnostics reports on it as on epr_solve.  Arguments, ownership and the other
 * errors as epr_solve. */
#define EPR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int epr_solve_noalloc(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                      const epr_material* mat, const epr_opts* opts, const float* intensity,
                      float* thickness, float* phase_out, void* stream);

/* Solve n independent problems (sizes, distances, spectra and materials may differ; all must
 * have the same n_lines) with the same options.  Each stage of an iteration is one launch
 * covering every problem, and the whole opts->n_iter loop is captured once into a HIP graph
 * that is cached on the handle (keyed by the problem list) and replayed.  Results equal
 * n calls of epr_solve up to floating-point summation order.  problems: host array of n.
 * EPR_AUTO is not accepted here (EPR_ERR_UNSUPPORTED): select per problem first.  With
 * opts->oversample = f every problem's thickness is on its internal grid, [f ny][f nx]. */
int epr_solve_batched(epr_handle h, int32_t n, const epr_problem* problems,
                      const epr_opts* opts, void* stream);

/* epr_solve_batched with an x-dependent spectrum per problem (Methods 4.3 remark on spatially
 * varying spectra; as epr_solve_xspec): profiles is a host array of n profiles, profiles[i]
 * for problems[i] (whose spec gives n_lines, energy_ref_kev and the exponents; its energy and
 * weight arrays are not read).  Every problem uses the column-mean Paganin filter
 * (EPR_FLAG_BLOCK_PRECOND gives EPR_ERR_UNSUPPORTED here).  Results equal n calls of
 * epr_solve_xspec up to floating-point summation order; the graph is cached and replayed as in
 * epr_solve_batched (keyed by the problems and the profiles' contents). */
int epr_solve_batched_xspec(epr_handle h, int32_t n, const epr_problem* problems,
                            const epr_spectrum_profile* profiles, const epr_opts* opts,
                            void* stream);

/* Detector intensity under an x-dependent spectrum (Eq. 5 with the per-column constants of
 * epr_solve_xspec; Methods 4.3 remark on spatially varying spectra): the forward model that
 * epr_solve_xspec inverts, sum_s F_s[I_s] with I_s = w_s(x) exp(-mu_s(x) tau) and the shift
 * u_s = -(L delta_s(x) / p^2) D tau, for a single-material thickness map.  Every model but
 * EPR_AUTO (EPR_ERR_UNSUPPORTED); no oversampling.  spec gives n_lines, energy_ref_kev and the
 * exponents (its energy and weight arrays are not read), profile the spectrum per column, mat the
 * material.  thickness, intensity: device [ny][nx], must not alias.  Synchronises the stream
 * before replacing the handle's device copy of the per-column table. */
int epr_forward_xspec(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                      const epr_spectrum_profile* profile, const epr_material* mat, int model,
                      const float* thickness, float* intensity, void* stream);

/* Per-line back-transport under an x-dependent spectrum (as epr_adjoint, Eq. 4, with the
 * column shifts of epr_forward_xspec): identity for the local models, the exact adjoint M_s^* of
 * the splat for EPR_NONLOCAL and EPR_NONLOCAL_L2.  resid_lines, obj_lines: device
 * [n_lines][ny][nx], must not alias. */
int epr_adjoint_xspec(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                      const epr_spectrum_profile* profile, const epr_material* mat, int model,
                      const float* thickness, const float* resid_lines, float* obj_lines,
                      void* stream);

/* Vector-Jacobian product of epr_forward with respect to phase and absorb, for every model
 * but EPR_AUTO (EPR_ERR_UNSUPPORTED): given grad_intensity = dL/d(intensity), writes
 * grad_phase = dL/d(phase) and grad_absorb = dL/d(absorb) (device [ny][nx] each, overwritten).
 * Non-local models: the transpose of the splat is the bilinear interpolation of Eq. 4, and the
 * splat's weights are differentiated inside each cell (piecewise linear in the shift).  Local
 * closures (Eq. 1, Methods 4.1) and the diffraction-pressure term of EPR_NONLOCAL_L2: the chain
 * rule through the derivative compositions of Eq. 1 with the exact transpose of D.  The ray maps
 * and closure terms are recomputed from `phase` and `absorb`; nothing is saved from the forward
 * call.  Uses the handle's workspace (2 + 2 n_lines planes of ny x nx floats for the
 * second-order models).  The gradients must not alias each other or the inputs. */
int epr_forward_vjp(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec, int model,
                    const float* phase, const float* absorb, const float* grad_intensity,
                    float* grad_phase, float* grad_absorb, void* stream);

/* Vector-Jacobian product of epr_forward_oversampled (Section 3.2) with respect to the maps on
 * the internal grid, for every model but EPR_AUTO (EPR_ERR_UNSUPPORTED): grad_intensity
 * = dL/d(intensity) on the detector ([ny][nx]) is spread over the internal grid (the transpose
 * of the detector mean: each value copied to its f x f internal pixels and divided by f^2),
 * then the internal-grid product of epr_forward_vjp writes grad_phase and grad_absorb (device
 * [f ny][f nx] each, overwritten).  oversample = f is 1 (plain epr_forward_vjp), 2 or 4, and
 * the internal grid must satisfy the size rules.  The gradients must not alias each other or
 * the inputs.  Uses the handle's workspace (that of epr_forward_vjp on the internal grid plus
 * one internal-grid plane). */
int epr_forward_vjp_oversampled(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                                int model, int32_t oversample, const float* phase,
                                const float* absorb, const float* grad_intensity,
                                float* grad_phase, float* grad_absorb, void* stream);

/* Vector-Jacobian product of epr_forward_xspec with respect to the thickness, for every model
 * but EPR_AUTO (EPR_ERR_UNSUPPORTED): given grad_intensity = dL/d(intensity), writes
 * grad_thickness = dL/d(tau) = sum_s -mu_s(x) I_s dL/dI_s + D_x^T(b_s(x) dL/du_x,s)
 * + D_y^T(b_s(x) dL/du_y,s) (device [ny][nx], overwritten), the per-line gradients being those
 * of epr_forward_vjp with each line's constants read at the pixel's column (the pressure
 * coefficient of a column scales the term after its outer derivative).  Arguments as for
 * epr_forward_xspec; grad_thickness must not alias thickness or grad_intensity.  Synchronises
 * the stream before replacing the handle's device copy of the per-column table; uses the
 * handle's workspace as epr_forward_vjp does. */
int epr_forward_xspec_vjp(epr_handle h, const epr_geometry* geom, const epr_spectrum* spec,
                          const epr_spectrum_profile* profile, const epr_material* mat,
                          int model, const float* thickness, const float* grad_intensity,
                          float* grad_thickness, void* stream);

/* Diagnostics of the last epr_solve / epr_solve_xspec / epr_solve_batched on this handle.
 * Synchronises the stream of that call.
 * Failure detection: every solve clears one device flag per problem, and the update kernel
 * sets it when a preconditioned residual or the projected thickness of any pixel is a NaN or
 * an infinity (non-finite data, for example; data <= 0 is floored by the projection and stays
 * finite).  A NaN would otherwise be hidden by the floor of the update.  When a flag is set the
 * call fills *out and returns EPR_ERR_NONFINITE; the thickness of that problem is unspecified. */
typedef struct {
  int32_t n_iter;             /* iterations recorded                                    */
  int32_t n_problems;         /* problems of the last call                              */
  int32_t model;              /* model used (the one chosen when the call asked for EPR_AUTO) */
  float max_shift_px;         /* largest |u_s| (pixels) at the last non-local iteration (else 0) */
  float residual[256];        /* ||e||/||d|| per iteration of problem 0, in the caller's order
                                 (EPR_FLAG_RESIDUALS; batched solves included)           */
  int32_t nonfinite;          /* number of problems whose update met a NaN or an infinity */
  int32_t first_nonfinite;    /* index (caller's order) of the first such problem, or -1   */
} epr_diagnostics;

int epr_get_diagnostics(epr_handle h, epr_diagnostics* out);

/* Autotuner of the launch choices (they change the time, not the iteration: every choice
 * computes the same values up to float32 summation order): the splat tile shape (transport
 * models), the lines a row-pass workgroup transforms one after the other (1, 2 or 4: the
 * lines of a row block share its thickness stencil), and the radix order of every transform
 * length that has several compiled orders
 * (row lengths nx/2 = 512, 1024, 1280, 2048; column lengths ny = 1024, 2048, 2160).  Every
 * candidate is timed on one iteration of the batched solve of the given problems (a batch of
 * one for a single problem), replayed from its graph, after two iterations from each
 * problem's own thickness, all on copies: the shifts, and with them the halo every splat tile
 * reads, are representative.  The dimensions are tuned one after the other, each with the
 * others at their best so far; a candidate replaces the value in use only when it is at least
 * 1 % faster (smaller differences are timing noise).  The choices are kept on the handle for
 * every later call
 * (sizes are those of the internal grid when opts->oversample > 1).  The problems' data and
 * thickness are only read; the handle's cached batched graph is replaced (the next
 * epr_solve_batched captures its own again) and epr_get_diagnostics still reports on the
 * caller's last solve.
 * cache_json (may be NULL) is a file path: when it holds a flat JSON object of integers
 * {"splat_tx": 64, "splat_ty": 32, "row_1024": 0, "col_2048": 1, ...} whose entries are all
 * valid for these problems (a tile of at most 4096 pixels whose per-line LDS accumulators fit
 * in 160 KB for their line count, radix-order indices in range), those choices are taken
 * without timing anything; an absent, malformed or invalid file is ignored, and the timed
 * choices are written to it.  Synchronous (synchronises the device first). */
int epr_autotune(epr_handle h, int32_t n, const epr_problem* problems, const epr_opts* opts,
                 const char* cache_json);

/* Per-stage kernel timing with HIP events recorded on the launch stream around every stage
 * launch.
 * Stages: 0 max-gradient, 1 splat, 2 local closure, 3 row FFT (+ back-transport), 4 column
 * FFT + filter, 5 row inverse FFT + update, 6 vector-Jacobian product, 7 detector binning and
 * residual split (oversampled solves). */
#define EPR_N_STAGES 8
typedef struct {
  double ms[EPR_N_STAGES];        /* summed kernel time per stage since the last reset       */
  int64_t launches[EPR_N_STAGES]; /* launches per stage since the last reset                 */
  /* The same totals split by size class: class 0 = problems up to 2048 x 2048 pixels (spectral
   * kernels of 512 threads), class 1 = larger ones (1024 threads).  A batched solve makes one
   * launch per stage and size class present in the batch. */
  double ms_class[EPR_N_STAGES][2];
  int64_t launches_class[EPR_N_STAGES][2];
} epr_timing;

/* Enable (1) or disable (0) timing and reset the totals.  While enabled, epr_solve_batched
 * enqueues its launch sequence directly on the stream instead of replaying the cached graph
 * (same kernels, grids and order), because events inside a graph cannot be timed. */
int epr_set_timing(epr_handle h, int enabled);

/* Synchronise the last stream used and return the totals accumulated since the reset. */
int epr_get_timing(epr_handle h, epr_timing* out);

/* Host-only helpers (no device needed). */

/* Radix sequence of the library's FFT for length n (a product of 2, 3 and 5): writes up to
 * `capacity` radices to `radices` (host) and returns the number of stages, EPR_ERR_SHAPE if n
 * has another prime factor, EPR_ERR_INVALID_ARG for n < 1 or a NULL array with capacity > 0. */
int epr_fft_plan(int32_t n, int32_t* radices, int32_t capacity);

/* Validate a problem description exactly as the solver entry points do, without a device.
 * mat and opts may be NULL (not checked).  The message goes to msg (host, msg_len bytes, may
 * be NULL).  Returns EPR_OK or the EPR_ERR_* the solver would return. */
int epr_check_problem(const epr_geometry* geom, const epr_spectrum* spec,
                      const epr_material* mat, const epr_opts* opts, char* msg, size_t msg_len);

#ifdef __cplusplus
}
#endif

#endif /* EPR_H_ */
