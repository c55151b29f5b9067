"""FP64 CPU oracle of the fast eikonal phase-retrieval (EPR) iteration.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the entry module and the CPU-baseline
leg of the benchmark may import or run this module.  The HIP library shares no code, header,
table or constant with it; the two meet only through the seeded inputs of ``synthetic/``.

It follows Mirone et al., "Fast Eikonal Phase Retrieval for High-Throughput Beamlines"
(arXiv:2601.22793).  Citations below name the paper's sections and equations:

* Eq. (1)  local O(L^2) intensity closure (Methods 4.1; the same expansion is Eq. S20)
* Eq. (2)  per-line ray map r' = r + (L/k_s) grad phi_s, worked in pixel units (Methods 4.2)
* Eq. (3)  non-local forward operator M_s (Methods 4.2)
* the unnumbered display after Eq. (3): conservative bilinear redistribution ("splat")
* Eq. (4)  adjoint of the splat = bilinear interpolation (Methods 4.2)
* Eq. (5)  incoherent spectral sum (Methods 4.3)
* Eq. (6)  single-material relation phi_s = (delta_s / 2 beta_s) ln I_s (Methods 4.3)
* Eq. (7)  single-thickness parameterisation I_s = f_s exp(-gamma_s tau) (Methods 4.4)
* Methods 4.4 "Iteration structure" and "Projection to the single-thickness manifold"
* Section 2 "Linear term and relation to Paganin": the FFT-diagonal preconditioner P_{1,s}^-1
* Eq. S8   eps = L / k

Readings where the paper is silent or under-specified (each is stated where it is used):

R1  derivatives: one operator D = numpy.gradient with unit (pixel) spacing -- central
    differences inside, first-order one-sided differences on the first/last sample.  Every
    higher derivative in Eq. (1) is a composition of D, as the equation is written.
R2  boundaries: splat mass landing off the grid is lost, the interpolation reads zero off the
    grid, the preconditioner is periodic (no padding).
R3  preconditioner symbol: 1 / (1 + 4 pi^2 alpha_s (fx^2 + fy^2)) on numpy's fftfreq/rfftfreq
    grids, alpha_s = eps_s delta_s / (2 beta_s p^2) = L delta_s / (mu_s p^2) in pixel^2.
R4  start from tau = 0 (so the first iteration is exactly a Paganin retrieval).
R5  the preconditioned residual is added to each line's intensity with relaxation omega.
R7  residual split: pi_s = max(P_s, 0) / sum_s' max(P_s', 0), falling back to the line weight
    w_s where that sum is <= 1e-30; e_s = pi_s e, so sum_s e_s = e exactly.
R8  projection: weighted least squares of ln(I_s / w_s) = -mu_s tau with weights w_s after
    flooring I_s at 1e-6 w_s, i.e. tau = -sum_s w_s mu_s ln(I_s/w_s) / sum_s w_s mu_s^2.
R9  the non-local model is the pure transport M_s (no diffraction-pressure term).
R22 the "second-order non-local" model adds the diffraction-pressure (WKB1) term of Eq. (1),
    evaluated from I_s on the object grid, to the transported intensity: P_s = M_s[I_s] -
    eps^2/4 d_i(I_s d_i Q_s).  Moving that O(L^2) term along the ray map would change it only at
    O(L^3).  Its residual goes back through M_s^* like the pure transport's.
R11 per-line material constants follow power laws delta ~ E^-n_delta, beta ~ E^-n_beta from a
    reference energy; the spectral fraction f_s is the line weight w_s and gamma_s = mu_s.
R15 floor (not truncation) gives the lower cell corner, so negative targets work.
R21 oversampled grids (Section 3.2: factor 2 for the local solver, 4 for the non-local one):
    the detector pixel records the mean of its f x f internal pixels (binning B), and the
    detector residual goes back to the internal grid by replication, the right inverse of B,
    so that the preconditioned update matches a detector-level residual one to one.
R23 x-dependent effective spectrum (the file format and the block-wise interpolation are in
    the absent supplementary information): per line, energy and weight tabulated on column
    blocks and interpolated linearly in x; all constants follow per column.  Shifts come from
    the thickness gradient alone, u_s = -L delta_s(x) D tau / p^2.  The default preconditioner
    uses the column mean of alpha_s, which keeps it FFT-diagonal.
R24 block-wise interpolated preconditioner for that spectrum (the paper's remark names a
    block-wise filtering with interpolation; its details are in the absent supplementary
    information): each column block b filters the residual with the Paganin filter of its own
    centre constant alpha_s^(b), and column x takes the blend sum_b lambda_b(x) of those
    outputs with the same linear-interpolation weights lambda_b(x) as the spectrum (hat
    functions of the block centres, held constant beyond the outer ones; they sum to 1).
R19 the regime histogram's bin of a pixel is decided in float32 (the paper gives no
    precision; a float that decides an integer is computed as the kernel computes it).
R20 "eta < 1 over most of the field of view" (Section 2) is read as: at most a fraction
    max_fraction (default 1 %) of the pixels have eta_s >= 1, for every line, measured on the
    Paganin retrieval of the data.

Pins (tests/test_oracle_*.py) fix every function against something other than itself:
numpy.gradient exactness on polynomials, scipy.ndimage.map_coordinates, brute-force dense
transposes, conservation, closed forms (thin lens, Gaussian diffraction pressure, homogeneous
sphere, pure cosine filtering, constant shifts), the textbook Paganin retrieval and solver
invariants.  The non-local solver trajectory beyond its components is pinned only by its
invariants (line splitting, resume, identical lines, local/non-local agreement as L -> 0).
"""

from dataclasses import dataclass

import numpy as np

HC_EV_M = 1.239841984e-6   # h c in eV m
LOCAL_L1, LOCAL_L2, NONLOCAL = "local_l1", "local_l2", "nonlocal"
NONLOCAL_L2 = "nonlocal_l2"   # transport plus the diffraction-pressure term (R22)
MODELS = (LOCAL_L1, LOCAL_L2, NONLOCAL)
TRANSPORT_MODELS = (NONLOCAL, NONLOCAL_L2)   # models back-transported with M_s^*


# ----------------------------------------------------------------------------------------------
# Per-line constants
# ----------------------------------------------------------------------------------------------

@dataclass
class Lines:
    """Per-line constants, all float64 arrays of length N_s."""
    w: np.ndarray        # spectral weight (sum 1)
    k: np.ndarray        # wavenumber 2 pi / lambda_s            [1/m]
    delta: np.ndarray    # refractive decrement at E_s
    beta: np.ndarray     # absorption index at E_s
    mu: np.ndarray       # linear attenuation 2 k_s beta_s        [1/m]
    eps_px: np.ndarray   # eps_s / p^2 = L / (k_s p^2)            (Eq. S8, pixel units)
    alpha_px: np.ndarray # eps_px delta_s / (2 beta_s)            [pixel^2] (R3)
    phase_scale: np.ndarray   # phi_s / phi_ref = k_s delta_s / (k_ref delta_ref)
    absorb_scale: np.ndarray  # A_s / A_ref = mu_s / mu_ref


def line_constants(energies_kev, weights, pixel_m, distance_m, delta_ref=1.0, beta_ref=1.0,
                   energy_ref_kev=60.0, delta_exponent=2.0, beta_exponent=3.0):
    """Constants of each spectral line (Methods 4.2-4.3, Eq. S8; reading R11)."""
    e = np.asarray(energies_kev, dtype=np.float64) * 1e3
    w = np.asarray(weights, dtype=np.float64)
    lam = HC_EV_M / e
    k = 2.0 * np.pi / lam
    ratio = (energy_ref_kev * 1e3) / e
    delta = delta_ref * ratio ** delta_exponent
    beta = beta_ref * ratio ** beta_exponent
    mu = 2.0 * k * beta
    eps_px = distance_m / k / pixel_m ** 2
    alpha_px = eps_px * delta / (2.0 * beta)
    k_ref = 2.0 * np.pi / (HC_EV_M / (energy_ref_kev * 1e3))
    phase_scale = (k * delta) / (k_ref * delta_ref)
    absorb_scale = mu / (2.0 * k_ref * beta_ref)
    return Lines(w, k, delta, beta, mu, eps_px, alpha_px, phase_scale, absorb_scale)


# ----------------------------------------------------------------------------------------------
# Derivative operator (R1)
# ----------------------------------------------------------------------------------------------

def dx(f):
    """D_x: derivative along x (axis 1) in pixel units (R1)."""
    return np.gradient(f, axis=1)


def dy(f):
    """D_y: derivative along y (axis 0) in pixel units (R1)."""
    return np.gradient(f, axis=0)


def gradient_matrix(n):
    """Dense n x n matrix of D along one axis: column j is D applied to the unit vector e_j."""
    return np.gradient(np.eye(n), axis=0)


def _gradient_matrix_sparse(n):
    """gradient_matrix(n) held as a sparse matrix (the same entries; at most three per row)."""
    from scipy import sparse
    return sparse.csr_matrix(gradient_matrix(n))


def dx_transpose(g):
    """D_x^T: exact transpose of D_x (used by the vector-Jacobian product): g times the matrix
    of D along x, row by row."""
    return np.asarray((_gradient_matrix_sparse(g.shape[1]).T @ np.asarray(g).T).T)


def dy_transpose(g):
    """D_y^T: exact transpose of D_y."""
    return np.asarray(_gradient_matrix_sparse(g.shape[0]).T @ np.asarray(g))


# ----------------------------------------------------------------------------------------------
# Forward operators
# ----------------------------------------------------------------------------------------------

def shift_field(phi, eps_px):
    """Eq. (2) in pixel units: u_s = (eps_s / p^2) grad phi_s.  Returns (u_x, u_y)."""
    return eps_px * dx(phi), eps_px * dy(phi)


def local_forward(I, phi, eps_px, order=2):
    """Local closure P_{m,s}[I_s] of Eq. (1), truncated at order m in eps (m = 1 or 2).

    P = I - eps d_i(I d_i phi)
          + eps^2/2 d_i d_j(I d_i phi d_j phi) - eps^2/4 d_i(I d_i Q),
    Q = lap(sqrt I) / sqrt I, with eps in pixel units and d = D (R1).
    """
    e = eps_px
    gx, gy = dx(phi), dy(phi)
    P = I - e * (dx(I * gx) + dy(I * gy))
    if order >= 2:
        P = P + 0.5 * e * e * (dx(dx(I * gx * gx)) + dx(dy(I * gx * gy))
                               + dy(dx(I * gy * gx)) + dy(dy(I * gy * gy)))
        A = np.sqrt(I)
        Q = (dx(dx(A)) + dy(dy(A))) / A
        P = P - 0.25 * e * e * (dx(I * dx(Q)) + dy(I * dy(Q)))
    return P


def diffraction_pressure(I, eps_px):
    """The WKB1 term of Eq. (1) alone: -eps^2/4 d_i(I d_i Q), Q = lap(sqrt I) / sqrt I."""
    e = eps_px
    A = np.sqrt(I)
    Q = (dx(dx(A)) + dy(dy(A))) / A
    return -0.25 * e * e * (dx(I * dx(Q)) + dy(I * dy(Q)))


def _corners(ux, uy):
    """Lower-left cell corner and fractional offsets of the mapped points (R15).

    Returns (x0, y0, fx, fy) with x0 = floor(x + u_x), fx = x + u_x - x0, same for y.
    """
    ny, nx = ux.shape
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    xt = x + ux
    yt = y + uy
    x0 = np.floor(xt)
    y0 = np.floor(yt)
    return x0.astype(np.int64), y0.astype(np.int64), xt - x0, yt - y0


def _bilinear_taps(ux, uy):
    """The four (row offset, column offset, weight) taps of the paper's bilinear weights:
    w00 = (1-dx)(1-dy) at (y0, x0), w10 = dx(1-dy) at (y0, x0+1), w01 = (1-dx)dy at (y0+1, x0),
    w11 = dx dy at (y0+1, x0+1)."""
    x0, y0, fx, fy = _corners(ux, uy)
    return x0, y0, (
        (0, 0, (1 - fx) * (1 - fy)),
        (0, 1, fx * (1 - fy)),
        (1, 0, (1 - fx) * fy),
        (1, 1, fx * fy),
    )


def splat(I, ux, uy):
    """Discrete non-local forward M_s (display after Eq. (3)): every source pixel (y, x) adds
    I(y, x) * w_ij to the four detector pixels around (x + u_x, y + u_y).  Off-grid targets
    are dropped (R2)."""
    ny, nx = I.shape
    x0, y0, taps = _bilinear_taps(ux, uy)
    P = np.zeros(ny * nx)
    for oy, ox, wgt in taps:
        ty, tx = y0 + oy, x0 + ox
        ok = (ty >= 0) & (ty < ny) & (tx >= 0) & (tx < nx)
        P += np.bincount((ty[ok] * nx + tx[ok]), weights=(I * wgt)[ok], minlength=ny * nx)
    return P.reshape(ny, nx)


def gather(e, ux, uy):
    """Adjoint M_s^* of Eq. (4): bilinear interpolation of e at (x + u_x, y + u_y), with zero
    outside the grid (R2)."""
    ny, nx = e.shape
    x0, y0, taps = _bilinear_taps(ux, uy)
    r = np.zeros((ny, nx))
    for oy, ox, wgt in taps:
        ty, tx = y0 + oy, x0 + ox
        ok = (ty >= 0) & (ty < ny) & (tx >= 0) & (tx < nx)
        vals = np.zeros((ny, nx))
        vals[ok] = e[ty[ok], tx[ok]]
        r += wgt * vals
    return r


# ----------------------------------------------------------------------------------------------
# Inversion pieces
# ----------------------------------------------------------------------------------------------

def split_residual(d, P_lines, weights):
    """Methods 4.4: detector residual e = d - sum_s P_s, split per line with positivity
    weights (R7).  Returns (e_s [N_s, ny, nx], e)."""
    e = d - P_lines.sum(axis=0)
    pos = np.maximum(P_lines, 0.0)
    tot = pos.sum(axis=0)
    hole = tot <= 1e-30
    share = pos / np.where(hole, 1.0, tot)
    share = np.where(hole[None], np.asarray(weights)[:, None, None], share)
    return share * e[None], e


def paganin_filter(r, alpha_px):
    """P_{1,s}^-1 (Section 2, linear term): the FFT-diagonal inverse of the linearised operator
    I - alpha lap, i.e. multiplication of the spectrum by 1 / (1 + 4 pi^2 alpha (fx^2 + fy^2))
    (R3)."""
    ny, nx = r.shape
    fy = np.fft.fftfreq(ny)[:, None]
    fx = np.fft.rfftfreq(nx)[None, :]
    H = 1.0 / (1.0 + 4.0 * np.pi ** 2 * alpha_px * (fy ** 2 + fx ** 2))
    return np.fft.irfft2(np.fft.rfft2(r) * H, s=(ny, nx))


def project_single_thickness(I_lines, lines):
    """Methods 4.4 projection onto Eq. (7) with f_s = w_s, gamma_s = mu_s (R8): floor each line
    at 1e-6 w_s, then weighted least squares of ln(I_s / w_s) = -mu_s tau."""
    w = lines.w[:, None, None]
    mu = lines.mu[:, None, None]
    Ic = np.maximum(I_lines, 1e-6 * w)
    return -(w * mu * np.log(Ic / w)).sum(axis=0) / (lines.w * lines.mu ** 2).sum()


def line_intensities(tau, lines):
    """Eq. (7): I_s = w_s exp(-mu_s tau)."""
    return lines.w[:, None, None] * np.exp(-lines.mu[:, None, None] * tau[None])


def line_phases(tau, lines):
    """Single-material phase per line, phi_s = -k_s delta_s tau (consistent with Eq. (6))."""
    return -(lines.k * lines.delta)[:, None, None] * tau[None]


def forward_lines(I_lines, phi_lines, lines, model):
    """Per-line predictions F_s[I_s] of Eq. (5): P_{m,s} for the local models, M_s non-local."""
    out = np.empty_like(I_lines)
    for s in range(I_lines.shape[0]):
        if model in TRANSPORT_MODELS:
            ux, uy = shift_field(phi_lines[s], lines.eps_px[s])
            out[s] = splat(I_lines[s], ux, uy)
            if model == NONLOCAL_L2:
                out[s] += diffraction_pressure(I_lines[s], lines.eps_px[s])
        else:
            order = 1 if model == LOCAL_L1 else 2
            out[s] = local_forward(I_lines[s], phi_lines[s], lines.eps_px[s], order)
    return out


# ----------------------------------------------------------------------------------------------
# Entry points mirrored by the C ABI
# ----------------------------------------------------------------------------------------------

def _as64(a):
    return np.asarray(a, dtype=np.float64)


def forward(phase, absorb, lines, model):
    """Detector intensity of Eq. (5) for object maps at the reference energy:
    phi_s = phase_scale_s * phase, I_s = w_s exp(-absorb_scale_s * absorb)."""
    phase, absorb = _as64(phase), _as64(absorb)
    I = lines.w[:, None, None] * np.exp(-lines.absorb_scale[:, None, None] * absorb[None])
    phi = lines.phase_scale[:, None, None] * phase[None]
    return forward_lines(I, phi, lines, model).sum(axis=0)


def adjoint(phase, resid_lines, lines, model):
    """Per-line back-transport: identity for the local models, M_s^* (Eq. (4)) non-local."""
    phase, resid = _as64(phase), _as64(resid_lines)
    if model not in TRANSPORT_MODELS:
        return resid.copy()
    out = np.empty_like(resid)
    for s in range(resid.shape[0]):
        ux, uy = shift_field(lines.phase_scale[s] * phase, lines.eps_px[s])
        out[s] = gather(resid[s], ux, uy)
    return out


def precondition(in_lines, lines):
    """Per-line Paganin-type filter P_{1,s}^-1 (R3)."""
    x = _as64(in_lines)
    return np.stack([paganin_filter(x[s], lines.alpha_px[s]) for s in range(x.shape[0])])


def bin_image(x, f):
    """Detector integration on an oversampled internal grid (Section 3.2): a detector pixel of
    size p covers f x f internal pixels of size p / f and records their mean."""
    x = _as64(x)
    if f == 1:
        return x
    ny, nx = x.shape[-2] // f, x.shape[-1] // f
    return x.reshape(*x.shape[:-2], ny, f, nx, f).mean(axis=(-3, -1))


def replicate(x, f):
    """Right inverse of bin_image (bin_image(replicate(x)) = x): every detector value copied to
    its f x f internal pixels (reading R21)."""
    x = _as64(x)
    if f == 1:
        return x
    return np.repeat(np.repeat(x, f, axis=-2), f, axis=-1)


def forward_oversampled(phase, absorb, lines, model, f):
    """Detector intensity of maps given on an oversampled internal grid (Section 3.2): the
    forward model of Eq. (5) on the internal grid (lines taken at the internal pixel size p / f),
    then the detector integration bin_image."""
    return bin_image(forward(phase, absorb, lines, model), f)


def adjoint_oversampled(phase, resid_lines, lines, model, f):
    """Exact adjoint of forward_oversampled's per-line operators: the transpose of bin_image
    (every detector value copied to its f x f internal pixels and divided by f^2), then the
    per-line back-transport on the internal grid."""
    return adjoint(phase, replicate(resid_lines, f) / float(f * f), lines, model)


def forward_oversampled_vjp(phase, absorb, grad_intensity, lines, model, f):
    """Vector-Jacobian product of forward_oversampled: the transpose of bin_image (the detector
    gradient copied to its f x f internal pixels and divided by f^2), then forward_vjp on the
    internal grid.  Returns (dL/dphase, dL/dabsorb) on the internal grid."""
    g = replicate(grad_intensity, f) / float(f * f)
    return forward_vjp(phase, absorb, g, lines, model)


def iterate(tau, d, lines, model, relaxation, oversample=1):
    """One EPR iteration (Methods 4.4).  Returns (new tau, residual e).

    With oversample = f > 1 (Section 3.2, reading R21) tau and every per-line quantity live on
    the internal grid of f ny x f nx pixels of size p / f (`lines` built for that pixel), d on
    the detector grid: the line predictions are binned to the detector before the sum and the
    split, and the split residuals are replicated back to the internal grid."""
    I = line_intensities(tau, lines)
    phi = line_phases(tau, lines)
    P = forward_lines(I, phi, lines, model)
    e_s, e = split_residual(d, bin_image(P, oversample), lines.w)
    e_s = replicate(e_s, oversample)
    if model in TRANSPORT_MODELS:
        r = np.empty_like(e_s)
        for s in range(len(lines.w)):
            ux, uy = shift_field(phi[s], lines.eps_px[s])
            r[s] = gather(e_s[s], ux, uy)
    else:
        r = e_s
    dI = precondition(r, lines)
    return project_single_thickness(I + relaxation * dI, lines), e


def solve(d, lines, model, n_iter, relaxation, tau0=None, history=None, oversample=1):
    """EPR solve from tau0 (zero: R4).  Returns tau (float64, on the internal grid when
    oversampling).  If `history` is a list, the relative residual ||e|| / ||d|| of every
    iteration is appended to it."""
    d = _as64(d)
    shape = (d.shape[0] * oversample, d.shape[1] * oversample)
    tau = np.zeros(shape) if tau0 is None else _as64(tau0).copy()
    dn = np.linalg.norm(d)
    for _ in range(n_iter):
        tau, e = iterate(tau, d, lines, model, relaxation, oversample)
        if history is not None:
            history.append(float(np.linalg.norm(e) / dn))
    return tau


def _closure_vjp(I, ux, uy, eps2, G, order, transport=True):
    """Gradients of <G, P> with respect to I, u_x and u_y for the closure of Eq. (1) written
    with the shift field (local_forward_shift, order m = 1 or 2), or -- transport=False -- for
    its diffraction-pressure term alone.  The chain rule taken backwards through the terms as
    written there, with D^T the exact transpose of D:

      first order   P1 = I - (d_x(I u_x) + d_y(I u_y))
        dI   = G - (u_x k_x + u_y k_y),   k = D^T G
        du_x = -I k_x,                    du_y = -I k_y
      second order  P2 = 1/2 (d_x d_x(I u_x u_x) + d_x d_y(I u_x u_y) + d_y d_x(I u_y u_x)
                              + d_y d_y(I u_y u_y))
        with h_ab the transpose of d_a d_b applied to G:
        dI   += 1/2 (u_x^2 h_xx + u_x u_y (h_xy + h_yx) + u_y^2 h_yy)
        du_x += 1/2 I (2 u_x h_xx + u_y (h_xy + h_yx)),  du_y likewise
      pressure      P3 = -eps2/4 (d_x(I d_x Q) + d_y(I d_y Q)),  Q = lap(A) / A,  A = sqrt(I)
        (eps2 may vary across columns: it scales the term after its outer derivative, so the
        term's gradient is that of c = 1 for the weighted G' = eps2/4 G)
        dI   += -(d_x Q k'_x + d_y Q k'_y),   k' = D^T G'
        dQ    = -(D_x^T(I k'_x) + D_y^T(I k'_y))
        dA    = lap^T(dQ / A) - (dQ / A) Q,   dI += dA / (2 A)
    Returns (dI, du_x, du_y)."""
    dI = np.zeros_like(G)
    dux = np.zeros_like(G)
    duy = np.zeros_like(G)
    if transport:
        kx, ky = dx_transpose(G), dy_transpose(G)
        dI += G - (ux * kx + uy * ky)
        dux += -I * kx
        duy += -I * ky
        if order >= 2:
            hxx, hyy = dx_transpose(kx), dy_transpose(ky)
            hxy = dy_transpose(kx)   # transpose of d_x d_y
            hyx = dx_transpose(ky)   # transpose of d_y d_x
            dI += 0.5 * (ux * ux * hxx + ux * uy * (hxy + hyx) + uy * uy * hyy)
            dux += 0.5 * I * (2 * ux * hxx + uy * (hxy + hyx))
            duy += 0.5 * I * (ux * (hxy + hyx) + 2 * uy * hyy)
    if order >= 2 or not transport:
        Gc = 0.25 * eps2 * G
        kx, ky = dx_transpose(Gc), dy_transpose(Gc)
        A = np.sqrt(I)
        Q = (dx(dx(A)) + dy(dy(A))) / A
        dI += -(dx(Q) * kx + dy(Q) * ky)
        dQ = -(dx_transpose(I * kx) + dy_transpose(I * ky))
        t = dQ / A
        dA = dx_transpose(dx_transpose(t)) + dy_transpose(dy_transpose(t)) - t * Q
        dI += dA / (2 * A)
    return dI, dux, duy


def _local_line_vjp(I, phi, e, G, order, transport=True):
    """Gradients of <G, P> with respect to I and to phi for one line of the local closure
    P_{m,s} of Eq. (1) (local_forward with order m), or -- transport=False -- of its
    diffraction-pressure term alone (diffraction_pressure): _closure_vjp at u = e D phi and
    eps2 = e^2, then dphi = D_x^T(e du_x) + D_y^T(e du_y).  Returns (dI, dphi)."""
    dI, dux, duy = _closure_vjp(I, e * dx(phi), e * dy(phi), e * e, G, order, transport)
    return dI, dx_transpose(e * dux) + dy_transpose(e * duy)


def _transport_vjp(I, ux, uy, g):
    """Gradients of <g, M(u)[I]> (the splat after Eq. (3)) with respect to I, u_x and u_y:
    dI = M^* g (bilinear interpolation of g at the mapped points, Eq. 4) and
    du = I times the in-cell derivative of that interpolant (the splat is piecewise linear in u):
    in x (1-dy)(g10 - g00) + dy (g11 - g01), in y (1-dx)(g01 - g00) + dx (g11 - g10), g_ij the
    value at the paper's tap w_ij.  Returns (dI, du_x, du_y)."""
    ny, nx = g.shape
    x0, y0, fx, fy = _corners(ux, uy)

    def tap(oy, ox):
        ty, tx = y0 + oy, x0 + ox
        ok = (ty >= 0) & (ty < ny) & (tx >= 0) & (tx < nx)
        v = np.zeros((ny, nx))
        v[ok] = g[ty[ok], tx[ok]]
        return v

    g00, g10, g01, g11 = tap(0, 0), tap(0, 1), tap(1, 0), tap(1, 1)
    dI = (1 - fx) * (1 - fy) * g00 + fx * (1 - fy) * g10 + (1 - fx) * fy * g01 + fx * fy * g11
    dux = I * ((1 - fy) * (g10 - g00) + fy * (g11 - g01))
    duy = I * ((1 - fx) * (g01 - g00) + fx * (g11 - g10))
    return dI, dux, duy


def forward_vjp(phase, absorb, grad_intensity, lines, model=NONLOCAL):
    """Vector-Jacobian product of `forward` with respect to (phase, absorb), for every model.

    Local models: per line, the chain rule through the closure of Eq. (1) (_local_line_vjp),
    then I_s = w_s exp(-a_s A) and phi_s = b_s phase give g_A = sum_s -a_s I_s dI_s and
    g_phase = sum_s b_s dphi_s.  The second-order non-local model (R22) adds the pressure
    term's part to the transport's below.

    The non-local (transport) part:

    With P = sum_s M_s(u_s)[I_s], I_s = w_s exp(-a_s A), u_s = eps_s D(b_s phase):
      dL/dI_s = M_s^* g                         (linearity of Eq. (3) in I_s; Eq. (4))
      dL/du_s = I_s * grad_u [bilinear interpolation of g at x + u_s]
                (in x: (1-dy)(g10 - g00) + dy (g11 - g01); in y: (1-dx)(g01 - g00) + dx (g11 - g10),
                 g_ij the residual at the paper's tap w_ij)
      g_A     = sum_s -a_s I_s dL/dI_s
      g_phase = sum_s b_s eps_s (D_x^T dL/du_x + D_y^T dL/du_y)
    """
    phase, absorb, g = _as64(phase), _as64(absorb), _as64(grad_intensity)
    ny, nx = g.shape
    g_phase = np.zeros((ny, nx))
    g_abs = np.zeros((ny, nx))
    if model not in TRANSPORT_MODELS or model == NONLOCAL_L2:
        order = 1 if model == LOCAL_L1 else 2
        for s in range(len(lines.w)):
            a, b = lines.absorb_scale[s], lines.phase_scale[s]
            I = lines.w[s] * np.exp(-a * absorb)
            dI, dphi = _local_line_vjp(I, b * phase, lines.eps_px[s], g, order,
                                       transport=model not in TRANSPORT_MODELS)
            g_abs += -a * I * dI
            g_phase += b * dphi
        if model not in TRANSPORT_MODELS:
            return g_phase, g_abs
    for s in range(len(lines.w)):
        a, b = lines.absorb_scale[s], lines.phase_scale[s]
        I = lines.w[s] * np.exp(-a * absorb)
        ux, uy = shift_field(b * phase, lines.eps_px[s])
        gI, gux, guy = _transport_vjp(I, ux, uy, g)
        g_abs += -a * I * gI
        g_phase += b * lines.eps_px[s] * (dx_transpose(gux) + dy_transpose(guy))
    return g_phase, g_abs


# ----------------------------------------------------------------------------------------------
# Regime diagnostics (Section 2, "Eikonal transverse shift and local versus non-local regime";
# the per-line shift distributions of the bamboo stress test, Section 3.1)
# ----------------------------------------------------------------------------------------------

def shift_ratio_factors(lines):
    """|b_s| of eta_s = ||Delta_s|| / p = |b_s| ||D tau||: Delta_s = (L / k_s) grad phi_s with
    phi_s = -k_s delta_s tau, so in pixel units |b_s| = eps_px_s k_s delta_s = L delta_s / p^2."""
    return np.abs(lines.eps_px * lines.k * lines.delta)


def regime_histogram(tau, lines, n_bins, eta_max):
    """Per line s, the histogram over the image of the shift-to-pixel ratio eta_s (Section 2):
    n_bins bins of width eta_max / n_bins, then one bin for eta_s >= eta_max.  Shape
    (N_s, n_bins + 1), int64.

    A float decides each integer bin, so the decision is taken in float32, in the order the
    kernel uses (reading R19): g = sqrt(D_x tau * D_x tau + D_y tau * D_y tau) with every
    operation rounded (no fused multiply-add), eta = |b_s| g, bin = floor(eta * (n_bins /
    eta_max)) capped at n_bins."""
    t = np.asarray(tau, dtype=np.float32)
    gx = np.gradient(t, axis=1)
    gy = np.gradient(t, axis=0)
    g = np.sqrt(gx * gx + gy * gy)
    scale = np.float32(n_bins) / np.float32(eta_max)
    c = shift_ratio_factors(lines).astype(np.float32)
    out = np.zeros((len(c), n_bins + 1), dtype=np.int64)
    for s in range(len(c)):
        b = np.floor((c[s] * g) * scale)
        b = np.minimum(b, np.float32(n_bins)).astype(np.int64)
        out[s] = np.bincount(b.ravel(), minlength=n_bins + 1)
    return out


def select_model(d, lines, max_fraction=0.01):
    """Automatic local / non-local choice (Section 2: the local O(L^2) closure assumes eta < 1
    over most of the field of view; reading R20): the regime is measured on the Paganin
    retrieval of the data (one iteration from tau = 0 with relaxation 1, where every model
    coincides), and the local L^2 model is chosen when, for every line, at most max_fraction of
    the pixels have eta_s >= 1; otherwise the non-local model."""
    tau, _ = iterate(np.zeros_like(_as64(d)), _as64(d), lines, LOCAL_L1, 1.0)
    over = regime_histogram(tau, lines, 1, 1.0)[:, 1]
    return LOCAL_L2 if all(float(n) <= max_fraction * tau.size for n in over) else NONLOCAL


# ----------------------------------------------------------------------------------------------
# x-dependent effective spectrum (Methods 4.3, remark on spatially varying spectra, with the
# x-dependent db_s of Eq. (6); supplementary note on the spatially varying effective spectrum)
# ----------------------------------------------------------------------------------------------

def column_line_constants(block_x, block_energies_kev, block_weights, nx, pixel_m, distance_m,
                          delta_ref=1.0, beta_ref=1.0, energy_ref_kev=60.0, delta_exponent=2.0,
                          beta_exponent=3.0, oversample=1):
    """Per-column line constants of a spectrum tabulated on column blocks (R23).  Block b is
    centred on detector column block_x[b] (increasing) and gives every line an energy and a
    weight; column x takes, per line, the energy and the weight interpolated linearly between
    the two nearest block centres (held constant beyond the outer ones), and every constant
    follows from them as in line_constants.  Returns a Lines whose fields are [N_s][nx].
    With oversample = f the columns are those of the internal grid (f nx columns of pixel
    p / f); internal column j sits at detector coordinate (j + 1/2) / f - 1/2."""
    bx = np.asarray(block_x, dtype=np.float64)
    E = np.atleast_2d(np.asarray(block_energies_kev, dtype=np.float64))
    W = np.atleast_2d(np.asarray(block_weights, dtype=np.float64))
    f = oversample
    x = (np.arange(nx * f, dtype=np.float64) + 0.5) / f - 0.5 if f > 1 else np.arange(nx, dtype=np.float64)
    Ex = np.stack([np.interp(x, bx, E[:, s]) for s in range(E.shape[1])])
    Wx = np.stack([np.interp(x, bx, W[:, s]) for s in range(W.shape[1])])
    return line_constants(Ex, Wx, pixel_m / f, distance_m, delta_ref, beta_ref, energy_ref_kev,
                          delta_exponent, beta_exponent)


def local_forward_shift(I, ux, uy, eps2, order=2):
    """Eq. (1) written with the shift field u = eps D phi (pixels) instead of phi:
    P = I - d_i(I u_i) + 1/2 d_i d_j(I u_i u_j) - eps^2/4 d_i(I d_i Q).  eps2 may vary across
    columns (a row vector)."""
    P = I - (dx(I * ux) + dy(I * uy))
    if order >= 2:
        P = P + 0.5 * (dx(dx(I * ux * ux)) + dx(dy(I * ux * uy))
                       + dy(dx(I * uy * ux)) + dy(dy(I * uy * uy)))
        A = np.sqrt(I)
        Q = (dx(dx(A)) + dy(dy(A))) / A
        P = P - 0.25 * eps2 * (dx(I * dx(Q)) + dy(I * dy(Q)))
    return P


def column_shifts(tau, cl):
    """u_s = b_s(x) D tau with b_s = -eps_s k_s delta_s = -L delta_s / p^2 per column (R23: the
    refraction of a ray comes from the thickness gradient at its own effective energy; the slow
    variation of the spectrum across columns is not an object gradient)."""
    b = -cl.eps_px * cl.k * cl.delta
    gx, gy = dx(tau), dy(tau)
    return [(b[s] * gx, b[s] * gy) for s in range(b.shape[0])]


def _column_predictions(I, tau, cl, model):
    """Per-line predictions under per-column constants: the transport (plus, for the
    second-order model, the diffraction pressure with the column's eps) or the local closure."""
    shifts = column_shifts(tau, cl)
    P = np.empty_like(I)
    for s, (ux, uy) in enumerate(shifts):
        if model in TRANSPORT_MODELS:
            P[s] = splat(I[s], ux, uy)
            if model == NONLOCAL_L2:
                P[s] += diffraction_pressure(I[s], cl.eps_px[s])
        else:
            P[s] = local_forward_shift(I[s], ux, uy, cl.eps_px[s] ** 2,
                                       1 if model == LOCAL_L1 else 2)
    return P, shifts


def forward_columns(tau, cl, model, oversample=1):
    """Detector intensity of a single-material thickness map under a per-column spectrum:
    sum_s F_s[I_s], I_s = w_s(x) exp(-mu_s(x) tau) (binned to the detector when tau and cl are
    on an internal grid of factor `oversample`)."""
    tau = _as64(tau)
    I = cl.w[:, None, :] * np.exp(-cl.mu[:, None, :] * tau[None])
    P, _ = _column_predictions(I, tau, cl, model)
    return bin_image(P.sum(axis=0), oversample)


def adjoint_columns(tau, resid_lines, cl, model):
    """Per-line back-transport under a per-column spectrum: identity for the local models, the
    adjoint M_s^* of the splat (Eq. 4) at the column shifts of R23 for the transport models."""
    tau, r = _as64(tau), _as64(resid_lines)
    if model not in TRANSPORT_MODELS:
        return r.copy()
    return np.stack([gather(r[s], ux, uy) for s, (ux, uy) in enumerate(column_shifts(tau, cl))])


def forward_columns_vjp(tau, grad_intensity, cl, model):
    """dL/dtau of forward_columns (no oversampling) for g = dL/d(intensity): per line, the
    gradients with respect to I_s and u_s (_transport_vjp for the transport, plus the pressure
    term's for the second-order model; _closure_vjp for the local closures, with the column's
    eps^2), then I_s = w_s(x) exp(-mu_s(x) tau) and u_s = b_s(x) D tau give
    dL/dtau = sum_s -mu_s I_s dI_s + D_x^T(b_s du_x) + D_y^T(b_s du_y)."""
    tau, g = _as64(tau), _as64(grad_intensity)
    I = cl.w[:, None, :] * np.exp(-cl.mu[:, None, :] * tau[None])
    b = -cl.eps_px * cl.k * cl.delta
    gx, gy = dx(tau), dy(tau)
    out = np.zeros_like(tau)
    for s in range(I.shape[0]):
        ux, uy = b[s] * gx, b[s] * gy
        if model in TRANSPORT_MODELS:
            dI, dux, duy = _transport_vjp(I[s], ux, uy, g)
            if model == NONLOCAL_L2:
                dI = dI + _closure_vjp(I[s], ux, uy, cl.eps_px[s] ** 2, g, 2, transport=False)[0]
        else:
            dI, dux, duy = _closure_vjp(I[s], ux, uy, cl.eps_px[s] ** 2, g,
                                        1 if model == LOCAL_L1 else 2)
        out += -cl.mu[s] * I[s] * dI + dx_transpose(b[s] * dux) + dy_transpose(b[s] * duy)
    return out


def block_weights(block_x, nx, oversample=1):
    """lambda_b(x) of R24: the linear-interpolation weight of block centre b at each column
    (internal columns when oversampling, at the same coordinates as column_line_constants);
    [n_blocks][nx f], summing to 1 over the blocks."""
    bx = np.asarray(block_x, dtype=np.float64)
    f = oversample
    x = (np.arange(nx * f, dtype=np.float64) + 0.5) / f - 0.5 if f > 1 else np.arange(nx, dtype=np.float64)
    return np.stack([np.interp(x, bx, np.eye(len(bx))[b]) for b in range(len(bx))])


def block_alphas(block_energies_kev, pixel_m, distance_m, delta_ref=1.0, beta_ref=1.0,
                 energy_ref_kev=60.0, delta_exponent=2.0, beta_exponent=3.0, oversample=1):
    """alpha_s^(b) of R24: each line's preconditioner constant at block b's own energies
    (pixel p / f on an internal grid); [n_blocks][N_s]."""
    E = np.atleast_2d(np.asarray(block_energies_kev, dtype=np.float64))
    return np.stack([line_constants(E[b], np.full(E.shape[1], 1.0 / E.shape[1]),
                                    pixel_m / oversample, distance_m, delta_ref, beta_ref,
                                    energy_ref_kev, delta_exponent, beta_exponent).alpha_px
                     for b in range(E.shape[0])])


def blockwise_paganin(r, alphas, lam):
    """Block-wise interpolated preconditioner of one line (R24): sum_b lambda_b(x) times the
    Paganin filter of r at alpha^(b)."""
    out = np.zeros_like(_as64(r))
    for b in range(len(alphas)):
        out += lam[b][None, :] * paganin_filter(r, alphas[b])
    return out


def iterate_columns(tau, d, cl, model, relaxation, oversample=1, block=None):
    """One EPR iteration (Methods 4.4) with per-column line constants (R23): per-column I_s, shifts,
    split fallback weights and projection; the preconditioner of line s is the Paganin filter
    at the column mean of alpha_s (an FFT-diagonal approximate inverse; the fixed point does not
    depend on it).  With oversample = f (R21) tau and cl are on the internal grid: predictions
    are binned, the residual is split on the detector grid (fallback: the line's weight averaged
    over the detector column's f internal columns) and replicated back.  block = (alphas,
    lambdas) of R24 (block_alphas, block_weights) selects the block-wise interpolated
    preconditioner instead."""
    tau = _as64(tau)
    f = oversample
    I = cl.w[:, None, :] * np.exp(-cl.mu[:, None, :] * tau[None])
    P, shifts = _column_predictions(I, tau, cl, model)
    Pd = bin_image(P, f)
    e = _as64(d) - Pd.sum(axis=0)
    pos = np.maximum(Pd, 0.0)
    tot = pos.sum(axis=0)
    hole = tot <= 1e-30
    wd = cl.w.reshape(cl.w.shape[0], -1, f).mean(axis=2) if f > 1 else cl.w
    share = np.where(hole[None], wd[:, None, :], pos / np.where(hole, 1.0, tot))
    e_s = replicate(share * e[None], f)
    r = np.empty_like(e_s)
    for s, (ux, uy) in enumerate(shifts):
        r[s] = gather(e_s[s], ux, uy) if model in TRANSPORT_MODELS else e_s[s]
    if block is None:
        alpha = cl.alpha_px.mean(axis=1)
        dI = np.stack([paganin_filter(r[s], alpha[s]) for s in range(r.shape[0])])
    else:
        alphas, lam = block
        dI = np.stack([blockwise_paganin(r[s], alphas[:, s], lam) for s in range(r.shape[0])])
    w = cl.w[:, None, :]
    mu = cl.mu[:, None, :]
    J = np.maximum(I + relaxation * dI, 1e-6 * w)
    return -(w * mu * np.log(J / w)).sum(axis=0) / (cl.w * cl.mu ** 2).sum(axis=0)[None, :], e


def solve_columns(d, cl, model, n_iter, relaxation, tau0=None, history=None, oversample=1,
                  block=None):
    """EPR solve with a per-column spectrum (R23), from tau0 (zero: R4); block as in
    iterate_columns."""
    d = _as64(d)
    f = oversample
    tau = np.zeros((d.shape[0] * f, d.shape[1] * f)) if tau0 is None else _as64(tau0).copy()
    dn = np.linalg.norm(d)
    for _ in range(n_iter):
        tau, e = iterate_columns(tau, d, cl, model, relaxation, f, block)
        if history is not None:
            history.append(float(np.linalg.norm(e) / dn))
    return tau
