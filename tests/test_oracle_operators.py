"""Pins of the FP64 oracle's operators against facts that do not depend on the oracle itself:
exactness of finite differences on polynomials, library routines, brute-force transposes,
conservation, and closed forms of the method's special cases."""

import numpy as np
import pytest
from scipy.ndimage import map_coordinates

from oracle import epr_oracle as O


def rng(seed=0):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------------------------
# Per-line constants (Eq. S8, Methods 4.3)
# --------------------------------------------------------------------------------------------

def test_wavelength_and_pixel_constants_textbook():
    # textbook: lambda[Angstrom] = 12.3984 / E[keV]
    L = O.line_constants([60.0], [1.0], pixel_m=5e-6, distance_m=1.0, delta_ref=5e-7,
                         beta_ref=5e-10)
    lam = 2 * np.pi / L.k[0]
    assert lam == pytest.approx(12.39841984e-10 / 60.0, rel=1e-12)
    # eps = lambda L / (2 pi), in pixel^2 units
    assert L.eps_px[0] == pytest.approx(lam * 1.0 / (2 * np.pi) / 25e-12, rel=1e-12)
    assert L.eps_px[0] == pytest.approx(0.131551, rel=1e-5)
    # attenuation coefficient mu = 4 pi beta / lambda
    assert L.mu[0] == pytest.approx(4 * np.pi * 5e-10 / lam, rel=1e-12)
    # Paganin coefficient delta L / (mu p^2)
    assert L.alpha_px[0] == pytest.approx(5e-7 * 1.0 / (L.mu[0] * 25e-12), rel=1e-12)


def test_power_law_scales():
    L = O.line_constants([60.0, 120.0], [0.5, 0.5], 1e-5, 1.0, 4e-7, 4e-10, energy_ref_kev=60.0)
    assert L.delta[1] == pytest.approx(4e-7 / 4, rel=1e-14)
    assert L.beta[1] == pytest.approx(4e-10 / 8, rel=1e-14)
    # phase ~ k delta ~ E^-1 ; absorption ~ k beta ~ E^-2
    assert L.phase_scale[1] == pytest.approx(0.5, rel=1e-14)
    assert L.absorb_scale[1] == pytest.approx(0.25, rel=1e-14)
    assert L.phase_scale[0] == pytest.approx(1.0, rel=1e-14)


# --------------------------------------------------------------------------------------------
# Derivative operator (R1)
# --------------------------------------------------------------------------------------------

def test_D_exact_on_planes_including_edges():
    y, x = np.mgrid[0:7, 0:9].astype(float)
    f = 0.3 * x - 1.7 * y + 2.0
    assert np.array_equal(O.dx(f), np.full(f.shape, 0.3)) or np.allclose(O.dx(f), 0.3, atol=1e-14)
    assert np.allclose(O.dy(f), -1.7, atol=1e-14)


def test_D_exact_on_quadratics_inside():
    y, x = np.mgrid[0:8, 0:10].astype(float)
    f = x ** 2 + 3 * x * y - y ** 2
    assert np.allclose(O.dx(f)[:, 1:-1], (2 * x + 3 * y)[:, 1:-1], atol=1e-12)
    assert np.allclose(O.dy(f)[1:-1, :], (3 * x - 2 * y)[1:-1, :], atol=1e-12)


def test_D_matrix_and_transpose_brute_force():
    r = rng(1)
    f = r.standard_normal((6, 11))
    g = r.standard_normal((6, 11))
    assert np.allclose(O.gradient_matrix(11) @ f[0], O.dx(f)[0], atol=1e-14)
    # <D f, g> = <f, D^T g> for both axes
    assert np.vdot(O.dx(f), g) == pytest.approx(np.vdot(f, O.dx_transpose(g)), rel=1e-13)
    assert np.vdot(O.dy(f), g) == pytest.approx(np.vdot(f, O.dy_transpose(g)), rel=1e-13)


# --------------------------------------------------------------------------------------------
# Splat (display after Eq. (3)) and its adjoint (Eq. (4))
# --------------------------------------------------------------------------------------------

def test_splat_zero_shift_is_identity_bit_exact():
    I = rng(2).random((13, 17))
    z = np.zeros_like(I)
    assert np.array_equal(O.splat(I, z, z), I)


def test_splat_conserves_mass_when_on_grid():
    r = rng(3)
    ny, nx = 40, 50
    I = r.random((ny, nx))
    ux = r.uniform(-3, 3, (ny, nx))
    uy = r.uniform(-3, 3, (ny, nx))
    # keep every target inside by zeroing the intensity of sources near the border
    I[:4] = I[-5:] = 0
    I[:, :4] = I[:, -5:] = 0
    P = O.splat(I, ux, uy)
    assert P.sum() == pytest.approx(I.sum(), rel=1e-14)


def test_splat_integer_shift_is_zero_filled_roll():
    I = rng(4).random((12, 15))
    ux = np.full(I.shape, 2.0)
    uy = np.full(I.shape, -3.0)
    expect = np.zeros_like(I)
    expect[0:12 - 3, 2:15] = I[3:12, 0:13]
    assert np.array_equal(O.splat(I, ux, uy), expect)


def _shift_zero_fill(a, sy, sx):
    """Array moved by (+sy, +sx) pixels with zero fill (sy, sx in {0, 1})."""
    out = np.zeros_like(a)
    out[sy:, sx:] = a[:a.shape[0] - sy, :a.shape[1] - sx]
    return out


def test_splat_fractional_constant_shift_is_donor_cell_update():
    # a constant shift (a, b) in [0,1)^2 is the corner-transport upwind (donor-cell) update
    I = rng(5).random((10, 14))
    a, b = 0.3, 0.65
    P = O.splat(I, np.full(I.shape, a), np.full(I.shape, b))
    expect = ((1 - a) * (1 - b) * I + a * (1 - b) * _shift_zero_fill(I, 0, 1)
              + (1 - a) * b * _shift_zero_fill(I, 1, 0) + a * b * _shift_zero_fill(I, 1, 1))
    assert np.allclose(P, expect, rtol=0, atol=1e-15)


def test_splat_negative_fractional_shift_uses_floor():
    # u = -0.25 lands between x-1 and x, a quarter pixel from x: 0.75 of the mass stays at x
    I = np.zeros((3, 5))
    I[1, 2] = 1.0
    P = O.splat(I, np.full(I.shape, -0.25), np.zeros(I.shape))
    assert P[1, 1] == pytest.approx(0.25, abs=1e-15)
    assert P[1, 2] == pytest.approx(0.75, abs=1e-15)
    assert P.sum() == pytest.approx(1.0, abs=1e-15)


def test_gather_is_scipy_bilinear_interpolation():
    r = rng(6)
    ny, nx = 23, 31
    e = r.standard_normal((ny, nx))
    ux = r.uniform(-4, 4, (ny, nx))
    uy = r.uniform(-4, 4, (ny, nx))
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    ref = map_coordinates(e, [y + uy, x + ux], order=1, mode="grid-constant", cval=0.0)
    assert np.allclose(O.gather(e, ux, uy), ref, rtol=0, atol=1e-13)


def test_gather_is_dense_transpose_of_splat():
    r = rng(7)
    ny, nx = 7, 9
    ux = r.uniform(-2.5, 2.5, (ny, nx))
    uy = r.uniform(-2.5, 2.5, (ny, nx))
    n = ny * nx
    M = np.zeros((n, n))
    Mstar = np.zeros((n, n))
    for j in range(n):
        ej = np.zeros(n)
        ej[j] = 1.0
        M[:, j] = O.splat(ej.reshape(ny, nx), ux, uy).ravel()
        Mstar[:, j] = O.gather(ej.reshape(ny, nx), ux, uy).ravel()
    assert np.allclose(Mstar, M.T, rtol=0, atol=1e-15)


def test_adjoint_identity_1e12():
    r = rng(8)
    ny, nx = 64, 80
    ux = r.uniform(-6, 6, (ny, nx))
    uy = r.uniform(-6, 6, (ny, nx))
    a = r.standard_normal((ny, nx))
    b = r.standard_normal((ny, nx))
    lhs = np.vdot(O.splat(a, ux, uy), b)
    rhs = np.vdot(a, O.gather(b, ux, uy))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# --------------------------------------------------------------------------------------------
# Local closure (Eq. (1))
# --------------------------------------------------------------------------------------------

def test_local_uniform_flat_is_identity():
    I = np.full((16, 16), 0.7)
    z = np.zeros_like(I)
    for order in (1, 2):
        assert np.allclose(O.local_forward(I, z, 0.4, order), I, rtol=0, atol=1e-15)


def test_local_thin_lens_closed_form():
    # phi = a (x^2 + y^2) / 2 gives u = eps a (x, y): first-order term -2 eps a, second-order
    # 3 eps^2 a^2 (uniform I: Q = 0); exact transport I / (1 + eps a)^2 agrees to O(eps^2).
    ny, nx = 32, 36
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    a, eps = 0.05, 0.7
    phi = a * ((x - 17.3) ** 2 + (y - 15.1) ** 2) / 2
    I = np.ones((ny, nx))
    inner = (slice(3, -3), slice(3, -3))
    P1 = O.local_forward(I, phi, eps, 1)
    P2 = O.local_forward(I, phi, eps, 2)
    assert np.allclose(P1[inner], 1 - 2 * eps * a, rtol=0, atol=1e-13)
    assert np.allclose(P2[inner], 1 - 2 * eps * a + 3 * (eps * a) ** 2, rtol=0, atol=1e-13)


def _gauss(shape, sigma, c):
    y, x = np.mgrid[0:shape[0], 0:shape[1]].astype(float)
    r2 = (x - c[1]) ** 2 + (y - c[0]) ** 2
    return r2, np.exp(-r2 / sigma ** 2)


def test_local_diffraction_pressure_gaussian_converges_second_order():
    # I = exp(-r^2/s^2), phi = 0: only the WKB1 term survives,
    #   -(eps^2/4) div(I grad Q) = -(eps^2 / s^4) (1 - r^2/s^2) exp(-r^2/s^2)
    eps = 0.5
    errs = []
    for sigma in (4.0, 8.0, 16.0):
        n = int(12 * sigma)
        r2, I = _gauss((n, n), sigma, (n / 2 + 0.3, n / 2 - 0.2))
        P = O.local_forward(I, np.zeros_like(I), eps, 2)
        exact = -(eps ** 2 / sigma ** 4) * (1 - r2 / sigma ** 2) * np.exp(-r2 / sigma ** 2)
        inner = (slice(5, -5), slice(5, -5))
        errs.append(np.linalg.norm((P - I - exact)[inner]) / np.linalg.norm(exact[inner]))
    assert errs[0] < 0.25
    assert errs[1] / errs[2] > 3.5 and errs[0] / errs[1] > 3.5


@pytest.mark.parametrize("order", [1, 2])
def test_local_constant_shift_matches_translated_intensity(order):
    # phi = a x + b y is a uniform shift v = eps (a, b): the closure is the Taylor series of the
    # translated intensity I(x - v) to order m, plus (m = 2) the Gaussian WKB1 term above.
    n, sigma = 240, 30.0
    c = (120.4, 119.7)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    eps, a, b = 1.0, 0.5, -0.36  # v = (0.5, -0.36) px
    vx, vy = eps * a, eps * b
    I = np.exp(-((x - c[1]) ** 2 + (y - c[0]) ** 2) / sigma ** 2)
    P = O.local_forward(I, a * x + b * y, eps, order)
    r2s = (x - vx - c[1]) ** 2 + (y - vy - c[0]) ** 2
    shifted = np.exp(-r2s / sigma ** 2)
    r2 = (x - c[1]) ** 2 + (y - c[0]) ** 2
    wkb1 = -(eps ** 2 / sigma ** 4) * (1 - r2 / sigma ** 2) * np.exp(-r2 / sigma ** 2)
    inner = (slice(6, -6), slice(6, -6))
    if order == 2:
        # O(v^3/sigma^3) and O(h^2) residuals (~1e-5); a dropped 1/2 or cross term gives >1.5e-4
        err = np.abs((P - shifted - wkb1)[inner]).max()
        assert err < 3e-5
    else:
        # first order leaves the O(v^2) term out
        err = np.abs((P - shifted)[inner]).max()
        assert 1e-4 < err < 2e-3


# --------------------------------------------------------------------------------------------
# Preconditioner (Section 2, linear term)
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(24, 40), (25, 30), (16, 16)])
def test_paganin_scales_each_cosine_by_the_symbol(shape):
    ny, nx = shape
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    alpha = 3.7
    for m, k in [(0, 0), (1, 0), (0, 3), (2, 5), (ny // 2, nx // 2), (ny // 2 - 1, 1)]:
        r = np.cos(2 * np.pi * (k * x / nx + m * y / ny))
        fy, fx = m / ny, k / nx
        out = O.paganin_filter(r, alpha)
        assert np.allclose(out, r / (1 + 4 * np.pi ** 2 * alpha * (fx ** 2 + fy ** 2)),
                           rtol=0, atol=1e-13)


def test_paganin_homogeneous_sphere_round_trip():
    # spectral L1 data of a homogeneous sphere: the filter returns the attenuation exactly and
    # -ln / mu gives the analytic chord 2 sqrt(R^2 - r^2)
    n, p = 128, 1e-6
    L = O.line_constants([60.0], [1.0], p, 0.5, delta_ref=4e-7, beta_ref=4e-10)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    R = 30.0
    r2 = (x - 64.0) ** 2 + (y - 63.0) ** 2
    T = 2 * np.sqrt(np.maximum(R ** 2 - r2, 0)) * p
    I = np.exp(-L.mu[0] * T)
    fy = np.fft.fftfreq(n)[:, None]
    fx = np.fft.rfftfreq(n)[None, :]
    data = np.fft.irfft2(np.fft.rfft2(I) * (1 + 4 * np.pi ** 2 * L.alpha_px[0] * (fx ** 2 + fy ** 2)),
                         s=(n, n))
    Trec = -np.log(O.paganin_filter(data, L.alpha_px[0])) / L.mu[0]
    assert np.linalg.norm(Trec - T) / np.linalg.norm(T) < 1e-12


def test_paganin_preserves_mean():
    r = rng(9).random((20, 26))
    assert O.paganin_filter(r, 5.0).mean() == pytest.approx(r.mean(), rel=1e-14)


# --------------------------------------------------------------------------------------------
# Residual split (R7) and projection (R8)
# --------------------------------------------------------------------------------------------

def test_split_sums_to_residual_and_is_proportional():
    r = rng(10)
    P = r.random((3, 8, 9))
    d = r.random((8, 9)) * 3
    w = np.array([0.5, 0.3, 0.2])
    es, e = O.split_residual(d, P, w)
    assert np.allclose(es.sum(0), e, atol=1e-15)
    assert np.allclose(e, d - P.sum(0))
    assert np.allclose(es[1] / es[0], P[1] / P[0], rtol=1e-12)


def test_split_negative_and_hole_fallback():
    P = np.zeros((2, 2, 2))
    P[0, 0, 0] = -1.0     # negative prediction takes no share
    P[1, 0, 0] = 2.0
    d = np.ones((2, 2))
    w = np.array([0.25, 0.75])
    es, e = O.split_residual(d, P, w)
    assert es[0, 0, 0] == 0.0 and es[1, 0, 0] == pytest.approx(e[0, 0])
    # (1,1): every line is zero -> split by the spectral weights
    assert es[0, 1, 1] == pytest.approx(0.25 * e[1, 1]) and es[1, 1, 1] == pytest.approx(0.75)


def test_projection_idempotent_on_single_thickness():
    L = O.line_constants([66.25, 90.0, 140.0], [0.5, 0.3, 0.2], 1e-5, 20.0, 4e-7, 4e-10)
    tau = rng(11).uniform(0, 5e-3, (9, 7))
    I = O.line_intensities(tau, L)
    assert np.allclose(O.project_single_thickness(I, L), tau, rtol=1e-13, atol=0)


def test_projection_floor():
    L = O.line_constants([60.0], [1.0], 1e-5, 20.0, 4e-7, 4e-10)
    I = np.array([[[-0.5, 0.0]]])
    tau = O.project_single_thickness(I, L)
    assert np.allclose(tau, -np.log(1e-6) / L.mu[0], rtol=1e-14)


# --------------------------------------------------------------------------------------------
# Forward / adjoint entry points
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("model", O.MODELS)
def test_forward_flat_object_is_spectral_sum_of_weights(model):
    L = O.line_constants([66.0, 100.0], [0.6, 0.4], 1e-5, 20.0, 4e-7, 4e-10)
    z = np.zeros((12, 10))
    assert np.allclose(O.forward(z, z, L, model), 1.0, atol=1e-15)


def test_forward_absorption_only_is_beer_lambert():
    L = O.line_constants([66.0, 100.0], [0.6, 0.4], 1e-5, 20.0, 4e-7, 4e-10)
    A = rng(12).uniform(0, 2, (9, 11))
    for model in (O.LOCAL_L1, O.NONLOCAL):   # (L2 adds the diffraction-pressure term)
        P = O.forward(np.zeros_like(A), A, L, model)
        expect = 0.6 * np.exp(-A * L.absorb_scale[0]) + 0.4 * np.exp(-A * L.absorb_scale[1])
        assert np.allclose(P, expect, rtol=1e-14)


def test_adjoint_local_is_identity_and_nonlocal_transposes_forward():
    L = O.line_constants([66.0, 100.0], [0.6, 0.4], 1e-5, 20.0, 4e-7, 4e-10)
    r = rng(13)
    phase = 40 * r.standard_normal((20, 24))
    res = r.standard_normal((2, 20, 24))
    assert np.array_equal(O.adjoint(phase, res, L, O.LOCAL_L2), res)
    # per-line duality: <M_s x, y_s> = <x, M_s^* y_s>
    adj = O.adjoint(phase, res, L, O.NONLOCAL)
    x = r.standard_normal((20, 24))
    for s in range(2):
        ux, uy = O.shift_field(L.phase_scale[s] * phase, L.eps_px[s])
        lhs = np.vdot(O.splat(x, ux, uy), res[s])
        assert lhs == pytest.approx(np.vdot(x, adj[s]), rel=1e-12)
