"""Pins of the oracle's second-order non-local model: the ray-map transport M_s of Eq. (3) plus
the diffraction-pressure (WKB1) term of Eq. (1), evaluated from I_s on the object grid."""

import numpy as np

from oracle import epr_oracle as O


def _gauss(n, sigma, c):
    y, x = np.mgrid[0:n, 0:n].astype(float)
    r2 = (x - c[1]) ** 2 + (y - c[0]) ** 2
    return x, y, r2, np.exp(-r2 / sigma ** 2)


def _lines(eps_px):
    # one line whose eps / p^2 equals eps_px: L / (k p^2) = eps_px with p = 1 um
    L = O.line_constants([40.0], [1.0], 1e-6, 1.0, 1e-6, 1e-9)
    L.eps_px = np.array([eps_px])
    return L


def test_zero_phase_reduces_to_the_local_second_order_closure():
    # phi = 0: the ray map is the identity and the local transport terms vanish, so both
    # second-order models are I plus the same diffraction-pressure term
    _, _, _, I = _gauss(64, 9.0, (30.3, 33.8))
    I = 0.2 + I
    L = _lines(0.7)
    phi = np.zeros((1,) + I.shape)
    a = O.forward_lines(I[None], phi, L, O.NONLOCAL_L2)
    b = O.forward_lines(I[None], phi, L, O.LOCAL_L2)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


def test_integer_shift_of_a_gaussian_is_translation_plus_the_closed_form_wkb1():
    # phi = a x + b y with eps (a, b) = (2, -1) px: the splat translates exactly (zero fill),
    # and the WKB1 term of I = exp(-r^2/s^2) is -(eps^2/s^4)(1 - r^2/s^2) exp(-r^2/s^2)
    n, sigma, eps = 200, 30.0, 1.0
    c = (100.4, 99.7)
    x, y, r2, I = _gauss(n, sigma, c)
    a, b = 2.0, -1.0
    L = _lines(eps)
    P = O.forward_lines(I[None], (a * x + b * y)[None], L, O.NONLOCAL_L2)[0]
    shifted = np.exp(-((x - a - c[1]) ** 2 + (y - b - c[0]) ** 2) / sigma ** 2)
    wkb1 = -(eps ** 2 / sigma ** 4) * (1 - r2 / sigma ** 2) * np.exp(-r2 / sigma ** 2)
    inner = (slice(6, -6), slice(6, -6))
    # O(h^2) stencil error of the WKB1 term only (~1e-7 here); a wrong sign or factor of the
    # term (its peak is 1.2e-6) or a dropped transport fails
    assert np.abs((P - shifted - wkb1)[inner]).max() < 5e-8
    assert np.abs(wkb1).max() > 1e-6


def test_uniform_intensity_has_no_diffraction_pressure():
    # Q = lap(sqrt I) / sqrt I vanishes for uniform I: the model is the pure transport
    n = 64
    y, x = np.mgrid[0:n, 0:n].astype(float)
    phi = 0.02 * ((x - 31.5) ** 2 + (y - 30.2) ** 2)
    I = np.full((n, n), 0.8)
    L = _lines(0.9)
    a = O.forward_lines(I[None], phi[None], L, O.NONLOCAL_L2)
    b = O.forward_lines(I[None], phi[None], L, O.NONLOCAL)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


def test_the_added_term_is_second_order_in_distance():
    _, _, _, I = _gauss(64, 7.0, (31.2, 32.9))
    I = 0.3 + I
    y, x = np.mgrid[0:64, 0:64].astype(float)
    phi = 0.3 * np.sin(x / 9.0) * np.cos(y / 11.0)
    diffs = []
    for eps in (0.8, 0.4):
        L = _lines(eps)
        d = (O.forward_lines(I[None], phi[None], L, O.NONLOCAL_L2)
             - O.forward_lines(I[None], phi[None], L, O.NONLOCAL))
        diffs.append(np.linalg.norm(d))
    assert abs(diffs[0] / diffs[1] - 4.0) < 1e-9


def test_second_order_nonlocal_inverse_crime():
    # a strongly absorbing object (delta / beta = 10, I down to 0.09) where the diffraction
    # pressure is a few per cent of the transport's change: data made by the second-order
    # non-local model are inverted more accurately by that model than by the pure transport
    n = 64
    L = O.line_constants([35.0, 55.0], [0.5, 0.5], 1e-6, 0.5, 1e-6, 1e-7)
    _, _, _, g = _gauss(n, 4.0, (31.4, 32.2))
    truth = 1e-5 * g
    I, phi = O.line_intensities(truth, L), O.line_phases(truth, L)
    d = O.forward_lines(I, phi, L, O.NONLOCAL_L2).sum(axis=0)
    err = {}
    for m in (O.NONLOCAL_L2, O.NONLOCAL):
        h = []
        t = O.solve(d, L, m, 20, 0.4, history=h)
        assert h[-1] < 0.15 * h[0]
        err[m] = np.linalg.norm(t - truth) / np.linalg.norm(truth)
    assert err[O.NONLOCAL_L2] < 0.9 * err[O.NONLOCAL]
