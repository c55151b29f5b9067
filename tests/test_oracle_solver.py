"""Pins of the FP64 oracle's solver and vector-Jacobian product: the textbook Paganin
retrieval, invariants of the iteration, inverse-crime recovery, the local/non-local limit and
finite differences."""

import numpy as np
import pytest

from oracle import epr_oracle as O
from synthetic import workload


def smooth_object(shape, seed, amp_phase, amp_abs):
    """Smooth random phase/absorption maps (sum of a few Gaussian blobs) with a flat margin."""
    r = np.random.default_rng(seed)
    ny, nx = shape
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    t = np.zeros(shape)
    for _ in range(5):
        cy, cx = r.uniform(0.3, 0.7) * ny, r.uniform(0.3, 0.7) * nx
        s = r.uniform(0.06, 0.12) * min(shape)
        t += r.uniform(0.5, 1.0) * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * s * s))
    t /= t.max()
    return -amp_phase * t, amp_abs * t


def textbook_paganin(d, pixel_m, distance_m, delta, mu):
    """Single-distance phase retrieval of a homogeneous object (Paganin et al. 2002), written
    in physical frequencies:  T = -(1/mu) ln F^-1[ mu F[d] / (mu + delta L 4 pi^2 |f|^2) ]."""
    ny, nx = d.shape
    fy = np.fft.fftfreq(ny, d=pixel_m)[:, None]
    fx = np.fft.fftfreq(nx, d=pixel_m)[None, :]
    filt = mu / (mu + delta * distance_m * 4 * np.pi ** 2 * (fx ** 2 + fy ** 2))
    return -np.log(np.real(np.fft.ifft2(np.fft.fft2(d) * filt))) / mu


@pytest.mark.parametrize("model", O.MODELS)
def test_first_iteration_is_textbook_paganin(model):
    # from tau = 0 every line is flat and unshifted, so the first update is the Paganin filter
    n, p, dist = 96, 2e-6, 0.3
    L = O.line_constants([30.0], [1.0], p, dist, delta_ref=1e-6, beta_ref=2e-9)
    r = np.random.default_rng(1)
    d = 1.0 + 0.05 * r.standard_normal((n, n))
    tau = O.solve(d, L, model, 1, 1.0)
    ref = textbook_paganin(d, p, dist, L.delta[0], L.mu[0])
    assert np.linalg.norm(tau - ref) / np.linalg.norm(ref) < 1e-11


def test_first_iteration_recovers_homogeneous_sphere():
    # linear (first-order) data of a homogeneous sphere: one iteration returns the analytic chord
    n, p, dist = 128, 1e-6, 0.5
    L = O.line_constants([60.0], [1.0], p, dist, delta_ref=4e-7, beta_ref=4e-10)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    T = 2 * np.sqrt(np.maximum(30.0 ** 2 - (x - 64.0) ** 2 - (y - 63.0) ** 2, 0)) * p
    I = np.exp(-L.mu[0] * T)
    # linearised propagation of a homogeneous object: (1 - (delta L / mu) lap) I, spectrally
    fy = np.fft.fftfreq(n, d=p)[:, None]
    fx = np.fft.fftfreq(n, d=p)[None, :]
    lap = -4 * np.pi ** 2 * (fx ** 2 + fy ** 2)
    d = np.real(np.fft.ifft2(np.fft.fft2(I) * (1 - L.delta[0] * dist / L.mu[0] * lap)))
    tau = O.solve(d, L, O.LOCAL_L1, 1, 1.0)
    assert np.linalg.norm(tau - T) / np.linalg.norm(T) < 1e-12


def _poly_setup(shape=(48, 56), seed=3):
    L = O.line_constants([66.25, 91.25, 141.25], [0.5, 0.3, 0.2], 1e-5, 20.0, 4e-7, 4e-10)
    phase, absorb = smooth_object(shape, seed, 300.0, 0.8)
    d = O.forward(phase, absorb, L, O.NONLOCAL)
    return L, d


def test_splitting_a_line_leaves_the_trajectory_unchanged():
    L, d = _poly_setup()
    Ls = O.line_constants([66.25, 91.25, 91.25, 141.25], [0.5, 0.15, 0.15, 0.2], 1e-5, 20.0,
                          4e-7, 4e-10)
    for model in (O.NONLOCAL, O.LOCAL_L2):
        t1 = O.solve(d, L, model, 3, 0.4)
        t2 = O.solve(d, Ls, model, 3, 0.4)
        assert np.linalg.norm(t1 - t2) / np.linalg.norm(t1) < 1e-12


def test_identical_lines_equal_mono():
    L1 = O.line_constants([80.0], [1.0], 1e-5, 20.0, 4e-7, 4e-10)
    L3 = O.line_constants([80.0, 80.0, 80.0], [0.2, 0.3, 0.5], 1e-5, 20.0, 4e-7, 4e-10)
    phase, absorb = smooth_object((40, 40), 4, 200.0, 0.5)
    d = O.forward(phase, absorb, L1, O.NONLOCAL)
    assert np.allclose(O.forward(phase, absorb, L3, O.NONLOCAL), d, rtol=1e-13)
    t1 = O.solve(d, L1, O.NONLOCAL, 3, 0.4)
    t3 = O.solve(d, L3, O.NONLOCAL, 3, 0.4)
    assert np.linalg.norm(t1 - t3) / np.linalg.norm(t1) < 1e-12


def test_resume_is_bit_exact():
    L, d = _poly_setup()
    t20 = O.solve(d, L, O.NONLOCAL, 6, 0.4)
    t10 = O.solve(d, L, O.NONLOCAL, 3, 0.4)
    assert np.array_equal(O.solve(d, L, O.NONLOCAL, 3, 0.4, tau0=t10), t20)


def test_split_sums_to_residual_inside_iteration():
    L, d = _poly_setup()
    tau = O.solve(d, L, O.NONLOCAL, 2, 0.4)
    I = O.line_intensities(tau, L)
    P = O.forward_lines(I, O.line_phases(tau, L), L, O.NONLOCAL)
    es, e = O.split_residual(d, P, L.w)
    assert np.allclose(es.sum(0), e, atol=1e-15)


def test_local_inverse_crime_recovers_thickness():
    # noise-free local second-order data of a single-material object with sub-pixel shifts
    w = workload("local-mono-256")
    obj = w.true_object()
    L = O.line_constants(w.energies_kev, w.weights, w.pixel_m, w.distance_m, w.delta_ref,
                         w.beta_ref, w.energy_ref_kev, w.delta_exponent, w.beta_exponent)
    d = O.forward(obj["phase"], obj["absorb"], L, O.LOCAL_L2)
    tau_true = obj["tau_soft"]
    hist = []
    tau = O.solve(d, L, O.LOCAL_L2, w.n_iter, w.relaxation, history=hist)
    # object maps are float32 inputs: compare with the thickness they encode
    tau_enc = obj["absorb"].astype(np.float64) / L.mu[0]
    err = np.linalg.norm(tau - tau_enc) / np.linalg.norm(tau_enc)
    assert err < 1e-4
    assert hist[-1] < 1e-6 and hist[0] > hist[-1]
    assert np.linalg.norm(tau_enc - tau_true) / np.linalg.norm(tau_true) < 1e-6


def test_nonlocal_residual_decreases_on_inverse_crime():
    L = O.line_constants([60.0], [1.0], 1e-5, 20.0, 4e-7, 4e-10)
    n = 96
    _, absorb = smooth_object((n, n), 5, 0.0, 1.0)
    tau_true = 1.0e-3 * absorb
    phase = -L.k[0] * L.delta[0] * tau_true
    d = O.forward(phase, L.mu[0] * tau_true, L, O.NONLOCAL)
    ux, uy = O.shift_field(phase, L.eps_px[0])
    assert 1.0 < np.hypot(ux, uy).max() < 6.0
    hist = []
    O.solve(d, L, O.NONLOCAL, 12, 0.4, history=hist)
    assert all(b < a for a, b in zip(hist, hist[1:]))
    assert hist[-1] < 0.5 * hist[0]


def test_local_and_nonlocal_agree_to_first_order_in_distance():
    # ||P_nonlocal - P_local|| / ||P_local|| shrinks linearly with L (slope 1 on a log scale)
    # once the shifts are sub-pixel (0.17 px down to 0.02 px here); the ratio to the transport
    # term itself stays bounded: the splat is an upwind discretisation of the same transport
    phase, absorb = smooth_object((64, 64), 6, 40.0, 0.3)
    diffs = []
    for dist in (1.0, 0.5, 0.25, 0.125):
        L = O.line_constants([60.0], [1.0], 1e-5, dist, 4e-7, 4e-10)
        pn = O.forward(phase, absorb, L, O.NONLOCAL)
        pl = O.forward(phase, absorb, L, O.LOCAL_L2)
        diffs.append(np.linalg.norm(pn - pl) / np.linalg.norm(pl))
    slopes = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
    assert np.all(np.abs(slopes - 1.0) < 0.1)


def test_vjp_matches_central_differences():
    L = O.line_constants([66.25, 103.75], [0.6, 0.4], 1e-5, 20.0, 4e-7, 4e-10)
    n = 40
    phase, absorb = smooth_object((n, n), 7, 150.0, 0.6)
    r = np.random.default_rng(8)
    g = r.standard_normal((n, n))
    gp, ga = O.forward_vjp(phase, absorb, g, L)

    def loss(ph, ab):
        return np.vdot(g, O.forward(ph, ab, L, O.NONLOCAL))

    checked = 0
    for _ in range(40):
        j, i = r.integers(8, n - 8, size=2)
        # absorption enters smoothly: O(h^2) central difference
        h = 1e-5
        e = np.zeros((n, n))
        e[j, i] = h
        fd = (loss(phase, absorb + e) - loss(phase, absorb - e)) / (2 * h)
        assert fd == pytest.approx(ga[j, i], rel=1e-6, abs=1e-9)
        # phase enters piecewise linearly: skip the rare points where a kink is crossed
        hp = 1e-6
        e[j, i] = hp
        l0 = loss(phase, absorb)
        fwd = (loss(phase + e, absorb) - l0) / hp
        bwd = (l0 - loss(phase - e, absorb)) / hp
        if abs(fwd - bwd) > 1e-6 * max(1.0, abs(fwd)):
            continue
        assert 0.5 * (fwd + bwd) == pytest.approx(gp[j, i], rel=1e-6, abs=1e-8)
        checked += 1
    assert checked >= 30
