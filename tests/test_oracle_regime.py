"""Pins of the oracle's regime diagnostics (the shift-to-pixel ratio eta of Section 2 and its
per-line distribution, Section 3.1) and of the automatic local / non-local choice, plus the
strong-shift stress test: beyond one pixel of shift the local second-order closure diverges
while the non-local transport stays stable (Section 3.1)."""

import math

import numpy as np
import pytest

from oracle import epr_oracle as O
from synthetic import workload
from tests.helpers import oracle_lines


def physical_eta(lines_spec, grad_px):
    """eta_s = ||Delta_s|| / p from the definitions alone: Delta_s = (L / k_s) grad phi_s with
    phi_s = -k_s delta_s tau, so ||Delta_s|| = L delta_s ||grad tau||; with the thickness
    gradient given per pixel (metres per pixel), ||grad tau|| = grad_px / p."""
    e, dist, p, d_ref, e_ref, d_exp = lines_spec
    delta = d_ref * (e_ref / np.asarray(e, dtype=np.float64)) ** d_exp
    return dist * delta * (grad_px / p) / p


def _fibre_spec():
    w = workload("fibres-stress-256")
    return w, oracle_lines(w), (w.energies_kev, w.distance_m, w.pixel_m, w.delta_ref,
                                w.energy_ref_kev, w.delta_exponent)


def _expected_bins(eta, n_bins, eta_max):
    v = np.asarray(eta) * (n_bins / eta_max)
    frac = v - np.floor(v)
    # the fixture must keep every value well inside a bin so fp32 and fp64 agree on it
    assert np.all((frac > 1e-5) & (frac < 1 - 1e-5)), v
    return np.minimum(np.floor(v), n_bins).astype(int)


def test_zero_thickness_falls_in_the_first_bin():
    _, L, _ = _fibre_spec()
    h = O.regime_histogram(np.zeros((24, 40)), L, 16, 2.0)
    assert h.shape == (10, 17)
    assert np.all(h[:, 0] == 24 * 40) and np.all(h[:, 1:] == 0)


@pytest.mark.parametrize("direction", ["x", "y", "diagonal"])
def test_uniform_ramp_lands_in_the_bin_of_its_physical_shift(direction):
    # tau = c x (or c y, or c (x + y)) with c a power of two: every sample and every difference
    # is exact in float32, so D tau = c on every pixel, edges included
    _, L, spec = _fibre_spec()
    ny, nx = 48, 64
    c = 2.0 ** -14
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    tau = {"x": c * x, "y": c * y, "diagonal": c * (x + y)}[direction]
    grad = c * (math.sqrt(2.0) if direction == "diagonal" else 1.0)
    n_bins, eta_max = 64, 2.0
    want = _expected_bins(physical_eta(spec, grad), n_bins, eta_max)
    h = O.regime_histogram(tau, L, n_bins, eta_max)
    for s in range(len(want)):
        assert h[s, want[s]] == ny * nx, (s, want[s], np.nonzero(h[s])[0])
    # lower energies refract more: the bins never decrease towards lower energy
    assert np.all(np.diff(want) <= 0)


def test_shifts_beyond_the_range_go_to_the_overflow_bin():
    _, L, spec = _fibre_spec()
    c = 2.0 ** -10  # eta ~ 11 .. 3 px
    tau = c * np.arange(32, dtype=np.float64)[None, :].repeat(8, axis=0)
    assert physical_eta(spec, c).min() > 2.0
    h = O.regime_histogram(tau, L, 8, 2.0)
    assert np.all(h[:, 8] == tau.size) and np.all(h[:, :8] == 0)


def test_histogram_matches_brute_force_on_a_tiny_field():
    # per-pixel loops in float64 from the definition of D (central inside, one-sided edges)
    _, L, spec = _fibre_spec()
    r = np.random.default_rng(11)
    ny, nx = 7, 9
    tau = (r.uniform(0.0, 2e-4, (ny, nx))).astype(np.float32).astype(np.float64)
    n_bins, eta_max = 12, 3.0

    def diff(f, i, n):
        if i == 0:
            return f(1) - f(0)
        if i == n - 1:
            return f(n - 1) - f(n - 2)
        return 0.5 * (f(i + 1) - f(i - 1))

    want = np.zeros((len(L.w), n_bins + 1), dtype=np.int64)
    for yy in range(ny):
        for xx in range(nx):
            gx = diff(lambda j: tau[yy, j], xx, nx)
            gy = diff(lambda j: tau[j, xx], yy, ny)
            b = _expected_bins(physical_eta(spec, math.hypot(gx, gy)), n_bins, eta_max)
            for s in range(len(b)):
                want[s, b[s]] += 1
    np.testing.assert_array_equal(O.regime_histogram(tau, L, n_bins, eta_max), want)


def test_every_pixel_is_counted_once_per_line():
    w, L, _ = _fibre_spec()
    tau = w.true_object()["tau_soft"]
    h = O.regime_histogram(tau, L, 32, 4.0)
    assert np.all(h.sum(axis=1) == tau.size)
    # a stress object: for the lowest line a large part of the field is beyond one pixel
    frac_over = h[0, 8:].sum() / tau.size
    assert frac_over > 0.3


def test_selection_follows_the_shift_regime():
    weak = workload("local-mono-256", shape=(128, 128))
    Lw = oracle_lines(weak)
    ow = weak.true_object()
    dw = O.forward(ow["phase"], ow["absorb"], Lw, O.LOCAL_L2)
    assert O.select_model(dw, Lw) == O.LOCAL_L2

    w, L, _ = _fibre_spec()
    o = w.true_object()
    d = O.forward(o["phase"], o["absorb"], L, O.NONLOCAL)
    assert O.select_model(d, L) == O.NONLOCAL
    # the threshold is on the worst line's fraction of pixels with eta >= 1
    tau1 = O.solve(d, L, O.LOCAL_L1, 1, 1.0)
    worst = O.regime_histogram(tau1, L, 1, 1.0)[:, 1].max() / d.size
    assert 0.0 < worst < 1.0
    assert O.select_model(d, L, max_fraction=worst) == O.LOCAL_L2
    assert O.select_model(d, L, max_fraction=worst * 0.999) == O.NONLOCAL


def test_strong_shifts_make_the_local_closure_diverge_but_not_the_transport():
    w = workload("fibres-stress-256", shape=(128, 256))
    L = oracle_lines(w)
    o = w.true_object()
    truth = o["tau_soft"]
    d = O.forward(o["phase"], o["absorb"], L, O.NONLOCAL)

    def errors(model, n):
        tau, out = None, []
        for _ in range(n):
            tau = O.solve(d, L, model, 1, w.relaxation, tau0=tau)
            out.append(np.linalg.norm(tau - truth) / np.linalg.norm(truth))
        return np.array(out)

    loc = errors(O.LOCAL_L2, 10)
    nl = errors(O.NONLOCAL, 10)
    assert loc[-1] > 3.0 * loc.min() and loc[-1] > 1.0          # diverges
    assert np.all(np.diff(nl) <= 1e-9) and nl[-1] < 0.3          # stable, converging
