"""Pins of the oracle's oversampled iteration (Section 3.2: the solvers run on an internal grid
finer than the detector by a factor 2 or 4).  The detector pixel integrates its f x f internal
pixels; the residual returns to the internal grid by replication."""

import numpy as np
import pytest

from oracle import epr_oracle as O
from tests.test_oracle_solver import textbook_paganin


def test_binning_inverts_replication_and_averages_blocks():
    r = np.random.default_rng(2)
    x = r.standard_normal((3, 5, 7))
    for f in (1, 2, 4):
        np.testing.assert_array_equal(O.bin_image(O.replicate(x, f), f), x)
    # a detector pixel records the mean of its f x f internal pixels
    fine = np.arange(4 * 6, dtype=float).reshape(4, 6)
    want = np.array([[(0 + 1 + 6 + 7) / 4, (2 + 3 + 8 + 9) / 4, (4 + 5 + 10 + 11) / 4],
                     [(12 + 13 + 18 + 19) / 4, (14 + 15 + 20 + 21) / 4, (16 + 17 + 22 + 23) / 4]])
    np.testing.assert_array_equal(O.bin_image(fine, 2), want)


@pytest.mark.parametrize("f", [2, 4])
@pytest.mark.parametrize("model", O.MODELS)
def test_first_oversampled_iteration_is_paganin_of_the_replicated_data(model, f):
    # from tau = 0 the lines are flat and unshifted, so the update is the Paganin filter at the
    # internal pixel size applied to the detector image copied onto the internal grid
    n, p, dist = 24, 2e-6, 0.3
    L = O.line_constants([30.0], [1.0], p / f, dist, delta_ref=1e-6, beta_ref=2e-9)
    r = np.random.default_rng(1)
    d = 1.0 + 0.05 * r.standard_normal((n, n + 8))
    tau = O.solve(d, L, model, 1, 1.0, oversample=f)
    assert tau.shape == (f * n, f * (n + 8))
    ref = textbook_paganin(np.kron(d, np.ones((f, f))), p / f, dist, L.delta[0], L.mu[0])
    assert np.linalg.norm(tau - ref) / np.linalg.norm(ref) < 1e-11


def test_factor_one_is_the_plain_iteration():
    r = np.random.default_rng(4)
    L = O.line_constants([40.0, 70.0], [0.6, 0.4], 3e-6, 2.0, 1e-6, 1e-9)
    d = 1.0 + 0.03 * r.standard_normal((20, 26))
    tau = 1e-5 * r.random((20, 26))
    a, ea = O.iterate(tau, d, L, O.NONLOCAL, 0.4)
    b, eb = O.iterate(tau, d, L, O.NONLOCAL, 0.4, oversample=1)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ea, eb)


def _blob(n, f, centre=(24.1, 23.3), sigma=6.0):
    """A Gaussian sampled at the centres of the internal pixels of an n x n detector."""
    c = (np.arange(n * f) + 0.5) / f - 0.5
    y, x = np.meshgrid(c, c, indexing="ij")
    return np.exp(-((x - centre[1]) ** 2 + (y - centre[0]) ** 2) / (2 * sigma * sigma))


def test_oversampling_removes_the_splat_quantisation():
    # at small distance the binned transport and the binned first-order closure differ by the
    # splat's discretisation only, which falls in proportion to the internal pixel size
    n, p, dist = 48, 2e-6, 0.01
    ratio = []
    for f in (1, 2, 4):
        L = O.line_constants([40.0], [1.0], p / f, dist, 1e-6, 1e-9)
        tau = 2e-5 * _blob(n, f)
        I, phi = O.line_intensities(tau, L), O.line_phases(tau, L)
        pn = O.bin_image(O.forward_lines(I, phi, L, O.NONLOCAL), f)
        pl = O.bin_image(O.forward_lines(I, phi, L, O.LOCAL_L1), f)
        ratio.append(np.linalg.norm(pn - pl) / np.linalg.norm(pl - O.bin_image(I, f)))
    assert ratio[0] > 0.2
    assert 0.45 < ratio[1] / ratio[0] < 0.65 and 0.45 < ratio[2] / ratio[1] < 0.65


def test_oversampled_local_inverse_crime():
    # data made by the local L2 model on the internal grid and binned to the detector: the
    # oversampled solve drives the detector residual down and recovers the binned thickness
    n, p, dist, f = 40, 2e-6, 0.4, 2
    L = O.line_constants([35.0, 50.0], [0.5, 0.5], p / f, dist, 1e-6, 2e-9)
    truth = 1.5e-5 * _blob(n, f, (19.6, 20.2), 5.0)
    I, phi = O.line_intensities(truth, L), O.line_phases(truth, L)
    d = O.bin_image(O.forward_lines(I, phi, L, O.LOCAL_L2).sum(axis=0), f)
    hist = []
    tau = O.solve(d, L, O.LOCAL_L2, 12, 1.0, history=hist, oversample=f)
    assert hist[-1] < 1e-3 * hist[0]
    tb, ref = O.bin_image(tau, f), O.bin_image(truth, f)
    assert np.linalg.norm(tb - ref) / np.linalg.norm(ref) < 0.01


def test_oversampled_forward_and_adjoint_are_transposes():
    # <bin(M_s I), r> = <I, M_s^* (B^T r)> per line at f = 2 and 4, shifts of a few pixels, and
    # f = 1 reduces to the plain operators
    rng = np.random.default_rng(31)
    for f in (1, 2, 4):
        L = O.line_constants([40.0, 70.0], [0.6, 0.4], 2e-6 / f, 0.5, 4e-7, 4e-10)
        n = 12 * f
        y, x = np.mgrid[0:n, 0:n].astype(float)
        phase = -40.0 * f * np.exp(-((x - n / 2) ** 2 + (y - n / 2) ** 2) / (2 * (2.5 * f) ** 2))
        r = rng.standard_normal((2, 12, 12))
        back = O.adjoint_oversampled(phase, r, L, O.NONLOCAL, f)
        for s in range(2):
            ux, uy = O.shift_field(L.phase_scale[s] * phase, L.eps_px[s])
            if f > 1:
                assert np.abs(ux).max() > 1.0
            I = rng.uniform(0.5, 1.5, (n, n))
            lhs = np.vdot(O.bin_image(O.splat(I, ux, uy), f), r[s])
            assert lhs == pytest.approx(np.vdot(I, back[s]), rel=1e-12)
        if f == 1:
            absorb = 0.1 * np.abs(phase) / 40.0
            np.testing.assert_array_equal(O.forward_oversampled(phase, absorb, L, O.NONLOCAL, 1),
                                          O.forward(phase, absorb, L, O.NONLOCAL))


def test_oversampled_forward_of_flat_maps_is_flat():
    L = O.line_constants([40.0, 70.0], [0.6, 0.4], 1e-6, 0.5, 4e-7, 4e-10)
    for model in (O.NONLOCAL, O.LOCAL_L2):
        out = O.forward_oversampled(np.zeros((24, 24)), np.full((24, 24), 0.3), L, model, 4)
        assert out.shape == (6, 6)
        np.testing.assert_allclose(out, np.sum(L.w * np.exp(-0.3 * L.absorb_scale)), rtol=1e-14)


def _vjp_case(f, seed=5):
    from tests.test_oracle_vjp import setup
    n, m = 5, 6
    phase, absorb, _ = setup((n * f, m * f), seed)
    g = np.random.default_rng(seed + 7).standard_normal((n, m))
    L = O.line_constants([22.0, 31.0], [0.55, 0.45], 1e-6 / f, 0.5, 4e-7, 4e-10)
    return phase, absorb, g, L


@pytest.mark.parametrize("model", [O.LOCAL_L1, O.LOCAL_L2])
@pytest.mark.parametrize("f", [2, 4])
def test_oversampled_vjp_matches_central_differences_everywhere(model, f):
    from tests.test_oracle_vjp import fd_gradient
    phase, absorb, g, L = _vjp_case(f)
    gp, ga = O.forward_oversampled_vjp(phase, absorb, g, L, model, f)
    assert gp.shape == phase.shape and ga.shape == absorb.shape
    fp = fd_gradient(lambda ph: np.vdot(g, O.forward_oversampled(ph, absorb, L, model, f)), phase, 1e-5)
    fa = fd_gradient(lambda ab: np.vdot(g, O.forward_oversampled(phase, ab, L, model, f)), absorb, 1e-5)
    np.testing.assert_allclose(gp, fp, rtol=1e-6, atol=1e-7 * np.abs(fp).max())
    np.testing.assert_allclose(ga, fa, rtol=1e-6, atol=1e-7 * np.abs(fa).max())


def test_oversampled_nonlocal_vjp_matches_central_differences_off_kinks():
    f = 2
    phase, absorb, g, L = _vjp_case(f, seed=9)
    gp, ga = O.forward_oversampled_vjp(phase, absorb, g, L, O.NONLOCAL, f)

    def loss(ph, ab):
        return np.vdot(g, O.forward_oversampled(ph, ab, L, O.NONLOCAL, f))

    l0, h, checked = loss(phase, absorb), 1e-7, 0
    for idx in np.ndindex(phase.shape):
        e = np.zeros_like(phase)
        e[idx] = h
        fwd, bwd = (loss(phase + e, absorb) - l0) / h, (l0 - loss(phase - e, absorb)) / h
        if abs(fwd - bwd) > 1e-4 * max(1.0, abs(fwd)):
            continue
        assert 0.5 * (fwd + bwd) == pytest.approx(gp[idx], rel=1e-4, abs=1e-6 * np.abs(gp).max())
        # absorption enters smoothly: central differences everywhere
        fa = (loss(phase, absorb + e) - loss(phase, absorb - e)) / (2 * h)
        assert fa == pytest.approx(ga[idx], rel=1e-4, abs=1e-6 * np.abs(ga).max())
        checked += 1
    assert checked >= phase.size // 2


def test_oversampled_vjp_at_factor_one_is_the_plain_vjp():
    phase, absorb, _, L = _vjp_case(1)
    g = np.random.default_rng(3).standard_normal(phase.shape)
    for model in O.MODELS:
        a = O.forward_oversampled_vjp(phase, absorb, g, L, model, 1)
        b = O.forward_vjp(phase, absorb, g, L, model)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
