"""Pins of the oracle's x-dependent effective spectrum: per-line energies and weights tabulated
on column blocks and interpolated linearly across the detector (Methods 4.3 remark and the
supplementary note on spatially varying spectra)."""

import numpy as np
import pytest

from oracle import epr_oracle as O

P, DIST = 2e-6, 0.4
MAT = (1e-6, 2e-9)


def _profile(nx):
    # harder (higher-energy) lines in the middle of the field, as behind a cylindrical container
    bx = [0.0, nx / 2.0, nx - 1.0]
    E = [[30.0, 45.0, 60.0], [34.0, 50.0, 66.0], [30.0, 45.0, 60.0]]
    W = [[0.5, 0.3, 0.2], [0.3, 0.4, 0.3], [0.5, 0.3, 0.2]]
    return bx, E, W


def _blob(n, m, sigma, c, amp):
    y, x = np.mgrid[0:n, 0:m].astype(float)
    return amp * np.exp(-((x - c[1]) ** 2 + (y - c[0]) ** 2) / (2 * sigma ** 2))


def test_constants_at_block_centres_and_halfway():
    nx = 41
    bx, E, W = [0.0, 20.0, 40.0], [[30.0, 50.0], [40.0, 70.0], [30.0, 50.0]], \
        [[0.6, 0.4], [0.2, 0.8], [0.6, 0.4]]
    cl = O.column_line_constants(bx, E, W, nx, P, DIST, *MAT)
    for b, x in enumerate((0, 20, 40)):
        ref = O.line_constants(E[b], W[b], P, DIST, *MAT)
        for f in ("w", "k", "delta", "beta", "mu", "eps_px", "alpha_px"):
            np.testing.assert_allclose(getattr(cl, f)[:, x], getattr(ref, f), rtol=1e-14)
    # halfway between centres 0 and 20 the energies and weights are the averages
    ref = O.line_constants([35.0, 60.0], [0.4, 0.6], P, DIST, *MAT)
    np.testing.assert_allclose(cl.k[:, 10], ref.k, rtol=1e-14)
    np.testing.assert_allclose(cl.w[:, 10], ref.w, rtol=1e-14)
    np.testing.assert_allclose(cl.w.sum(axis=0), 1.0, rtol=1e-14)


def test_uniform_profile_reduces_to_the_uniform_solver():
    n = 48
    E, W = [35.0, 55.0], [0.55, 0.45]
    cl = O.column_line_constants([5.0, 30.0], [E, E], [W, W], n, P, DIST, *MAT)
    L = O.line_constants(E, W, P, DIST, *MAT)
    tau_true = _blob(n, n, 6.0, (23.5, 24.2), 2e-5)
    for model in O.MODELS:
        phase = O.line_phases(tau_true, L)[0] / L.phase_scale[0]   # maps at the reference
        absorb = tau_true * L.mu[0] / L.absorb_scale[0]
        d = O.forward(phase, absorb, L, model)
        a = O.solve(d, L, model, 4, 0.5)
        b = O.solve_columns(d, cl, model, 4, 0.5)
        assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-12, model


def test_first_iteration_closed_form():
    # from tau = 0: I_s = w_s(x), no shift, P = 1, e_s = w_s(x) (d - 1), and the update is
    # tau = -sum_s w mu ln(1 + omega F_s[w_s (d - 1)] / w_s) / sum_s w mu^2 with F_s the Paganin
    # filter at the column mean of alpha_s
    ny, nx, om = 24, 40, 0.7
    bx, E, W = _profile(nx)
    cl = O.column_line_constants(bx, E, W, nx, P, DIST, *MAT)
    r = np.random.default_rng(6)
    d = 1.0 + 0.03 * r.standard_normal((ny, nx))
    fy = np.fft.fftfreq(ny)[:, None]
    fx = np.fft.rfftfreq(nx)[None, :]
    num = np.zeros((ny, nx))
    for s in range(3):
        a = cl.alpha_px[s].mean()
        H = 1.0 / (1.0 + 4 * np.pi ** 2 * a * (fx ** 2 + fy ** 2))
        dI = np.fft.irfft2(np.fft.rfft2(cl.w[s] * (d - 1.0)) * H, s=(ny, nx))
        num += cl.w[s] * cl.mu[s] * np.log(1.0 + om * dI / cl.w[s])
    want = -num / (cl.w * cl.mu ** 2).sum(axis=0)
    # (the second-order closure adds the diffraction pressure of the weight profile itself)
    for model in (O.LOCAL_L1, O.NONLOCAL):
        got, _ = O.iterate_columns(np.zeros((ny, nx)), d, cl, model, om)
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-12, model


@pytest.mark.parametrize("model", [O.NONLOCAL, O.LOCAL_L2])
def test_profile_matters_for_recovery(model):
    # data made under the x-dependent spectrum: its own model recovers the thickness better
    # than the uniform model with the column-averaged spectrum
    ny, nx = 48, 64
    bx, E, W = _profile(nx)
    cl = O.column_line_constants(bx, E, W, nx, P, DIST, *MAT)
    truth = _blob(ny, nx, 6.0, (24.2, 20.3), 2.5e-5) + _blob(ny, nx, 5.0, (22.0, 44.1), 2e-5)
    d = O.forward_columns(truth, cl, model)
    tx = O.solve_columns(d, cl, model, 12, 0.6)
    Lm = O.line_constants(np.mean(E, axis=0), np.mean(W, axis=0), P, DIST, *MAT)
    tu = O.solve(d, Lm, model, 12, 0.6)
    ex = np.linalg.norm(tx - truth) / np.linalg.norm(truth)
    eu = np.linalg.norm(tu - truth) / np.linalg.norm(truth)
    assert ex < 0.01 and ex < 0.1 * eu, (ex, eu)


def test_internal_columns_sit_at_their_detector_coordinates():
    # oversampling by f: internal column j is centred at detector coordinate (j + 1/2) / f - 1/2
    bx, E, W = [0.0, 10.0], [[30.0, 50.0], [40.0, 70.0]], [[0.6, 0.4], [0.2, 0.8]]
    cl = O.column_line_constants(bx, E, W, 12, P, DIST, *MAT, oversample=2)
    assert cl.w.shape == (2, 24)
    for j in (0, 1, 5, 20, 23):
        xd = (j + 0.5) / 2 - 0.5
        ek = [np.interp(xd, bx, [E[0][s], E[1][s]]) for s in range(2)]
        wk = [np.interp(xd, bx, [W[0][s], W[1][s]]) for s in range(2)]
        ref = O.line_constants(ek, wk, P / 2, DIST, *MAT)
        np.testing.assert_allclose(cl.k[:, j], ref.k, rtol=1e-14)
        np.testing.assert_allclose(cl.w[:, j], ref.w, rtol=1e-14)
        np.testing.assert_allclose(cl.eps_px[:, j], ref.eps_px, rtol=1e-14)


@pytest.mark.parametrize("model,f", [(O.NONLOCAL, 2), (O.LOCAL_L2, 2), (O.NONLOCAL_L2, 1),
                                     (O.NONLOCAL_L2, 2)])
def test_uniform_profile_reduces_to_the_uniform_solver_in_every_mode(model, f):
    n = 32
    E, W = [35.0, 55.0], [0.55, 0.45]
    cl = O.column_line_constants([5.0, 20.0], [E, E], [W, W], n, P, DIST, *MAT, oversample=f)
    L = O.line_constants(E, W, P / f, DIST, *MAT)
    r = np.random.default_rng(8)
    d = 1.0 + 0.03 * r.standard_normal((n, n))
    a = O.solve(d, L, model, 3, 0.5, oversample=f)
    b = O.solve_columns(d, cl, model, 3, 0.5, oversample=f)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-12


def test_first_oversampled_iteration_closed_form():
    # from tau = 0 and no shift: P_s = w_s(x) on the internal grid, the binned sum is 1, the
    # split gives each detector pixel the share wd_s (the line weight averaged over its f
    # internal columns), replicated; the update follows as in the non-oversampled closed form
    ny, nx, f, om = 12, 20, 2, 0.7
    bx, E, W = _profile(nx)
    cl = O.column_line_constants(bx, E, W, nx, P, DIST, *MAT, oversample=f)
    r = np.random.default_rng(6)
    d = 1.0 + 0.03 * r.standard_normal((ny, nx))
    wd = cl.w.reshape(3, nx, f).mean(axis=2)
    fy = np.fft.fftfreq(ny * f)[:, None]
    fx = np.fft.rfftfreq(nx * f)[None, :]
    num = np.zeros((ny * f, nx * f))
    for s in range(3):
        H = 1.0 / (1.0 + 4 * np.pi ** 2 * cl.alpha_px[s].mean() * (fx ** 2 + fy ** 2))
        rs = np.kron(wd[s][None, :] * (d - 1.0), np.ones((f, f)))
        dI = np.fft.irfft2(np.fft.rfft2(rs) * H, s=rs.shape)
        num += cl.w[s] * cl.mu[s] * np.log(1.0 + om * dI / cl.w[s])
    want = -num / (cl.w * cl.mu ** 2).sum(axis=0)
    for model in (O.LOCAL_L1, O.NONLOCAL):
        got, _ = O.iterate_columns(np.zeros((ny * f, nx * f)), d, cl, model, om, oversample=f)
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-12, model


# ---- block-wise interpolated preconditioner (R24) -------------------------------------------

def test_block_weights_are_the_spectrum_interpolation():
    nx = 50
    bx = [3.0, 20.0, 41.5]
    lam = O.block_weights(bx, nx)
    np.testing.assert_allclose(lam.sum(axis=0), 1.0, rtol=0, atol=1e-15)
    assert (lam >= 0).all()
    # blending the block energies with lambda reproduces the per-column energy interpolation
    E = np.array([[30.0, 50.0], [40.0, 70.0], [35.0, 55.0]])
    cl = O.column_line_constants(bx, E, np.full((3, 2), 0.5), nx, P, DIST, *MAT)
    E_blend = lam.T @ E
    k_blend = 2 * np.pi * E_blend.T * 1e3 / O.HC_EV_M
    np.testing.assert_allclose(k_blend, cl.k, rtol=1e-14)
    # one at its own centre (column 20), constant beyond the outer centres
    np.testing.assert_allclose(lam[:, 20], [0.0, 1.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(lam[:, :4], np.array([[1.0], [0.0], [0.0]]) * np.ones(4), atol=1e-15)
    np.testing.assert_allclose(lam[:, 42:], np.array([[0.0], [0.0], [1.0]]) * np.ones(8), atol=1e-15)
    # oversampled: the internal columns' coordinates, as the constants use them
    lam2 = O.block_weights(bx, nx, oversample=2)
    x2 = (np.arange(2 * nx) + 0.5) / 2 - 0.5
    np.testing.assert_allclose(lam2[1], np.interp(x2, bx, [0.0, 1.0, 0.0]), atol=1e-15)


def test_block_alphas_are_the_line_constants_at_the_block_energies():
    E = [[30.0, 45.0, 60.0], [34.0, 50.0, 66.0]]
    a = O.block_alphas(E, P, DIST, *MAT)
    for b in range(2):
        L = O.line_constants(E[b], [0.2, 0.3, 0.5], P, DIST, *MAT)
        np.testing.assert_allclose(a[b], L.alpha_px, rtol=1e-15)
    # on an internal grid the pixel is p / f: alpha ~ 1 / p^2
    np.testing.assert_allclose(O.block_alphas(E, P, DIST, *MAT, oversample=2), 4 * a, rtol=1e-14)


def test_blockwise_filter_of_identical_blocks_is_the_paganin_filter():
    r = np.random.default_rng(4).standard_normal((24, 40))
    lam = O.block_weights([0.0, 13.0, 39.0], 40)
    out = O.blockwise_paganin(r, np.array([7.5, 7.5, 7.5]), lam)
    np.testing.assert_allclose(out, O.paganin_filter(r, 7.5), rtol=0, atol=1e-13)


@pytest.mark.parametrize("a,b", [(0, 0), (3, 0), (0, 5), (2, 7), (11, 19)])
def test_blockwise_filter_of_a_cosine_closed_form(a, b):
    # a single Fourier mode is an eigenfunction of every block's filter, so column x of the
    # output is the mode times sum_b lambda_b(x) / (1 + 4 pi^2 alpha_b ((a/ny)^2 + (b/nx)^2))
    ny, nx = 32, 48
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    r = np.cos(2 * np.pi * (a * y / ny + b * x / nx) + 0.3)
    alphas = np.array([2.0, 40.0, 9.0])
    lam = O.block_weights([4.0, 24.0, 40.0], nx)
    f2 = (a / ny) ** 2 + (b / nx) ** 2
    gain = (lam / (1 + 4 * np.pi ** 2 * alphas[:, None] * f2)).sum(axis=0)
    np.testing.assert_allclose(O.blockwise_paganin(r, alphas, lam), gain[None, :] * r,
                               rtol=0, atol=1e-13)


def test_blockwise_solver_reaches_the_same_fixed_point():
    # the preconditioner only scales the update; the fixed point P(tau) = d of the iteration
    # does not depend on it.  beta ~ E^-4 makes alpha ~ E vary between the blocks (with the
    # default exponents alpha is energy-independent and both preconditioners coincide); strong
    # absorption and a short distance make the iteration converge within 100 steps.
    n, m = 24, 32
    mat, dist, nb = (1e-6, 1e-7), 0.1, 4.0
    bx, E, W = [0.0, m / 2.0, m - 1.0], [[30.0, 45.0], [50.0, 75.0], [31.0, 47.0]], \
        [[0.6, 0.4], [0.45, 0.55], [0.55, 0.45]]
    cl = O.column_line_constants(bx, E, W, m, P, dist, *mat, beta_exponent=nb)
    tau_true = _blob(n, m, 4.0, (11.5, 15.2), 1.5e-5)
    d = O.forward_columns(tau_true, cl, O.LOCAL_L1)
    block = (O.block_alphas(E, P, dist, *mat, beta_exponent=nb), O.block_weights(bx, m))
    assert np.ptp(block[0][:, 0]) > 0.5 * block[0][:, 0].min()   # alphas differ by block
    h_mean, h_block = [], []
    a = O.solve_columns(d, cl, O.LOCAL_L1, 100, 1.0, history=h_mean)
    b = O.solve_columns(d, cl, O.LOCAL_L1, 100, 1.0, history=h_block, block=block)
    assert abs(h_mean[10] - h_block[10]) > 0.1 * h_mean[10]       # different trajectories
    assert h_mean[-1] < 1e-9 and h_block[-1] < 1e-9
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-7
    assert np.linalg.norm(a - tau_true) / np.linalg.norm(tau_true) < 1e-8


def test_column_adjoint_is_the_transpose_of_the_column_transport():
    # <M_s[I], r> = <I, M_s^* r> per line at the column shifts (brute force over the pinned
    # splat), and the local models' back-transport is the identity
    n, m = 20, 26
    bx, E, W = _profile(m)
    cl = O.column_line_constants(bx, E, W, m, P, DIST, *MAT)
    tau = _blob(n, m, 4.0, (9.5, 12.2), 4e-4)
    r = np.random.default_rng(3).standard_normal((len(W[0]), n, m))
    I = np.random.default_rng(4).uniform(0.5, 1.5, (n, m))
    back = O.adjoint_columns(tau, r, cl, O.NONLOCAL)
    shifts = O.column_shifts(tau, cl)
    assert max(np.abs(ux).max() for ux, _ in shifts) > 1.5   # shifts cross several cells
    for s, (ux, uy) in enumerate(shifts):
        lhs = np.vdot(O.splat(I, ux, uy), r[s])
        assert lhs == pytest.approx(np.vdot(I, back[s]), rel=1e-12)
    np.testing.assert_array_equal(O.adjoint_columns(tau, r, cl, O.LOCAL_L2), r)


def test_uniform_profile_column_adjoint_is_the_uniform_adjoint():
    n = 24
    E, W = [35.0, 55.0], [0.55, 0.45]
    cl = O.column_line_constants([5.0, 18.0], [E, E], [W, W], n, P, DIST, *MAT)
    L = O.line_constants(E, W, P, DIST, *MAT)
    tau = _blob(n, n, 4.0, (11.5, 12.2), 4e-4)
    phase = O.line_phases(tau, L)[0] / L.phase_scale[0]
    r = np.random.default_rng(5).standard_normal((2, n, n))
    np.testing.assert_allclose(O.adjoint_columns(tau, r, cl, O.NONLOCAL),
                               O.adjoint(phase, r, L, O.NONLOCAL), rtol=1e-12, atol=1e-12)
    # and the column forward model is the uniform one
    absorb = tau * L.mu[0] / L.absorb_scale[0]
    for model in (O.NONLOCAL, O.NONLOCAL_L2, O.LOCAL_L1, O.LOCAL_L2):
        np.testing.assert_allclose(O.forward_columns(tau, cl, model),
                                   O.forward(phase, absorb, L, model), rtol=1e-11)


def _fd_grad(loss, x, h):
    out = np.empty_like(x)
    for idx in np.ndindex(x.shape):
        e = np.zeros_like(x)
        e[idx] = h
        out[idx] = (loss(x + e) - loss(x - e)) / (2 * h)
    return out


@pytest.mark.parametrize("model", [O.LOCAL_L1, O.LOCAL_L2])
def test_column_vjp_matches_central_differences_everywhere(model):
    # the closures are smooth in tau: every pixel, borders included
    n, m = 9, 12
    bx, E, W = _profile(m)
    cl = O.column_line_constants(bx, E, W, m, 1e-6, 0.5, 1e-6, 1e-7)
    tau = _blob(n, m, 2.5, (4.5, 6.2), 2e-4) + 2e-5 * np.random.default_rng(2).standard_normal((n, m))
    g = np.random.default_rng(3).standard_normal((n, m))
    got = O.forward_columns_vjp(tau, g, cl, model)
    fd = _fd_grad(lambda t: np.vdot(g, O.forward_columns(t, cl, model)), tau, 1e-9)
    np.testing.assert_allclose(got, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
    if model == O.LOCAL_L2:
        assert np.abs(got - O.forward_columns_vjp(tau, g, cl, O.LOCAL_L1)).max() > 1e-3 * np.abs(got).max()


@pytest.mark.parametrize("model", [O.NONLOCAL, O.NONLOCAL_L2])
def test_column_vjp_matches_central_differences_off_kinks(model):
    n, m = 10, 12
    bx, E, W = _profile(m)
    cl = O.column_line_constants(bx, E, W, m, 1e-6, 0.5, 1e-6, 1e-7)
    tau = _blob(n, m, 2.5, (4.5, 6.2), 2e-4)
    g = np.random.default_rng(4).standard_normal((n, m))
    got = O.forward_columns_vjp(tau, g, cl, model)

    def loss(t):
        return np.vdot(g, O.forward_columns(t, cl, model))

    l0, h, checked = loss(tau), 1e-11, 0
    for idx in np.ndindex(tau.shape):
        e = np.zeros_like(tau)
        e[idx] = h
        fwd, bwd = (loss(tau + e) - l0) / h, (l0 - loss(tau - e)) / h
        if abs(fwd - bwd) > 1e-4 * max(1.0, abs(fwd)):
            continue
        assert 0.5 * (fwd + bwd) == pytest.approx(got[idx], rel=1e-4, abs=1e-5 * np.abs(got).max())
        checked += 1
    assert checked >= tau.size // 2


def test_uniform_profile_column_vjp_is_the_map_vjp():
    # tau enters the maps at the reference energy as phase = -k_ref delta_ref tau and
    # absorb = mu_ref tau: dL/dtau = -k_ref delta_ref dL/dphase + mu_ref dL/dabsorb
    n = 20
    E, W = [35.0, 55.0], [0.55, 0.45]
    cl = O.column_line_constants([5.0, 14.0], [E, E], [W, W], n, P, DIST, *MAT)
    L = O.line_constants(E, W, P, DIST, *MAT)
    tau = _blob(n, n, 3.0, (9.5, 10.2), 4e-4)
    cp = (O.line_phases(np.ones((1, 1)), L)[0] / L.phase_scale[0])[0, 0]
    ca = L.mu[0] / L.absorb_scale[0]
    g = np.random.default_rng(6).standard_normal((n, n))
    for model in (O.NONLOCAL, O.NONLOCAL_L2, O.LOCAL_L1, O.LOCAL_L2):
        gp, ga = O.forward_vjp(cp * tau, ca * tau, g, L, model)
        np.testing.assert_allclose(O.forward_columns_vjp(tau, g, cl, model), cp * gp + ca * ga,
                                   rtol=1e-10, atol=1e-12 * np.abs(gp).max())
