"""Pins of the oracle's vector-Jacobian products of the local closures (Eq. 1) and of the
second-order non-local model (transport plus diffraction pressure): central differences of the
oracle's own forward model, whose terms are pinned elsewhere, at every pixel of small grids
(borders included, where the one-sided differences make D^T differ from -D)."""

import numpy as np
import pytest

from oracle import epr_oracle as O

from tests.test_oracle_solver import smooth_object


def lines():
    return O.line_constants([22.0, 31.0], [0.55, 0.45], 1e-6, 0.5, 4e-7, 4e-10)


def setup(shape, seed):
    phase, absorb = smooth_object(shape, seed, 3.0, 0.4)
    r = np.random.default_rng(seed + 100)
    # a little texture so that no term is flat
    phase = phase + 0.2 * r.standard_normal(shape)
    absorb = absorb + 0.02 * r.standard_normal(shape)
    g = r.standard_normal(shape)
    return phase, absorb, g


def fd_gradient(loss, x, h):
    out = np.empty_like(x)
    for idx in np.ndindex(x.shape):
        e = np.zeros_like(x)
        e[idx] = h
        out[idx] = (loss(x + e) - loss(x - e)) / (2 * h)
    return out


@pytest.mark.parametrize("model", [O.LOCAL_L1, O.LOCAL_L2])
def test_local_vjp_matches_central_differences_everywhere(model):
    L = lines()
    assert 0.05 < L.eps_px.max() < 5.0   # every term of the closure contributes
    phase, absorb, g = setup((9, 11), 3)
    gp, ga = O.forward_vjp(phase, absorb, g, L, model)

    def lp(ph):
        return np.vdot(g, O.forward(ph, absorb, L, model))

    def la(ab):
        return np.vdot(g, O.forward(phase, ab, L, model))

    fp = fd_gradient(lp, phase, 1e-5)
    fa = fd_gradient(la, absorb, 1e-5)
    np.testing.assert_allclose(gp, fp, rtol=1e-6, atol=1e-7 * np.abs(fp).max())
    np.testing.assert_allclose(ga, fa, rtol=1e-6, atol=1e-7 * np.abs(fa).max())


def test_second_order_terms_matter():
    # the order-2 gradient differs from the order-1 one by more than the tolerance above, and
    # the pressure term's part is nonzero: a dropped term would fail the test above
    L = lines()
    phase, absorb, g = setup((9, 11), 3)
    p1, a1 = O.forward_vjp(phase, absorb, g, L, O.LOCAL_L1)
    p2, a2 = O.forward_vjp(phase, absorb, g, L, O.LOCAL_L2)
    assert np.abs(p2 - p1).max() > 1e-3 * np.abs(p2).max()
    assert np.abs(a2 - a1).max() > 1e-3 * np.abs(a2).max()
    q1, b1 = O.forward_vjp(phase, absorb, g, L, O.NONLOCAL)
    q2, b2 = O.forward_vjp(phase, absorb, g, L, O.NONLOCAL_L2)
    assert np.abs(b2 - b1).max() > 1e-3 * np.abs(b2).max()
    np.testing.assert_array_equal(q2, q1)   # the pressure term does not depend on the phase


def test_nonlocal_l2_vjp_matches_central_differences():
    # absorption enters smoothly: every pixel; the phase enters the transport piecewise
    # linearly: pixels away from a kink
    L = lines()
    phase, absorb, g = setup((10, 12), 5)
    gp, ga = O.forward_vjp(phase, absorb, g, L, O.NONLOCAL_L2)

    def la(ab):
        return np.vdot(g, O.forward(phase, ab, L, O.NONLOCAL_L2))

    fa = fd_gradient(la, absorb, 1e-5)
    np.testing.assert_allclose(ga, fa, rtol=1e-6, atol=1e-7 * np.abs(fa).max())

    def lp(ph):
        return np.vdot(g, O.forward(ph, absorb, L, O.NONLOCAL_L2))

    l0 = lp(phase)
    checked = 0
    for idx in np.ndindex(phase.shape):
        e = np.zeros_like(phase)
        e[idx] = 1e-7
        fwd = (lp(phase + e) - l0) / 1e-7
        bwd = (l0 - lp(phase - e)) / 1e-7
        if abs(fwd - bwd) > 1e-5 * max(1.0, abs(fwd)):
            continue
        assert 0.5 * (fwd + bwd) == pytest.approx(gp[idx], rel=1e-5, abs=1e-6)
        checked += 1
    assert checked >= phase.size // 2
