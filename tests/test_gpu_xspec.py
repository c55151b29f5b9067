"""Solves with an x-dependent effective spectrum on the GPU against the oracle: per-line energies
and weights on column blocks, interpolated across the detector; thickness within relative L2
1e-4; a uniform profile reproduces the uniform solver; argument checks."""

import numpy as np
import pytest

from oracle import epr_oracle as O
from tests.helpers import rel_l2, requires_gpu, to_dev, to_np

pytestmark = [pytest.mark.gpu, requires_gpu]

# delta / beta = 100: the thickness is well above the float32 floor of the projection
PIX, DIST, DREF, BREF = 5e-6, 2.0, 4e-7, 4e-9


def ctx():
    from paper_2601_22793_amd import Context
    return Context.get(0)


def profile(nx, n_lines=3):
    # harder spectrum in the middle of the field (a cylindrical container), three blocks
    bx = [0.0, nx / 2.0, nx - 1.0]
    base = np.linspace(45.0, 90.0, n_lines)
    E = np.stack([base, base + 8.0, base + 1.0])
    W = np.stack([np.linspace(0.5, 0.2, n_lines), np.full(n_lines, 1.0),
                  np.linspace(0.4, 0.3, n_lines)])
    W = W / W.sum(axis=1, keepdims=True)
    return bx, E, W


def thickness(shape, seed, max_shift_px, cl):
    r = np.random.default_rng(seed)
    ny, nx = shape
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    t = np.zeros(shape)
    for _ in range(6):
        cy, cx = r.uniform(0.3, 0.7) * ny, r.uniform(0.3, 0.7) * nx
        s = r.uniform(0.05, 0.1) * min(shape)
        t += r.uniform(0.5, 1.0) * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * s * s))
    b = np.abs(cl.eps_px * cl.k * cl.delta).max()
    g = np.hypot(*np.gradient(t)).max()
    return t * (max_shift_px / (b * g))


def api(shape, bx, E, W):
    from paper_2601_22793_amd import Geometry, Material, Spectrum, SpectrumProfile
    return (Geometry(shape[0], shape[1], PIX, DIST),
            Spectrum(list(E[0]), list(W[0]), 60.0, 2.0, 3.0),
            SpectrumProfile(bx, E, W), Material(DREF, BREF))


@pytest.mark.parametrize("shape,model,n_lines,shift", [((96, 128), "nonlocal", 3, 3.0),
                                                       ((90, 250), "nonlocal", 8, 2.0),
                                                       ((128, 128), "local_l2", 3, 0.5),
                                                       ((64, 96), "local_l1", 4, 0.5)])
def test_xspec_solve_matches_oracle(shape, model, n_lines, shift):
    print(f"xspec {shape} {model} lines={n_lines}", flush=True)
    bx, E, W = profile(shape[1], n_lines)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF)
    truth = thickness(shape, 7, shift, cl)
    d = O.forward_columns(truth, cl, model)
    ref = O.solve_columns(d, cl, model, 8, 0.5)
    geom, spec, prof, mat = api(shape, bx, E, W)
    tau = ctx().solve_xspec(to_dev(d), geom, spec, prof, mat, model, 8, 0.5)
    assert rel_l2(to_np(tau), ref) <= 1e-4


@pytest.mark.parametrize("shape,model,f", [((64, 80), "nonlocal", 2), ((48, 64), "local_l2", 2),
                                           ((96, 128), "nonlocal_l2", 1),
                                           ((40, 50), "nonlocal_l2", 2)])
def test_xspec_oversampled_and_second_order_match_oracle(shape, model, f):
    print(f"xspec {shape} {model} f={f}", flush=True)
    bx, E, W = profile(shape[1], 3)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF, oversample=f)
    ishape = (shape[0] * f, shape[1] * f)
    truth = thickness(ishape, 11, 2.0 if model != "local_l2" else 0.5, cl)
    d = O.forward_columns(truth, cl, model, oversample=f)
    ref = O.solve_columns(d, cl, model, 6, 0.5, oversample=f)
    geom, spec, prof, mat = api(shape, bx, E, W)
    tau = ctx().solve_xspec(to_dev(d), geom, spec, prof, mat, model, 6, 0.5, oversample=f)
    assert tuple(tau.shape) == ishape
    assert rel_l2(to_np(tau), ref) <= 1e-4


@pytest.mark.parametrize("model", ["nonlocal", "local_l2"])
def test_uniform_profile_equals_the_uniform_solver(model):
    shape = (96, 120)
    E1, W1 = np.array([50.0, 70.0]), np.array([0.6, 0.4])
    bx, E, W = [10.0, 90.0], np.stack([E1, E1]), np.stack([W1, W1])
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF)
    truth = thickness(shape, 3, 2.0 if model == "nonlocal" else 0.5, cl)
    d = O.forward_columns(truth, cl, model)
    geom, spec, prof, mat = api(shape, bx, E, W)
    a = to_np(ctx().solve_xspec(to_dev(d), geom, spec, prof, mat, model, 6, 0.5))
    b = to_np(ctx().solve(to_dev(d), geom, spec, mat, model, 6, 0.5))
    assert rel_l2(a, b) <= 1e-6


def test_xspec_argument_checks():
    from paper_2601_22793_amd import EprError, SpectrumProfile
    shape = (64, 64)
    bx, E, W = profile(64)
    geom, spec, prof, mat = api(shape, bx, E, W)
    d = to_dev(np.ones(shape))
    with pytest.raises(EprError) as ei:     # block centres must increase
        ctx().solve_xspec(d, geom, spec, SpectrumProfile([0.0, 0.0, 10.0], E, W), mat)
    assert ei.value.status == -1
    bad = W.copy()
    bad[1, 0] += 0.1                         # weights of a block must sum to 1
    with pytest.raises(EprError) as ei:
        ctx().solve_xspec(d, geom, spec, SpectrumProfile(bx, E, bad), mat)
    assert ei.value.status == -1
    with pytest.raises(EprError) as ei:
        ctx().solve_xspec(d, geom, spec, prof, mat, model="auto")
    assert ei.value.status == -6
