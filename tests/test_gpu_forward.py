"""Forward model and adjoint on the GPU against the FP64 oracle (relative L2 <= 1e-5), plus the
FP32 invariants of the splat (conservation, adjoint identity)."""

import numpy as np
import pytest

from oracle import epr_oracle as O
from synthetic import workload
from tests.helpers import api_objects, oracle_lines, rel_l2, requires_gpu, to_dev, to_np

pytestmark = [pytest.mark.gpu, requires_gpu]

TOL = 1e-5


def ctx():
    from paper_2601_22793_amd import Context
    return Context.get(0)


def nonlocal_case(shape, n_lines, max_shift=6.0, seed_off=0):
    base = "nonlocal-poly8-2048" if n_lines == 8 else "nonlocal-mono-2048"
    w = workload(base, shape=shape, max_shift_px=max_shift)
    w.seed += seed_off
    return w, w.true_object()


def local_case(shape, n_lines):
    w = workload("local-mono-256", shape=shape)
    if n_lines > 1:
        from synthetic import bremsstrahlung_bins
        e, wt = bremsstrahlung_bins(n_lines, np.random.default_rng(11))
        w.energies_kev, w.weights = e, wt
    return w, w.true_object()


@pytest.mark.parametrize("shape", [(90, 250), (256, 256), (160, 96)])
@pytest.mark.parametrize("n_lines", [1, 8])
def test_nonlocal_forward_matches_oracle(shape, n_lines):
    w, obj = nonlocal_case(shape, n_lines)
    print(f"nonlocal forward {shape} lines={n_lines}", flush=True)
    geom, spec, _ = api_objects(w)
    ref = O.forward(obj["phase"], obj["absorb"], oracle_lines(w), O.NONLOCAL)
    out = ctx().forward(to_dev(obj["phase"]), to_dev(obj["absorb"]), geom, spec, "nonlocal")
    assert rel_l2(to_np(out), ref) <= TOL


@pytest.mark.parametrize("model", ["local_l1", "local_l2"])
@pytest.mark.parametrize("shape,n_lines", [((90, 250), 1), ((256, 256), 1), ((128, 160), 8)])
def test_local_forward_matches_oracle(model, shape, n_lines):
    w, obj = local_case(shape, n_lines)
    print(f"{model} forward {shape} lines={n_lines}", flush=True)
    geom, spec, _ = api_objects(w)
    ref = O.forward(obj["phase"], obj["absorb"], oracle_lines(w), model)
    out = ctx().forward(to_dev(obj["phase"]), to_dev(obj["absorb"]), geom, spec, model)
    assert rel_l2(to_np(out), ref) <= TOL


def test_nonlocal_forward_halo_larger_than_tile():
    # shifts up to 40 px: the device-derived halo (41 px) exceeds the 64 x 32 splat tile
    w, obj = nonlocal_case((192, 200), 1, max_shift=40.0)
    geom, spec, _ = api_objects(w)
    ref = O.forward(obj["phase"], obj["absorb"], oracle_lines(w), O.NONLOCAL)
    out = ctx().forward(to_dev(obj["phase"]), to_dev(obj["absorb"]), geom, spec, "nonlocal")
    assert rel_l2(to_np(out), ref) <= TOL


def test_zero_phase_forward_is_beer_lambert_sum():
    w, obj = nonlocal_case((96, 128), 8)
    geom, spec, _ = api_objects(w)
    z = np.zeros_like(obj["phase"])
    ref = O.forward(z, obj["absorb"], oracle_lines(w), O.NONLOCAL)
    for model in ("nonlocal", "local_l1"):
        out = ctx().forward(to_dev(z), to_dev(obj["absorb"]), geom, spec, model)
        assert rel_l2(to_np(out), ref) <= 1e-6


def _mono_unit(shape, seed):
    """A one-line spectrum at the reference energy: I = exp(-absorb), u = eps D phase."""
    w, obj = nonlocal_case(shape, 1, seed_off=seed)
    return w, obj


def test_fp32_conservation_and_adjoint_identity():
    w, obj = _mono_unit((128, 160), 3)
    geom, spec, _ = api_objects(w)
    rng = np.random.default_rng(5)
    A = rng.uniform(0.0, 2.0, size=(128, 160)).astype(np.float32)
    # no mass within 12 px of the border, so every target (|u| <= 6 px) lands on the grid
    A[:12] = A[-12:] = 1e3
    A[:, :12] = A[:, -12:] = 1e3
    x = np.exp(-A.astype(np.float64))
    P = to_np(ctx().forward(to_dev(obj["phase"]), to_dev(A), geom, spec, "nonlocal"))
    assert abs(P.sum() - x.sum()) <= 1e-6 * x.sum()
    y = rng.standard_normal((1, 128, 160)).astype(np.float32)
    My = to_np(ctx().adjoint(to_dev(obj["phase"]), to_dev(y), geom, spec, "nonlocal"))
    lhs = float(np.vdot(P, y[0]))
    rhs = float(np.vdot(x, My[0]))
    assert abs(lhs - rhs) <= 1e-6 * np.sqrt(np.vdot(P, P) * np.vdot(y, y))


@pytest.mark.parametrize("shape,n_lines", [((90, 250), 8), ((256, 256), 1)])
def test_adjoint_matches_oracle(shape, n_lines):
    w, obj = nonlocal_case(shape, n_lines)
    geom, spec, _ = api_objects(w)
    rng = np.random.default_rng(7)
    res = rng.standard_normal((n_lines,) + shape).astype(np.float32)
    ref = O.adjoint(obj["phase"], res, oracle_lines(w), O.NONLOCAL)
    out = ctx().adjoint(to_dev(obj["phase"]), to_dev(res), geom, spec, "nonlocal")
    assert rel_l2(to_np(out), ref) <= TOL
    loc = ctx().adjoint(to_dev(obj["phase"]), to_dev(res), geom, spec, "local_l2")
    assert np.array_equal(to_np(loc), res.astype(np.float64))


@pytest.mark.parametrize("shape", [(96, 200), (64, 1200)])
@pytest.mark.parametrize("ux,uy", [(20.3, -6.2), (-13.7, 5.4)])
def test_adjoint_with_taps_beyond_the_border(shape, ux, uy):
    # a constant shift of many pixels: waves whose stencil lies inside the image still have taps
    # beyond its edges, which must read as zero (the interior path's vote falls back to the
    # clamped taps there)
    print(f"adjoint beyond border {shape} u=({ux}, {uy})", flush=True)
    w, _ = nonlocal_case(shape, 1)
    L = oracle_lines(w)
    k = L.eps_px[0] * L.phase_scale[0]
    y, x = np.mgrid[0:shape[0], 0:shape[1]].astype(np.float64)
    phase = ((ux * x + uy * y) / k).astype(np.float32)
    res = np.random.default_rng(3).standard_normal((1,) + shape).astype(np.float32)
    ref = O.adjoint(phase, res, L, O.NONLOCAL)
    geom, spec, _ = api_objects(w)
    out = ctx().adjoint(to_dev(phase), to_dev(res), geom, spec, "nonlocal")
    assert rel_l2(to_np(out), ref) <= TOL
