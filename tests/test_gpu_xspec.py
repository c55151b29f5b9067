"""Solves with an x-dependent effective spectrum on the GPU against the oracle: per-line energies
and weights on column blocks, interpolated across the detector; thickness within relative L2
1e-4; a uniform profile reproduces the uniform solver; argument checks."""

import numpy as np
import pytest

from oracle import epr_oracle as O
from tests.helpers import rel_l2, requires_gpu, to_dev, to_np

pytestmark = [pytest.mark.gpu, requires_gpu]

# delta / beta = 100 by default; test_xspec_solve_matches_oracle_weak_absorption takes the
# configurations' 1000
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


@pytest.mark.parametrize("shape,model,n_lines,shift", [((96, 128), "nonlocal", 3, 3.0),
                                                       ((90, 250), "nonlocal", 8, 2.0),
                                                       ((128, 128), "local_l2", 3, 0.5),
                                                       ((64, 96), "local_l1", 4, 0.5)])
def test_xspec_solve_matches_oracle_weak_absorption(shape, model, n_lines, shift):
    # delta / beta = 1000, the configurations' ratio: the absorption is weak, so a thickness
    # offset left in one iteration (which the strongly low-pass preconditioner removes only
    # slowly away from zero frequency) shows; the projection must not add a column-dependent
    # one (the float32 rounding of w_s(x) (1 / w_s(x)) once did, 7e-4 after 8 iterations)
    bref = 4e-10
    print(f"xspec delta/beta=1000 {shape} {model} lines={n_lines}", flush=True)
    bx, E, W = profile(shape[1], n_lines)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, bref)
    truth = thickness(shape, 7, shift, cl)
    d = O.forward_columns(truth, cl, model)
    ref = O.solve_columns(d, cl, model, 8, 0.5)
    from paper_2601_22793_amd import Material
    geom, spec, prof, _ = api(shape, bx, E, W)
    tau = ctx().solve_xspec(to_dev(d), geom, spec, prof, Material(DREF, bref), model, 8, 0.5)
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


# ---- block-wise interpolated preconditioner ---------------------------------------------------

def api_nb(shape, bx, E, W, nb):
    from paper_2601_22793_amd import Geometry, Material, Spectrum, SpectrumProfile
    return (Geometry(shape[0], shape[1], PIX, DIST),
            Spectrum(list(E[0]), list(W[0]), 60.0, 2.0, nb),
            SpectrumProfile(bx, E, W), Material(DREF, BREF))


@pytest.mark.parametrize("shape,model,n_lines,shift,f", [((96, 128), "nonlocal", 3, 3.0, 1),
                                                         ((90, 250), "nonlocal", 8, 2.0, 1),
                                                         ((128, 128), "local_l2", 3, 0.5, 1),
                                                         ((64, 96), "local_l1", 4, 0.5, 1),
                                                         ((96, 128), "nonlocal_l2", 3, 2.0, 1),
                                                         ((64, 80), "nonlocal", 3, 2.0, 2)])
def test_blockwise_preconditioner_matches_oracle(shape, model, n_lines, shift, f):
    # beta ~ E^-4 makes alpha ~ E differ between the blocks, so the block filters differ
    nb = 4.0
    print(f"xspec block-wise {shape} {model} lines={n_lines} f={f}", flush=True)
    bx, E, W = profile(shape[1], n_lines)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF, beta_exponent=nb,
                                 oversample=f)
    ishape = (shape[0] * f, shape[1] * f)
    truth = thickness(ishape, 7, shift, cl)
    d = O.forward_columns(truth, cl, model, oversample=f)
    block = (O.block_alphas(E, PIX, DIST, DREF, BREF, beta_exponent=nb, oversample=f),
             O.block_weights(bx, shape[1], f))
    ref = O.solve_columns(d, cl, model, 6, 0.5, oversample=f, block=block)
    mean = O.solve_columns(d, cl, model, 6, 0.5, oversample=f)
    assert rel_l2(mean, ref) > 1e-3     # the two preconditioners take different paths
    geom, spec, prof, mat = api_nb(shape, bx, E, W, nb)
    tau = ctx().solve_xspec(to_dev(d), geom, spec, prof, mat, model, 6, 0.5, oversample=f,
                            block_precond=True)
    assert rel_l2(to_np(tau), ref) <= 1e-4


def test_blockwise_with_energy_independent_alpha_is_the_mean_filter():
    # delta ~ E^-2, beta ~ E^-3: alpha does not depend on the energy, every block filter is the
    # same, and the block-wise solve is the column-mean one
    shape = (96, 128)
    bx, E, W = profile(shape[1], 3)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF)
    d = O.forward_columns(thickness(shape, 5, 2.0, cl), cl, "nonlocal")
    geom, spec, prof, mat = api(shape, bx, E, W)
    a = to_np(ctx().solve_xspec(to_dev(d), geom, spec, prof, mat, "nonlocal", 6, 0.5))
    b = to_np(ctx().solve_xspec(to_dev(d), geom, spec, prof, mat, "nonlocal", 6, 0.5,
                                block_precond=True))
    assert rel_l2(b, a) <= 1e-6


def test_blockwise_argument_checks():
    from paper_2601_22793_amd import EprError, SpectrumProfile
    shape = (64, 64)
    bx, E, W = profile(64)
    geom, spec, prof, mat = api(shape, bx, E, W)
    d = to_dev(np.ones(shape))
    n = 9   # more blocks than the block-wise preconditioner takes
    many = SpectrumProfile(list(np.linspace(0, 63, n)), np.repeat(E[:1], n, axis=0),
                           np.repeat(W[:1], n, axis=0))
    with pytest.raises(EprError) as ei:
        ctx().solve_xspec(d, geom, spec, many, mat, block_precond=True)
    assert ei.value.status == -6
    # the flag belongs to the x-dependent solve only
    import ctypes as C
    from paper_2601_22793_amd import _lib as L
    c = ctx()
    o = L.Opts(L.EPR_NONLOCAL, 2, 0.4, L.EPR_FLAG_BLOCK_PRECOND, 1)
    t = to_dev(np.zeros(shape))
    g, s, m = geom.c(), spec.c(), mat.c()
    st = c.lib.epr_solve(c.h, C.byref(g), C.byref(s), C.byref(m), C.byref(o),
                         C.c_void_p(d.data_ptr()), C.c_void_p(t.data_ptr()), None, None)
    assert st == L.EPR_ERR_UNSUPPORTED


# ---- batched x-dependent solve ------------------------------------------------------------------

def test_batched_xspec_matches_per_problem_and_oracle():
    # problems of different sizes (both spectral size classes), line-set energies and profiles,
    # against epr_solve_xspec one by one and the oracle
    import torch
    from paper_2601_22793_amd import Geometry, Material, Spectrum, SpectrumProfile
    cases = [((96, 128), 3, 3.0, 0), ((64, 80), 3, 2.0, 1), ((40, 2160), 3, 2.0, 2),
             ((128, 96), 3, 1.5, 3)]
    probs, profs, refs, datas = [], [], [], []
    for shape, n_lines, shift, k in cases:
        bx, E, W = profile(shape[1], n_lines)
        E = E + 2.0 * k                        # a different spectrum per problem
        cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF)
        truth = thickness(shape, 20 + k, shift, cl)
        d = O.forward_columns(truth, cl, "nonlocal")
        refs.append(O.solve_columns(d, cl, "nonlocal", 5, 0.5))
        geom = Geometry(shape[0], shape[1], PIX, DIST)
        spec = Spectrum(list(E[0]), list(W[0]), 60.0, 2.0, 3.0)
        prof = SpectrumProfile(bx, E, W)
        probs.append((to_dev(d), torch.zeros(shape, dtype=torch.float32, device="cuda"), geom,
                      spec, Material(DREF, BREF)))
        profs.append(prof)
        datas.append(d)
    print("batched xspec: 4 problems, 5 iterations", flush=True)
    c = ctx()
    for rep in range(2):   # the second call replays the cached graph
        for p in probs:
            p[1].zero_()
        c.solve_batched_xspec(probs, profs, "nonlocal", 5, 0.5)
        torch.cuda.synchronize()
        for i, p in enumerate(probs):
            single = c.solve_xspec(to_dev(datas[i]), p[2], p[3], profs[i], p[4], "nonlocal", 5, 0.5)
            got = to_np(p[1])
            assert rel_l2(got, to_np(single)) <= 1e-6, (rep, i)
            assert rel_l2(got, refs[i]) <= 1e-4, (rep, i)


def test_batched_xspec_oversampled_matches_per_problem():
    import torch
    from paper_2601_22793_amd import Geometry, Material, Spectrum, SpectrumProfile
    f = 2
    probs, profs, datas = [], [], []
    for k, (shape, model) in enumerate([((48, 64), "nonlocal"), ((40, 50), "nonlocal")]):
        bx, E, W = profile(shape[1], 3)
        E = E + 3.0 * k
        cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF, oversample=f)
        truth = thickness((shape[0] * f, shape[1] * f), 30 + k, 2.0, cl)
        d = O.forward_columns(truth, cl, model, oversample=f)
        geom = Geometry(shape[0], shape[1], PIX, DIST)
        spec = Spectrum(list(E[0]), list(W[0]), 60.0, 2.0, 3.0)
        probs.append((to_dev(d), torch.zeros((shape[0] * f, shape[1] * f), dtype=torch.float32,
                                             device="cuda"), geom, spec, Material(DREF, BREF)))
        profs.append(SpectrumProfile(bx, E, W))
        datas.append((d, cl))
    c = ctx()
    c.solve_batched_xspec(probs, profs, "nonlocal", 4, 0.5, oversample=f)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        single = c.solve_xspec(to_dev(datas[i][0]), p[2], p[3], profs[i], p[4], "nonlocal", 4, 0.5,
                               oversample=f)
        assert rel_l2(to_np(p[1]), to_np(single)) <= 1e-6, i
        ref = O.solve_columns(datas[i][0], datas[i][1], "nonlocal", 4, 0.5, oversample=f)
        assert rel_l2(to_np(p[1]), ref) <= 1e-4, i


@pytest.mark.parametrize("shape,model,n_lines,shift", [((96, 128), "nonlocal", 3, 3.0),
                                                       ((90, 250), "nonlocal_l2", 8, 2.0),
                                                       ((128, 128), "local_l2", 3, 0.5),
                                                       ((64, 96), "local_l1", 4, 0.5)])
def test_xspec_forward_matches_oracle(shape, model, n_lines, shift):
    bx, E, W = profile(shape[1], n_lines)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF)
    truth = thickness(shape, 9, shift, cl)
    ref = O.forward_columns(truth, cl, model)
    geom, spec, prof, mat = api(shape, bx, E, W)
    got = to_np(ctx().forward_xspec(to_dev(truth), geom, spec, prof, mat, model))
    print(f"xspec forward {shape} {model}: rel L2 {rel_l2(got, ref):.2e}", flush=True)
    assert rel_l2(got, ref) <= 1e-5


@pytest.mark.parametrize("shape,model,n_lines,shift", [((96, 128), "nonlocal", 3, 3.0),
                                                       ((90, 250), "nonlocal", 8, 5.0),
                                                       ((64, 96), "local_l2", 4, 0.5)])
def test_xspec_adjoint_matches_oracle(shape, model, n_lines, shift):
    bx, E, W = profile(shape[1], n_lines)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF)
    truth = thickness(shape, 10, shift, cl)
    r = np.random.default_rng(12).standard_normal((n_lines,) + shape).astype(np.float32)
    ref = O.adjoint_columns(truth, r, cl, model)
    geom, spec, prof, mat = api(shape, bx, E, W)
    got = to_np(ctx().adjoint_xspec(to_dev(truth), to_dev(r), geom, spec, prof, mat, model))
    print(f"xspec adjoint {shape} {model}: rel L2 {rel_l2(got, ref):.2e}", flush=True)
    assert rel_l2(got, ref) <= 1e-5
    if model == "local_l2":
        np.testing.assert_array_equal(got, r)


def test_xspec_forward_of_a_uniform_profile_is_the_uniform_forward():
    from paper_2601_22793_amd import Geometry, Material, Spectrum, SpectrumProfile
    shape = (64, 80)
    E, W = [40.0, 60.0, 85.0], [0.3, 0.5, 0.2]
    L = O.line_constants(E, W, PIX, DIST, DREF, BREF)
    cl = O.column_line_constants([0.0, 79.0], [E, E], [W, W], shape[1], PIX, DIST, DREF, BREF)
    tau = thickness(shape, 13, 2.0, cl)
    phase = (O.line_phases(tau, L)[0] / L.phase_scale[0]).astype(np.float32)
    absorb = (tau * L.mu[0] / L.absorb_scale[0]).astype(np.float32)
    geom = Geometry(shape[0], shape[1], PIX, DIST)
    spec = Spectrum(E, W, 60.0, 2.0, 3.0)
    prof = SpectrumProfile([0.0, 79.0], [E, E], [W, W])
    for model in ("nonlocal", "local_l2"):
        a = to_np(ctx().forward_xspec(to_dev(tau), geom, spec, prof, Material(DREF, BREF), model))
        b = to_np(ctx().forward(to_dev(phase), to_dev(absorb), geom, spec, model))
        assert rel_l2(a, b) <= 1e-5, model


def test_xspec_solve_with_grouped_row_lines_equals_one_line_per_workgroup(tmp_path):
    # the x-dependent row pass with four lines per workgroup (one after the other) gives the
    # one-line result
    import json
    import torch
    from paper_2601_22793_amd import Context
    shape, model, n_lines = (96, 128), "nonlocal", 8
    bx, E, W = profile(shape[1], n_lines)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF)
    d = O.forward_columns(thickness(shape, 7, 3.0, cl), cl, model)
    geom, spec, prof, mat = api(shape, bx, E, W)
    got = {}
    for lines in (1, 4):
        c = Context(0)
        try:
            path = str(tmp_path / f"lines{lines}.json")
            with open(path, "w") as fh:
                json.dump({"splat_tx": 64, "splat_ty": 32, "row_lines": lines}, fh)
            entry = (to_dev(d), torch.zeros(shape, dtype=torch.float32, device="cuda"), geom, spec,
                     mat)
            c.autotune([entry], model, cache_json=path)
            got[lines] = to_np(c.solve_xspec(to_dev(d), geom, spec, prof, mat, model, 8, 0.5))
        finally:
            c.close()
    assert rel_l2(got[4], got[1]) <= 1e-6


# ---- vector-Jacobian product with respect to the thickness ---------------------------------

def vjp_thickness(shape, seed, shift, cl):
    """thickness() with its far tails set to exactly zero, in float32 for both sides.  The
    non-local model is piecewise linear in the shift with kinks where a shift crosses an
    integer; a Gaussian tail leaves shifts of 1e-30 px or so whose sign (and so which cell's
    slope the gradient takes) float32 and float64 can disagree on, while at an exact zero both
    take the same one-sided slope."""
    t = thickness(shape, seed, shift, cl)
    t[t < 1e-6 * t.max()] = 0.0
    return t.astype(np.float32)

@pytest.mark.parametrize("shape,model,n_lines,shift", [((96, 128), "nonlocal", 3, 3.0),
                                                       ((90, 250), "nonlocal_l2", 8, 2.0),
                                                       ((128, 128), "local_l2", 3, 0.5),
                                                       ((64, 96), "local_l1", 4, 0.5)])
def test_xspec_vjp_matches_oracle(shape, model, n_lines, shift):
    print(f"xspec vjp {shape} {model} lines={n_lines}", flush=True)
    bx, E, W = profile(shape[1], n_lines)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF)
    truth = vjp_thickness(shape, 11, shift, cl)
    g = np.random.default_rng(14).standard_normal(shape).astype(np.float32)
    ref = O.forward_columns_vjp(truth, g, cl, model)
    geom, spec, prof, mat = api(shape, bx, E, W)
    got = to_np(ctx().forward_xspec_vjp(to_dev(truth), to_dev(g), geom, spec, prof, mat, model))
    print(f"  rel L2 {rel_l2(got, ref):.2e}", flush=True)
    assert rel_l2(got, ref) <= 1e-4


@pytest.mark.parametrize("model,base", [("nonlocal_l2", "nonlocal"), ("local_l2", "local_l1")])
def test_xspec_vjp_second_order_part_matches_oracle(model, base):
    # the part of the gradient that the second-order terms add (with the pressure coefficient
    # varying across the columns) is a small share of the whole: compared on its own
    shape, n_lines = (96, 128), 3
    bx, E, W = profile(shape[1], n_lines)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF)
    truth = vjp_thickness(shape, 15, 1.0, cl)
    g = np.random.default_rng(16).standard_normal(shape).astype(np.float32)
    ref = O.forward_columns_vjp(truth, g, cl, model) - O.forward_columns_vjp(truth, g, cl, base)
    geom, spec, prof, mat = api(shape, bx, E, W)
    t, gd = to_dev(truth), to_dev(g)
    got = to_np(ctx().forward_xspec_vjp(t, gd, geom, spec, prof, mat, model)) - \
        to_np(ctx().forward_xspec_vjp(t, gd, geom, spec, prof, mat, base))
    print(f"xspec vjp {model} - {base}: rel L2 {rel_l2(got, ref):.2e}", flush=True)
    assert rel_l2(got, ref) <= 1e-2


def test_xspec_vjp_of_a_uniform_profile_is_the_map_vjp():
    # tau enters the uniform model through phase = c_p tau and absorb = c_a tau, so
    # dL/dtau = c_p dL/dphase + c_a dL/dabsorb
    from paper_2601_22793_amd import Geometry, Material, Spectrum, SpectrumProfile
    shape = (64, 80)
    E, W = [40.0, 60.0, 85.0], [0.3, 0.5, 0.2]
    L = O.line_constants(E, W, PIX, DIST, DREF, BREF)
    cl = O.column_line_constants([0.0, 79.0], [E, E], [W, W], shape[1], PIX, DIST, DREF, BREF)
    tau = vjp_thickness(shape, 17, 2.0, cl)
    cp = float(O.line_phases(np.ones((1, 1)), L)[0][0, 0] / L.phase_scale[0])
    ca = float(L.mu[0] / L.absorb_scale[0])
    geom = Geometry(shape[0], shape[1], PIX, DIST)
    spec = Spectrum(E, W, 60.0, 2.0, 3.0)
    prof = SpectrumProfile([0.0, 79.0], [E, E], [W, W])
    g = to_dev(np.random.default_rng(18).standard_normal(shape).astype(np.float32))
    for model in ("nonlocal", "nonlocal_l2", "local_l1", "local_l2"):
        a = to_np(ctx().forward_xspec_vjp(to_dev(tau), g, geom, spec, prof, Material(DREF, BREF),
                                          model))
        gp, ga = ctx().forward_vjp(to_dev(cp * tau), to_dev(ca * tau), g, geom, spec, model)
        b = cp * to_np(gp).astype(np.float64) + ca * to_np(ga)
        assert rel_l2(a, b) <= 1e-4, model


def test_xspec_autograd_backward_is_the_vjp():
    import torch
    from paper_2601_22793_amd import epr_forward_xspec
    shape = (64, 96)
    bx, E, W = profile(shape[1], 4)
    cl = O.column_line_constants(bx, E, W, shape[1], PIX, DIST, DREF, BREF)
    geom, spec, prof, mat = api(shape, bx, E, W)
    tau = to_dev(thickness(shape, 19, 2.0, cl)).requires_grad_(True)
    g = to_dev(np.random.default_rng(20).standard_normal(shape).astype(np.float32))
    (epr_forward_xspec(tau, geom, spec, prof, mat, "nonlocal_l2") * g).sum().backward()
    ref = ctx().forward_xspec_vjp(tau.detach(), g, geom, spec, prof, mat, "nonlocal_l2")
    torch.cuda.synchronize()
    assert torch.equal(tau.grad, ref)


def test_xspec_vjp_argument_checks():
    import ctypes as C
    from paper_2601_22793_amd import EprError
    shape = (64, 64)
    bx, E, W = profile(64)
    geom, spec, prof, mat = api(shape, bx, E, W)
    t = to_dev(np.ones(shape))
    g = to_dev(np.ones(shape))
    with pytest.raises(EprError) as ei:
        ctx().forward_xspec_vjp(t, g, geom, spec, prof, mat, model="auto")
    assert ei.value.status == -6
    for call in (lambda: ctx().forward(t, t, geom, spec, "auto"),
                 lambda: ctx().forward_vjp(t, t, g, geom, spec, "auto"),
                 lambda: ctx().forward_xspec(t, geom, spec, prof, mat, "auto")):
        with pytest.raises(EprError) as ei:   # the operators need an explicit model
            call()
        assert ei.value.status == -6
    with pytest.raises(EprError) as ei:
        ctx().forward_xspec_vjp(t, g, geom, spec, prof, mat, model=9)
    assert ei.value.status == -1
    c = ctx()
    gg, ss, pp, mm = geom.c(), spec.c(), prof.c(), mat.c()
    for out in (t, g):   # the gradient must not overwrite an input
        st = c.lib.epr_forward_xspec_vjp(c.h, C.byref(gg), C.byref(ss), C.byref(pp), C.byref(mm),
                                         3, t.data_ptr(), g.data_ptr(), out.data_ptr(), None)
        assert st == -1
