"""Parity at the configurations' full sizes, in the launch configuration the benchmark times.

The FP64 references come from the oracle in CPU-only worker processes started with the test
session (tests/fullsize_oracle.py), so their minutes of work overlap the other GPU tests; this
module is collected last so that they are ready or nearly so.

* The 2048 x 2048 8-line forward model and adjoint on sampled row bands (the oracle computes
  each band from the band plus a margin wider than any shift, so its rows are exact oracle
  values of the full image).
* One 2048^2 projection, 1 line and 8 lines, 30 non-local iterations from the oracle's data:
  the retrieved thickness and phase against the oracle's, element by element.
* The 64-problem mixed batch (24 x 1024^2, 32 x 2048^2, 8 x 2160 x 2560, 8 lines) solved by the
  batched solver replaying its graph for 30 iterations: the first problem of each shape has
  the oracle's data and is compared with the oracle's solve, element by element.
* The vector-Jacobian product at 2048^2 with 8 lines against the oracle's, central differences
  (h = 1e-3) of the oracle's model at 64 pixels, and 50 Adam steps against the oracle's Adam.
"""

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import epr_oracle as O
from synthetic import batch_workloads, workload
from tests import fullsize_oracle as F
from tests.helpers import api_objects, oracle_lines, rel_l2, requires_gpu, to_dev, to_np

pytestmark = [pytest.mark.gpu, requires_gpu]

BANDS = [(0, 64), (1000, 1064), (1984, 2048)]


def ctx():
    from paper_2601_22793_amd import Context
    return Context.get(0)


def full_object():
    w = workload("nonlocal-poly8-2048")
    obj = w.true_object()
    L = oracle_lines(w)
    umax = 0.0
    for s in range(w.n_lines):
        ux, uy = O.shift_field(L.phase_scale[s] * obj["phase"].astype(np.float64), L.eps_px[s])
        umax = max(umax, float(np.abs(ux).max()), float(np.abs(uy).max()))
    margin = int(np.ceil(umax)) + 3
    return w, obj, L, margin


def test_forward_full_size_on_row_bands():
    w, obj, L, m = full_object()
    print(f"full-size forward {w.ny}x{w.nx} lines={w.n_lines} margin={m}", flush=True)
    geom, spec, _ = api_objects(w)
    out = to_np(ctx().forward(to_dev(obj["phase"]), to_dev(obj["absorb"]), geom, spec, "nonlocal"))
    for y0, y1 in BANDS:
        a0, a1 = max(y0 - m, 0), min(y1 + m, w.ny)
        ref = O.forward(obj["phase"][a0:a1], obj["absorb"][a0:a1], L, O.NONLOCAL)
        assert rel_l2(out[y0:y1], ref[y0 - a0:y1 - a0]) <= 1e-5, (y0, y1)


def test_adjoint_full_size_on_row_bands():
    w, obj, L, m = full_object()
    print(f"full-size adjoint {w.ny}x{w.nx} lines={w.n_lines} margin={m}", flush=True)
    geom, spec, _ = api_objects(w)
    res = np.random.default_rng(17).standard_normal((w.n_lines, w.ny, w.nx)).astype(np.float32)
    out = to_np(ctx().adjoint(to_dev(obj["phase"]), to_dev(res), geom, spec, "nonlocal"))
    for y0, y1 in BANDS:
        a0, a1 = max(y0 - m, 0), min(y1 + m, w.ny)
        ref = O.adjoint(obj["phase"][a0:a1], res[:, a0:a1], L, O.NONLOCAL)
        assert rel_l2(out[:, y0:y1], ref[:, y0 - a0:y1 - a0]) <= 1e-5, (y0, y1)


@pytest.mark.parametrize("name", ["nonlocal-mono-2048", "nonlocal-poly8-2048"])
def test_single_projection_full_size_matches_oracle(oracle_refs, name):
    w = workload(name)
    print(f"full-size solve {name}: {w.ny}x{w.nx}, {w.n_lines} line(s), {w.n_iter} iterations",
          flush=True)
    d = oracle_refs.load(name, "d")
    geom, spec, mat = api_objects(w)
    import torch
    phase = torch.empty((w.ny, w.nx), dtype=torch.float32, device="cuda")
    tau = ctx().solve(to_dev(d), geom, spec, mat, w.model, w.n_iter, w.relaxation,
                      phase_out=phase)
    got, got_phase = to_np(tau), to_np(phase)
    ref = oracle_refs.load(name, "tau")
    err = rel_l2(got, ref)
    print(f"{name}: thickness rel L2 vs oracle {err:.3e}", flush=True)
    assert err <= 1e-4
    # phase at the reference energy, -k_ref delta_ref tau
    ref_phase = -(2 * np.pi * w.energy_ref_kev * 1e3 / O.HC_EV_M) * w.delta_ref * ref
    assert rel_l2(got_phase, ref_phase) <= 1e-4


def test_batch64_full_configuration_matches_oracle(oracle_refs):
    import torch
    from paper_2601_22793_amd import Context
    wls = batch_workloads()
    picked = F.batch_indices()
    assert sorted(picked) == [(1024, 1024), (2048, 2048), (2160, 2560)]
    compared = set(picked.values())
    with ThreadPoolExecutor(16) as ex:
        objs = list(ex.map(lambda i: None if i in compared else wls[i].true_object(),
                           range(len(wls))))
    c = Context.get(0)
    gen = torch.Generator(device="cuda")
    probs = []
    for i, (w, obj) in enumerate(zip(wls, objs)):
        geom, spec, mat = api_objects(w)
        if obj is None:
            d = to_dev(oracle_refs.load(f"batch-{i}", "d"))
        else:
            # problems not compared: the benchmark's own data (GPU forward model + counting
            # noise), which fills the launch configuration
            clean = c.forward(to_dev(obj["phase"]), to_dev(obj["absorb"]), geom, spec, "nonlocal")
            gen.manual_seed(w.seed + 500)
            d = torch.poisson(clean.clamp_min(0) * w.photons, generator=gen) / w.photons
        probs.append((d.contiguous(), torch.zeros(w.shape, dtype=torch.float32, device="cuda"),
                      geom, spec, mat))
    n_iter = wls[0].n_iter
    print(f"batch64: {len(wls)} problems, {n_iter} iterations, graph replay", flush=True)
    c.set_timing(False)
    c.solve_batched(probs, "nonlocal", n_iter, wls[0].relaxation)
    torch.cuda.synchronize()
    assert c.diagnostics()["nonfinite"] == 0
    for shape, i in sorted(picked.items()):
        ref = oracle_refs.load(f"batch-{i}", "tau")
        err = rel_l2(to_np(probs[i][1]), ref)
        print(f"batch problem {i} {shape}: thickness rel L2 vs oracle {err:.3e}", flush=True)
        assert err <= 1e-4, (i, shape)


def vjp_case():
    w = workload("vjp-poly8-2048")
    return w, w.true_object()


def test_vjp_full_size_matches_oracle(oracle_refs):
    w, obj = vjp_case()
    geom, spec, _ = api_objects(w)
    g = F.vjp_cotangent(w.shape)
    gp, ga = ctx().forward_vjp(to_dev(obj["phase"]), to_dev(obj["absorb"]), to_dev(g), geom,
                               spec)
    rp = oracle_refs.load("vjp-poly8-2048", "grad_phase")
    ra = oracle_refs.load("vjp-poly8-2048", "grad_absorb")
    ep, ea = rel_l2(to_np(gp), rp), rel_l2(to_np(ga), ra)
    print(f"VJP 2048^2 x 8: rel L2 phase {ep:.3e}, absorption {ea:.3e}", flush=True)
    assert ep <= 1e-4 and ea <= 1e-4


def test_vjp_full_size_central_differences():
    # <g, P(phase, absorb)> is piecewise linear in the phase (the bilinear weights are linear
    # in the shift inside a cell), so its central difference is exact up to rounding unless a
    # mapped point crosses a cell edge within +-h: such pixels (one-sided differences disagree)
    # are redrawn.  The perturbation of pixel p moves only the sources whose central
    # difference reads p, so the oracle evaluates the functional on a window around p wider
    # than their footprints; every other source contributes the same to both evaluations.
    w, obj = vjp_case()
    geom, spec, _ = api_objects(w)
    L = oracle_lines(w)
    ph = obj["phase"].astype(np.float64)
    ab = obj["absorb"].astype(np.float64)
    g = F.vjp_cotangent(w.shape).astype(np.float64)
    gp, ga = ctx().forward_vjp(to_dev(ph), to_dev(ab), to_dev(g), geom, spec)
    gp, ga = to_np(gp), to_np(ga)
    rng = np.random.default_rng(5)
    h, m = 1e-3, 24

    def functional(p, a, j, i):
        sl = (slice(j - m, j + m + 1), slice(i - m, i + m + 1))
        return float(np.vdot(g[sl], O.forward(p[sl], a[sl], L, O.NONLOCAL)))

    checked = tried = 0
    worst = 0.0
    while checked < 64 and tried < 1000:
        tried += 1
        j, i = int(rng.integers(32, w.ny - 32)), int(rng.integers(32, w.nx - 32))
        e = np.zeros((2 * m + 1, 2 * m + 1))
        e[m, m] = h
        sl = (slice(j - m, j + m + 1), slice(i - m, i + m + 1))
        pw, aw = ph[sl].copy(), ab[sl].copy()
        f0 = functional(ph, ab, j, i)
        fp = float(np.vdot(g[sl], O.forward(pw + e, aw, L, O.NONLOCAL)))
        fm = float(np.vdot(g[sl], O.forward(pw - e, aw, L, O.NONLOCAL)))
        fwd, bwd = (fp - f0) / h, (f0 - fm) / h
        if abs(fwd - bwd) > 1e-6 * max(1.0, abs(fwd)):
            continue   # a kink inside [-h, h]
        fd = (fp - fm) / (2 * h)
        fa = (float(np.vdot(g[sl], O.forward(pw, aw + e, L, O.NONLOCAL))) -
              float(np.vdot(g[sl], O.forward(pw, aw - e, L, O.NONLOCAL)))) / (2 * h)
        rp = abs(gp[j, i] - fd) / abs(fd)
        ra = abs(ga[j, i] - fa) / abs(fa)
        worst = max(worst, rp, ra)
        assert rp <= 1e-4, (j, i, gp[j, i], fd)
        assert ra <= 1e-4, (j, i, ga[j, i], fa)
        checked += 1
    print(f"central differences: {checked} pixels ({tried} drawn), worst rel {worst:.2e}",
          flush=True)
    assert checked == 64


def test_refinement_full_size_follows_oracle(oracle_refs):
    # 50 Adam steps on 1/2 ||P(phase, absorb) - d||^2 at 2048^2 with 8 lines, ray maps
    # recomputed at every step (forward and backward); the GPU runs torch's Adam on float32
    # maps with the library's forward model and VJP, the oracle the same Adam in FP64
    import torch
    from paper_2601_22793_amd import epr_forward
    w, obj = vjp_case()
    geom, spec, _ = api_objects(w)
    d = oracle_refs.load("vjp-poly8-2048", "d")
    p0 = (F.ADAM_START[0] * obj["phase"]).astype(np.float32)
    a0 = (F.ADAM_START[1] * obj["absorb"]).astype(np.float32)
    phase = to_dev(p0).requires_grad_(True)
    absorb = to_dev(a0).requires_grad_(True)
    opt = torch.optim.Adam([{"params": [phase], "lr": F.ADAM_LR[0]},
                            {"params": [absorb], "lr": F.ADAM_LR[1]}])
    dd = to_dev(d)
    losses = []
    for _ in range(F.ADAM_STEPS):
        opt.zero_grad()
        P = epr_forward(phase, absorb, geom, spec)
        loss = 0.5 * ((P - dd).double() ** 2).sum()
        loss.backward()
        losses.append(float(loss.detach()))
        opt.step()
    ref = oracle_refs.load("vjp-poly8-2048", "losses")
    rel = np.abs(np.asarray(losses) - ref) / ref
    print(f"Adam 50 steps: loss {losses[0]:.4e} -> {losses[-1]:.4e}, worst per-step rel "
          f"{rel.max():.2e}", flush=True)
    assert losses[-1] < losses[0] and ref[-1] < ref[0]
    assert rel.max() <= 1e-4
    ep = rel_l2(to_np(phase), oracle_refs.load("vjp-poly8-2048", "phase"))
    ea = rel_l2(to_np(absorb), oracle_refs.load("vjp-poly8-2048", "absorb"))
    print(f"final maps rel L2: phase {ep:.2e}, absorption {ea:.2e}", flush=True)
    assert ep <= 1e-3 and ea <= 1e-3
