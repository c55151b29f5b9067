"""Differentiable forward models: the hand-written vector-Jacobian products against the FP64
oracle's (non-local model and local closures) and against central finite differences of the
non-local model; the autograd wrapper; a short Adam refinement against the same refinement run
by the oracle."""

import numpy as np
import pytest

from oracle import epr_oracle as O
from synthetic import workload
from tests.helpers import api_objects, oracle_lines, rel_l2, requires_gpu, to_dev, to_np

pytestmark = [pytest.mark.gpu, requires_gpu]


def ctx():
    from paper_2601_22793_amd import Context
    return Context.get(0)


def case(shape=(96, 128), n_lines=8):
    base = "vjp-poly8-2048" if n_lines == 8 else "nonlocal-mono-2048"
    w = workload(base, shape=shape)
    return w, w.true_object()


@pytest.mark.parametrize("shape,n_lines", [((96, 128), 8), ((128, 120), 1)])
def test_vjp_matches_oracle(shape, n_lines):
    w, obj = case(shape, n_lines)
    geom, spec, _ = api_objects(w)
    L = oracle_lines(w)
    g = np.random.default_rng(3).standard_normal(shape).astype(np.float32)
    rp, ra = O.forward_vjp(obj["phase"], obj["absorb"], g, L)
    gp, ga = ctx().forward_vjp(to_dev(obj["phase"]), to_dev(obj["absorb"]), to_dev(g), geom,
                               spec)
    assert rel_l2(to_np(gp), rp) <= 1e-4
    assert rel_l2(to_np(ga), ra) <= 1e-4


def local_case(shape, n_lines):
    """The local workload recipe with a solver material of delta / beta = 10 (strongly varying
    intensity, so that every term of the second-order closure contributes)."""
    w = workload("local-mono-256", shape=shape, beta_ref=5e-8)
    if n_lines > 1:
        from synthetic import bremsstrahlung_bins
        w.energies_kev, w.weights = bremsstrahlung_bins(n_lines, np.random.default_rng(21))
    return w, w.true_object()


@pytest.mark.parametrize("model", ["local_l1", "local_l2"])
@pytest.mark.parametrize("shape,n_lines", [((96, 128), 8), ((90, 80), 1)])
def test_local_vjp_matches_oracle(model, shape, n_lines):
    w, obj = local_case(shape, n_lines)
    geom, spec, _ = api_objects(w)
    L = oracle_lines(w)
    g = np.random.default_rng(6).standard_normal(shape).astype(np.float32)
    rp, ra = O.forward_vjp(obj["phase"], obj["absorb"], g, L, model)
    if model == "local_l2":
        p1, a1 = O.forward_vjp(obj["phase"], obj["absorb"], g, L, "local_l1")
        # the second-order terms' part is well above the tolerance
        assert rel_l2(rp, p1) > 1e-3 and rel_l2(ra, a1) > 1e-3
    gp, ga = ctx().forward_vjp(to_dev(obj["phase"]), to_dev(obj["absorb"]), to_dev(g), geom,
                               spec, model)
    print(f"{model} {shape} x {n_lines}: rel L2 phase {rel_l2(to_np(gp), rp):.2e} "
          f"absorb {rel_l2(to_np(ga), ra):.2e}", flush=True)
    assert rel_l2(to_np(gp), rp) <= 1e-4
    assert rel_l2(to_np(ga), ra) <= 1e-4


def test_autograd_wrapper_local_model():
    import torch
    from paper_2601_22793_amd.api import epr_forward
    w, obj = local_case((64, 80), 8)
    geom, spec, _ = api_objects(w)
    phase = to_dev(obj["phase"]).requires_grad_(True)
    absorb = to_dev(obj["absorb"]).requires_grad_(True)
    g = to_dev(np.random.default_rng(7).standard_normal((64, 80)).astype(np.float32))
    (epr_forward(phase, absorb, geom, spec, "local_l2") * g).sum().backward()
    gp, ga = ctx().forward_vjp(phase.detach(), absorb.detach(), g, geom, spec, "local_l2")
    torch.cuda.synchronize()
    assert torch.equal(phase.grad, gp) and torch.equal(absorb.grad, ga)


def test_vjp_matches_central_differences():
    # central differences of <g, P(phase, absorb)> in FP64 (the oracle's forward model) at 64
    # seeded pixels >= 16 px from the edges, h = 1e-3; the model is piecewise linear in the
    # phase, so pixels whose one-sided differences disagree (a cell edge is crossed) are redrawn
    w, obj = case((96, 128), 8)
    geom, spec, _ = api_objects(w)
    L = oracle_lines(w)
    ph = obj["phase"].astype(np.float64)
    ab = obj["absorb"].astype(np.float64)
    g = np.random.default_rng(4).standard_normal(ph.shape)
    gp, ga = ctx().forward_vjp(to_dev(ph), to_dev(ab), to_dev(g), geom, spec)
    gp, ga = to_np(gp), to_np(ga)
    rng = np.random.default_rng(5)
    h = 1e-3

    def loss(p, a):
        return float(np.vdot(g, O.forward(p, a, L, O.NONLOCAL)))

    checked = tried = 0
    while checked < 64 and tried < 400:
        tried += 1
        j, i = rng.integers(16, 80), rng.integers(16, 112)
        e = np.zeros_like(ph)
        e[j, i] = h
        l0 = loss(ph, ab)
        lp, lm = loss(ph + e, ab), loss(ph - e, ab)
        fwd, bwd = (lp - l0) / h, (l0 - lm) / h
        if abs(fwd - bwd) > 1e-3 * max(1.0, abs(fwd)):
            continue
        fd = (lp - lm) / (2 * h)
        assert gp[j, i] == pytest.approx(fd, rel=2e-3, abs=2e-3 * np.abs(gp).max())
        fa = (loss(ph, ab + e) - loss(ph, ab - e)) / (2 * h)
        assert ga[j, i] == pytest.approx(fa, rel=2e-3, abs=1e-3 * np.abs(ga).max())
        checked += 1
    assert checked == 64


def test_autograd_backward_is_the_vjp():
    import torch
    from paper_2601_22793_amd import epr_forward
    w, obj = case((64, 96), 8)
    geom, spec, _ = api_objects(w)
    phase = to_dev(obj["phase"]).requires_grad_(True)
    absorb = to_dev(obj["absorb"]).requires_grad_(True)
    d = to_dev(np.full((64, 96), 0.9, dtype=np.float32))
    P = epr_forward(phase, absorb, geom, spec)
    loss = 0.5 * ((P - d) ** 2).sum()
    loss.backward()
    gp, ga = ctx().forward_vjp(phase.detach(), absorb.detach(), (P - d).detach().contiguous(),
                               geom, spec)
    assert torch.allclose(phase.grad, gp, rtol=1e-5, atol=1e-7)
    assert torch.allclose(absorb.grad, ga, rtol=1e-5, atol=1e-7)


def _adam(grad_fn, x0, lrs, n, b1=0.9, b2=0.999, eps=1e-8):
    """Plain Adam on a list of float64 arrays; returns the per-step losses and the final x."""
    xs = [x.copy() for x in x0]
    m = [np.zeros_like(x) for x in xs]
    v = [np.zeros_like(x) for x in xs]
    losses = []
    for t in range(1, n + 1):
        loss, gs = grad_fn(xs)
        losses.append(loss)
        for k in range(len(xs)):
            m[k] = b1 * m[k] + (1 - b1) * gs[k]
            v[k] = b2 * v[k] + (1 - b2) * gs[k] ** 2
            mh = m[k] / (1 - b1 ** t)
            vh = v[k] / (1 - b2 ** t)
            xs[k] -= lrs[k] * mh / (np.sqrt(vh) + eps)
    return losses, xs


def test_refinement_follows_the_oracle():
    # 10 Adam steps on L = 1/2 ||P(phase, absorb) - d||^2 from a perturbed start, ray maps
    # recomputed every step; GPU (torch Adam + library VJP) against the same Adam in FP64
    import torch
    from paper_2601_22793_amd import epr_forward
    w, obj = case((64, 96), 8)
    geom, spec, _ = api_objects(w)
    L = oracle_lines(w)
    # counting noise keeps the residual, and so every gradient, well above float32 rounding
    # (Adam normalises each gradient by its running size, so on noise-free data the exactly
    # zero background residual would let rounding decide the steps there)
    d = w.add_noise(O.forward(obj["phase"], obj["absorb"], L, O.NONLOCAL))
    p0 = (0.9 * obj["phase"]).astype(np.float32)
    a0 = (1.1 * obj["absorb"]).astype(np.float32)
    lr_p, lr_a, n = 1e-2, 1e-4, 10

    def oracle_step(xs):
        P = O.forward(xs[0], xs[1], L, O.NONLOCAL)
        r = P - d
        gp, ga = O.forward_vjp(xs[0], xs[1], r, L)
        return 0.5 * float(np.vdot(r, r)), [gp, ga]

    ref_losses, _ = _adam(oracle_step, [p0.astype(np.float64), a0.astype(np.float64)],
                          [lr_p, lr_a], n)
    phase = to_dev(p0).requires_grad_(True)
    absorb = to_dev(a0).requires_grad_(True)
    opt = torch.optim.Adam([{"params": [phase], "lr": lr_p}, {"params": [absorb], "lr": lr_a}])
    dd = to_dev(d)
    losses = []
    for _ in range(n):
        opt.zero_grad()
        P = epr_forward(phase, absorb, geom, spec)
        loss = 0.5 * ((P - dd).double() ** 2).sum()
        loss.backward()
        losses.append(float(loss.detach()))
        opt.step()
    assert losses[-1] < 0.7 * losses[0]   # the oracle reaches 0.56 of the start
    for a, b in zip(losses, ref_losses):
        assert a == pytest.approx(b, rel=1e-4)
