"""FP64 oracle references of the full-size parity tests (test infrastructure).

Each case runs in its own CPU-only process (numpy and the oracle; never torch or the GPU),
started by the test session so that the minutes of FP64 work overlap the GPU tests:

    python -m tests.fullsize_oracle CASE OUTDIR

A case writes its arrays to OUTDIR/CASE.<name>.npy as soon as each is ready (the data first,
so the GPU side can start) and OUTDIR/CASE.done last.  Every stored value comes from the oracle
and the seeded input generators only.

Cases (the workloads are the configurations' seeded synthetic stand-ins):
  nonlocal-mono-2048     one 2048^2 projection, 1 line, non-local, 30 iterations, omega 0.4
  nonlocal-poly8-2048    one 2048^2 projection, 8 lines, non-local, 30 iterations, omega 0.4
  batch-<i>              problem i of the 64-problem mixed batch (8 lines, 30 iterations)
  vjp-poly8-2048         the vector-Jacobian product at 2048^2 with 8 lines for a seeded
                         cotangent, and 50 steps of Adam on 1/2 ||P(phase, absorb) - d||^2
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import epr_oracle as O  # noqa: E402
from synthetic import batch_workloads, workload  # noqa: E402

N_ITER = 30
ADAM_STEPS = 50
ADAM_LR = (1e-2, 1e-4)      # phase [rad], absorption [optical depth]
ADAM_START = (0.9, 1.1)     # start: the true maps scaled by these factors
VJP_SEED = 11


def lines_of(w):
    return O.line_constants(w.energies_kev, w.weights, w.pixel_m, w.distance_m, w.delta_ref,
                            w.beta_ref, w.energy_ref_kev, w.delta_exponent, w.beta_exponent)


def batch_indices():
    """Index of the first problem of each shape in the 64-problem batch (seeded order)."""
    out = {}
    for i, w in enumerate(batch_workloads()):
        out.setdefault(w.shape, i)
    return out


def case_workload(case):
    if case.startswith("batch-"):
        return batch_workloads()[int(case.split("-")[1])]
    return workload(case)


def data_of(w):
    """Detector data of a workload: the oracle's forward model of the seeded true object, with
    the workload's counting noise, rounded to float32 once (both sides read this array)."""
    obj = w.true_object()
    return w.add_noise(O.forward(obj["phase"], obj["absorb"], lines_of(w), w.model)), obj


def adam(grad_fn, x0, lrs, n, b1=0.9, b2=0.999, eps=1e-8):
    """Plain Adam on float64 arrays; returns the per-step losses and the final arrays."""
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


def vjp_cotangent(shape):
    return np.random.default_rng(VJP_SEED).standard_normal(shape).astype(np.float32)


def run(case, outdir):
    t0 = time.time()

    def save(name, arr):
        tmp = os.path.join(outdir, f"{case}.{name}.tmp.npy")
        np.save(tmp, arr)
        os.replace(tmp, os.path.join(outdir, f"{case}.{name}.npy"))

    info = {"case": case}
    w = case_workload(case)
    L = lines_of(w)
    if case == "vjp-poly8-2048":
        obj = w.true_object()
        g = vjp_cotangent(w.shape)
        gp, ga = O.forward_vjp(obj["phase"], obj["absorb"], g, L)
        save("grad_phase", gp)
        save("grad_absorb", ga)
        info["vjp_s"] = time.time() - t0
        # the data of the refinement: the true object's image with the workload's counting
        # noise.  (With noise-free data the residual is exactly zero over the flat background,
        # and Adam, which divides by the root of the running squared gradient, turns the
        # rounding-level gradients a float32 evaluation leaves there into full-size steps: a
        # float32 trajectory then cannot follow the FP64 one.)
        d = w.add_noise(O.forward(obj["phase"], obj["absorb"], L, O.NONLOCAL))
        save("d", d)
        x0 = [(ADAM_START[0] * obj["phase"]).astype(np.float32).astype(np.float64),
              (ADAM_START[1] * obj["absorb"]).astype(np.float32).astype(np.float64)]

        def step(xs):
            r = O.forward(xs[0], xs[1], L, O.NONLOCAL) - d
            gph, gab = O.forward_vjp(xs[0], xs[1], r, L)
            return 0.5 * float(np.vdot(r, r)), [gph, gab]

        losses, xs = adam(step, x0, ADAM_LR, ADAM_STEPS)
        save("losses", np.asarray(losses))
        save("phase", xs[0])
        save("absorb", xs[1])
    else:
        d, _ = data_of(w)
        save("d", d)
        hist = []
        tau = O.solve(d, L, w.model, N_ITER, w.relaxation, history=hist)
        save("tau", tau)
        save("history", np.asarray(hist))
    info["seconds"] = time.time() - t0
    with open(os.path.join(outdir, f"{case}.done"), "w") as fh:
        json.dump(info, fh)


if __name__ == "__main__":
    run(sys.argv[1], sys.argv[2])
