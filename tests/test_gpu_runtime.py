"""Runtime behaviour of the solvers on the GPU: failure detection (non-finite updates), the
graph-replayed single-problem solve against its eagerly enqueued launch sequence, the batched
solver's residual history in the caller's order, batches of different problems alternating on a
side stream, and calls from two torch streams kept in order by the binding."""

import numpy as np
import pytest

from oracle import epr_oracle as O
from synthetic import bremsstrahlung_bins, workload
from tests.helpers import api_objects, oracle_lines, rel_l2, requires_gpu, to_dev, to_np

pytestmark = [pytest.mark.gpu, requires_gpu]


def ctx():
    from paper_2601_22793_amd import Context
    return Context.get(0)


def case(shape, seed=0, n_iter=4, distance=20.0):
    w = workload("nonlocal-poly8-2048", shape=shape, distance_m=distance, scale_distance_m=20.0,
                 n_iter=n_iter)
    w.seed += seed
    e, wt = bremsstrahlung_bins(8, np.random.default_rng(200 + seed))
    w.energies_kev, w.weights = e, wt
    obj = w.true_object()
    L = oracle_lines(w)
    d = w.add_noise(O.forward(obj["phase"], obj["absorb"], L, O.NONLOCAL))
    return w, d, L


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("model", ["nonlocal", "local_l2"])
def test_nonfinite_data_is_flagged(bad, model):
    # (a short distance keeps the shifts sub-pixel, where the local closure holds)
    w, d, _ = case((64, 80), distance=2.0)
    geom, spec, mat = api_objects(w)
    c = ctx()
    c.solve(to_dev(d), geom, spec, mat, model, 3, 0.4)
    diag = c.diagnostics()
    assert diag["nonfinite"] == 0 and diag["first_nonfinite"] == -1
    d2 = d.copy()
    d2[30, 40] = bad
    print(f"non-finite data {bad} model {model}", flush=True)
    c.solve(to_dev(d2), geom, spec, mat, model, 3, 0.4)
    diag = c.diagnostics()
    assert diag["nonfinite"] == 1 and diag["first_nonfinite"] == 0
    # the next clean solve clears the flag
    c.solve(to_dev(d), geom, spec, mat, model, 3, 0.4)
    assert c.diagnostics()["nonfinite"] == 0


def test_nonpositive_data_is_floored_not_flagged():
    w, d, L = case((64, 80))
    d2 = d.copy()
    d2[20:30, 10:40] = -0.5
    d2[40:44, 50:60] = 0.0
    geom, spec, mat = api_objects(w)
    c = ctx()
    tau = c.solve(to_dev(d2), geom, spec, mat, "nonlocal", 3, 0.4)
    assert c.diagnostics()["nonfinite"] == 0
    ref = O.solve(d2, L, O.NONLOCAL, 3, 0.4)
    assert rel_l2(to_np(tau), ref) <= 1e-4


def test_nonfinite_flag_names_the_batched_problem():
    import torch
    batch = [case((64, 80), seed=i) for i in range(3)]
    probs = []
    for i, (w, d, _) in enumerate(batch):
        geom, spec, mat = api_objects(w)
        dd = d.copy()
        if i == 2:
            dd[5, 5] = np.nan
        probs.append((to_dev(dd), torch.zeros((w.ny, w.nx), device="cuda"), geom, spec, mat))
    c = ctx()
    c.solve_batched(probs, "nonlocal", 3, 0.4)
    diag = c.diagnostics()
    assert diag["nonfinite"] == 1 and diag["first_nonfinite"] == 2
    for i in (0, 1):
        assert np.all(np.isfinite(to_np(probs[i][1])))


@pytest.mark.parametrize("model,relax", [("nonlocal", 0.4), ("local_l2", 1.0),
                                         ("nonlocal_l2", 0.4)])
def test_solve_graph_replays_equal_the_eager_sequence(model, relax):
    # timing on: the iterations are enqueued directly; timing off: captured once, replayed
    import torch
    w, d, _ = case((96, 128))
    geom, spec, mat = api_objects(w)
    c = ctx()
    dd = to_dev(d)
    c.set_timing(True)
    eager = to_np(c.solve(dd, geom, spec, mat, model, 5, relax))
    c.set_timing(False)
    for rep in range(3):
        scratch = torch.randn(1 << 18, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        got = to_np(c.solve(dd, geom, spec, mat, model, 5, relax))
        assert np.array_equal(got, eager), rep
        del scratch


def test_batched_residual_history_is_problem_zero_in_caller_order():
    import torch
    # problem 0 is the larger one: the solver sorts problems by size class internally
    batch = [case((256, 2560), seed=0, n_iter=5), case((64, 80), seed=1, n_iter=5)]
    probs = []
    for w, d, _ in batch:
        geom, spec, mat = api_objects(w)
        probs.append((to_dev(d), torch.zeros((w.ny, w.nx), device="cuda"), geom, spec, mat))
    c = ctx()
    c.solve_batched(probs, "nonlocal", 5, 0.4, residuals=True)
    hist_b = c.diagnostics()["residual"]
    w, d, L = batch[0]
    ref = []
    O.solve(d, L, O.NONLOCAL, 5, 0.4, history=ref)
    assert len(hist_b) == 5
    np.testing.assert_allclose(hist_b, ref, rtol=1e-4)


def test_alternating_batches_on_a_side_stream():
    import torch
    a = [case((64, 80), seed=i) for i in range(2)]
    b = [case((96, 64), seed=10 + i) for i in range(3)]

    def probs_of(batch):
        out = []
        for w, d, _ in batch:
            geom, spec, mat = api_objects(w)
            out.append((to_dev(d), torch.zeros((w.ny, w.nx), device="cuda"), geom, spec, mat))
        return out

    pa, pb = probs_of(a), probs_of(b)
    c = ctx()
    singles = [to_np(c.solve(p[0], p[2], p[3], p[4], "nonlocal", 4, 0.4)) for p in pa + pb]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for rep in range(3):
            for p in pa + pb:
                p[1].zero_()
            c.solve_batched(pa, "nonlocal", 4, 0.4)
            c.solve_batched(pb, "nonlocal", 4, 0.4)
    side.synchronize()
    for ref, p in zip(singles, pa + pb):
        assert rel_l2(to_np(p[1]), ref) <= 1e-5


def test_calls_from_two_torch_streams_stay_ordered():
    # a long solve on one torch stream, then a forward model on another: the binding makes the
    # second stream wait for the first, since both calls use the handle's workspace
    import torch
    w, d, _ = case((512, 512), n_iter=30)
    geom, spec, mat = api_objects(w)
    obj = w.true_object()
    c = ctx()
    dd = to_dev(d)
    ref = to_np(c.solve(dd, geom, spec, mat, "nonlocal", 30, 0.4))
    fwd_ref = to_np(c.forward(to_dev(obj["phase"]), to_dev(obj["absorb"]), geom, spec))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ph, ab = to_dev(obj["phase"]), to_dev(obj["absorb"])
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        tau = c.solve(dd, geom, spec, mat, "nonlocal", 30, 0.4)
    with torch.cuda.stream(s2):
        fwd = c.forward(ph, ab, geom, spec)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(tau), ref)
    np.testing.assert_array_equal(to_np(fwd), fwd_ref)
