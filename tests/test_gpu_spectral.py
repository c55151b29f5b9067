"""Paganin-type preconditioner (row real FFT, column FFT with the fused filter, row inverse)
on the GPU against the FP64 oracle, at every transform length the workloads use."""

import numpy as np
import pytest

from oracle import epr_oracle as O
from synthetic import workload
from tests.helpers import api_objects, oracle_lines, rel_l2, requires_gpu, to_dev, to_np

pytestmark = [pytest.mark.gpu, requires_gpu]


def ctx():
    from paper_2601_22793_amd import Context
    return Context.get(0)


@pytest.mark.parametrize("shape,n_lines", [((256, 256), 8), ((90, 250), 1), ((2048, 2048), 1),
                                           ((2160, 2560), 1), ((1024, 1024), 2), ((30, 24), 3),
                                           ((4096, 64), 1), ((512, 4096), 1)])
def test_precondition_matches_oracle(shape, n_lines):
    print(f"precondition {shape} lines={n_lines}", flush=True)
    base = "nonlocal-poly8-2048" if n_lines > 1 else "nonlocal-mono-2048"
    w = workload(base, shape=shape)
    w.energies_kev, w.weights = w.energies_kev[:n_lines], w.weights[:n_lines] / w.weights[:n_lines].sum()
    geom, spec, mat = api_objects(w)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((n_lines,) + shape).astype(np.float32)
    x += 3.0  # non-zero mean: exercises the DC bin
    ref = O.precondition(x, oracle_lines(w))
    out = ctx().precondition(to_dev(x), geom, spec, mat)
    assert rel_l2(to_np(out), ref) <= 1e-5


def test_precondition_in_place():
    w = workload("nonlocal-poly8-2048", shape=(128, 96))
    geom, spec, mat = api_objects(w)
    x = np.random.default_rng(2).standard_normal((8, 128, 96)).astype(np.float32)
    ref = O.precondition(x, oracle_lines(w))
    t = to_dev(x)
    ctx().precondition(t, geom, spec, mat, out=t)
    assert rel_l2(to_np(t), ref) <= 1e-5
