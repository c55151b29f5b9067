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
                                           ((4096, 64), 1), ((512, 4096), 1), ((2304, 96), 2),
                                           ((2250, 64), 1)])
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


@pytest.mark.parametrize("shape,n_lines", [((2048, 2048), 8), ((2160, 2560), 8), ((4096, 4096), 1)])
def test_precondition_matches_the_library_fft(shape, n_lines):
    # cross-check at full size against the vendor FFT (torch.fft, i.e. rocFFT) in float32: the
    # same filter 1 / (1 + 4 pi^2 alpha_s (fx^2 + fy^2)) applied by an independent transform
    import torch
    print(f"library fft cross-check {shape} lines={n_lines}", flush=True)
    base = "nonlocal-poly8-2048" if n_lines > 1 else "nonlocal-mono-2048"
    w = workload(base, shape=shape)
    L = oracle_lines(w)
    geom, spec, mat = api_objects(w)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    x = torch.randn((n_lines,) + shape, generator=g, device="cuda", dtype=torch.float32) + 3.0
    out = ctx().precondition(x, geom, spec, mat)
    ny, nx = shape
    fy = torch.fft.fftfreq(ny, device="cuda", dtype=torch.float64)[:, None]
    fx = torch.fft.rfftfreq(nx, device="cuda", dtype=torch.float64)[None, :]
    for s in range(n_lines):
        filt = (1.0 / (1.0 + 4 * np.pi ** 2 * L.alpha_px[s] * (fx ** 2 + fy ** 2))).float()
        ref = torch.fft.irfft2(torch.fft.rfft2(x[s]) * filt, s=shape)
        err = float(torch.linalg.norm(out[s] - ref) / torch.linalg.norm(ref))
        assert err <= 1e-5, (s, err)
