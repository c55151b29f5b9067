"""Shared test helpers: workload -> oracle constants / binding objects, norms, device checks."""

import numpy as np
import pytest

from oracle import epr_oracle as O


def has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


requires_gpu = pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")


def oracle_lines(w, geom_distance=None):
    return O.line_constants(w.energies_kev, w.weights, w.pixel_m,
                            w.distance_m if geom_distance is None else geom_distance,
                            w.delta_ref, w.beta_ref, w.energy_ref_kev, w.delta_exponent,
                            w.beta_exponent)


def api_objects(w):
    from paper_2601_22793_amd import Geometry, Material, Spectrum
    return (Geometry(w.ny, w.nx, w.pixel_m, w.distance_m),
            Spectrum(list(map(float, w.energies_kev)), list(map(float, w.weights)),
                     w.energy_ref_kev, w.delta_exponent, w.beta_exponent),
            Material(w.delta_ref, w.beta_ref))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)
