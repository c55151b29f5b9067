"""Workload descriptions: geometry, spectrum, solver material, model, iteration count and the
seeded true object (phase and absorption at the reference energy).

Workloads
---------
* ``local-mono-256``      256x256, one line at 60 keV, pixel 5 um, L = 1 m, local second-order
                          closure, 20 iterations, relaxation 1.  Object: 20 ellipsoids of one
                          material (delta 5e-7, beta 5e-10), scaled so the thickness is at most
                          2 mm and the largest displacement at most 0.5 px.  Noise-free data.
* ``nonlocal-mono-2048``  2048x2048, one line at 60 keV, pixel 10 um, L = 20 m, non-local ray-map
                          model, 30 iterations, relaxation 0.4.  Object: soft-tissue body
                          (delta 4e-7, beta 4e-10) with bone-like inclusions (delta 1.2e-6,
                          beta 1.2e-8), largest displacement 6 px.  Poisson noise, 1e4 photons/px.
* ``nonlocal-poly8-2048`` as above with 8 equal bins over 60-160 keV (seeded bremsstrahlung-like
                          weights), delta ~ E^-2, beta ~ E^-3; the object is scaled so the
                          lowest-energy line is displaced by at most 6 px.
* ``fibres-stress-256``   256x256 strong-shift stress object after the bamboo test of the
                          paper's Section 3.1: pixel 1.12 um, L = 0.25 m, 10 equal-weight lines
                          at 50, 55, ..., 95 keV (mean 72.5 keV), delta 4e-8 and beta 4e-11 at
                          60 keV, a bundle of 14 parallel fibres scaled so the lowest-energy line
                          is displaced by up to 32 px (most of the fibre region by more than
                          1 px).  Noise-free; non-local model, relaxation 0.4.
* ``batch64``             64 problems of mixed sizes (24 x 1024^2, 32 x 2048^2,
                          8 x 2160 rows x 2560 columns) in seeded order, each a seeded
                          soft/bone object with its own spectrum, scaled at L = 20 m and imaged
                          at a per-problem distance L ~ U[5, 20] m.

Every workload can be shrunk to another shape (``workload(name, shape=...)``) with the same
recipe; the tests use that for oracle-sized parity cases.
"""

from dataclasses import dataclass, field, replace

import numpy as np

from .phantoms import (ellipsoid_phantom, fibre_phantom, max_forward_difference, poisson_counts,
                       scale_thickness, soft_bone_phantom)
from .spectrum import bremsstrahlung_bins

HC_EV_M = 1.239841984e-6  # Planck constant times speed of light, eV*m


def wavenumber(energy_kev):
    return 2.0 * np.pi * (np.asarray(energy_kev, dtype=np.float64) * 1e3) / HC_EV_M


@dataclass
class Workload:
    name: str
    ny: int
    nx: int
    pixel_m: float
    distance_m: float
    energies_kev: np.ndarray
    weights: np.ndarray
    delta_ref: float          # solver material at the reference energy
    beta_ref: float
    model: str                # "local_l1" | "local_l2" | "nonlocal"
    n_iter: int
    relaxation: float
    seed: int
    photons: float = 0.0      # 0: noise-free data
    energy_ref_kev: float = 60.0
    delta_exponent: float = 2.0
    beta_exponent: float = 3.0
    truth: str = "soft_bone"  # "ellipsoids" | "soft_bone" | "fibres"
    max_shift_px: float = 6.0
    scale_distance_m: float = 0.0   # distance used to scale the phantom (0: distance_m)
    info: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.ny, self.nx)

    @property
    def n_lines(self):
        return int(len(self.energies_kev))

    def true_object(self):
        """Return dict(phase, absorb, tau_soft, tau_bone) at the reference energy.

        phase and absorb are float32 [ny][nx]: phase = -k (delta_soft tau_soft + delta_bone
        tau_bone), absorb = 2 k (beta_soft tau_soft + beta_bone tau_bone).
        """
        rng = np.random.default_rng(self.seed)
        k = float(wavenumber(self.energy_ref_kev))
        e_min = float(np.min(self.energies_kev))
        # displacement grows as delta_s ~ (E_ref/E)^delta_exponent: scale at the lowest line
        line_factor = (self.energy_ref_kev / e_min) ** self.delta_exponent
        ldist = self.scale_distance_m or self.distance_m
        p2 = self.pixel_m ** 2
        if self.truth == "ellipsoids":
            tau = ellipsoid_phantom(self.shape, rng, centre_range=(0.125 * min(self.shape),
                                                                   0.875 * min(self.shape)))
            shift_per_grad = ldist * self.delta_ref * line_factor / p2
            tau, s = scale_thickness(tau, 2.0e-3, self.max_shift_px / shift_per_grad)
            self.info["scale"] = s
            phase = -k * self.delta_ref * tau
            absorb = 2.0 * k * self.beta_ref * tau
            soft, bone = tau, np.zeros_like(tau)
        elif self.truth == "fibres":
            tau = fibre_phantom(self.shape, rng)
            shift_per_grad = ldist * self.delta_ref * line_factor / p2
            s = self.max_shift_px / (shift_per_grad * max_forward_difference(tau))
            tau = tau * s
            self.info["scale"] = s
            phase = -k * self.delta_ref * tau
            absorb = 2.0 * k * self.beta_ref * tau
            soft, bone = tau, np.zeros_like(tau)
        else:
            d_soft, b_soft = 4.0e-7, 4.0e-10
            d_bone, b_bone = 1.2e-6, 1.2e-8
            soft, bone, info = soft_bone_phantom(
                self.shape, rng, self.pixel_m,
                shift_per_grad_soft=ldist * d_soft * line_factor / p2,
                shift_per_grad_bone=ldist * d_bone * line_factor / p2,
                target_max_shift_px=self.max_shift_px,
                soft_max_shift_px=min(4.0, self.max_shift_px))
            self.info.update(info)
            phase = -k * (d_soft * soft + d_bone * bone)
            absorb = 2.0 * k * (b_soft * soft + b_bone * bone)
        return {
            "phase": phase.astype(np.float32),
            "absorb": absorb.astype(np.float32),
            "tau_soft": soft,
            "tau_bone": bone,
        }

    def add_noise(self, intensity):
        """Counting noise of the workload (or a float32 copy when noise-free)."""
        if not self.photons:
            return np.asarray(intensity, dtype=np.float32).copy()
        rng = np.random.default_rng(self.seed + 500)
        return poisson_counts(intensity, self.photons, rng).astype(np.float32)


def _spectrum(n_lines, seed):
    if n_lines == 1:
        return np.array([60.0]), np.array([1.0])
    return bremsstrahlung_bins(n_lines, np.random.default_rng(seed + 77))


def _base(name):
    if name == "local-mono-256":
        return Workload(name, 256, 256, 5e-6, 1.0, np.array([60.0]), np.array([1.0]),
                        5e-7, 5e-10, "local_l2", 20, 1.0, seed=1000, truth="ellipsoids",
                        max_shift_px=0.5)
    if name == "nonlocal-mono-2048":
        return Workload(name, 2048, 2048, 10e-6, 20.0, np.array([60.0]), np.array([1.0]),
                        4e-7, 4e-10, "nonlocal", 30, 0.4, seed=2000, photons=1e4)
    if name == "nonlocal-poly8-2048":
        e, w = _spectrum(8, 3000)
        return Workload(name, 2048, 2048, 10e-6, 20.0, e, w, 4e-7, 4e-10, "nonlocal", 30, 0.4,
                        seed=3000, photons=1e4)
    if name == "vjp-poly8-2048":
        e, w = _spectrum(8, 5000)
        return Workload(name, 2048, 2048, 10e-6, 20.0, e, w, 4e-7, 4e-10, "nonlocal", 50, 0.4,
                        seed=5000, photons=1e4)
    if name == "fibres-stress-256":
        e = np.arange(50.0, 96.0, 5.0)
        return Workload(name, 256, 256, 1.12e-6, 0.25, e, np.full(10, 0.1), 4e-8, 4e-11,
                        "nonlocal", 5, 0.4, seed=6000, truth="fibres", max_shift_px=32.0)
    raise KeyError(name)


WORKLOADS = ("local-mono-256", "nonlocal-mono-2048", "nonlocal-poly8-2048", "vjp-poly8-2048",
             "fibres-stress-256")


def workload(name, shape=None, **overrides):
    """Named workload, optionally at another shape (same recipe) or with fields overridden."""
    w = _base(name)
    if shape is not None:
        w = replace(w, ny=int(shape[0]), nx=int(shape[1]), info={})
    if overrides:
        w = replace(w, **overrides)
    return w


BATCH_SIZES = ((24, (1024, 1024)), (32, (2048, 2048)), (8, (2160, 2560)))


def batch_workloads(n_lines=8, seed=4000, sizes=BATCH_SIZES, n_iter=30):
    """The mixed-size batch: list of Workload, seeded order and per-problem distance."""
    shapes = []
    for count, shp in sizes:
        shapes += [shp] * count
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(shapes))
    dists = rng.uniform(5.0, 20.0, size=len(shapes))
    out = []
    for i, j in enumerate(order):
        e, w = _spectrum(n_lines, seed + 1 + i)
        out.append(Workload(f"batch-{i}", shapes[j][0], shapes[j][1], 10e-6, float(dists[i]), e, w,
                            4e-7, 4e-10, "nonlocal", n_iter, 0.4, seed=seed + 1 + i,
                            photons=1e4, scale_distance_m=20.0))
    return out
