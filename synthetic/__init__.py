"""Seeded synthetic inputs shared by the oracle tests, the HIP tests and the benchmark.

This package produces *inputs only*: phantom thickness/phase/absorption maps, the discrete
spectrum (energies and weights), Poisson noise and the workload descriptions.  It contains none
of the phase-retrieval method's arithmetic (no ray map, splat, interpolation, preconditioner or
update): both the oracle and the HIP library compute those on their own from these inputs.
"""

from .spectrum import bremsstrahlung_bins
from .phantoms import (
    ellipsoid_phantom,
    soft_bone_phantom,
    scale_thickness,
    poisson_counts,
)
from .workloads import Workload, workload, WORKLOADS, batch_workloads

__all__ = [
    "bremsstrahlung_bins",
    "ellipsoid_phantom",
    "soft_bone_phantom",
    "scale_thickness",
    "poisson_counts",
    "Workload",
    "workload",
    "WORKLOADS",
    "batch_workloads",
]
