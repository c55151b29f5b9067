"""Seeded discrete polychromatic spectrum.

The paper discretises the beam spectrum into a small set of effective lines (Methods 4.3) but
gives no rule for choosing them.  The workload recipe used here: equal-width bins over
[e_lo, e_hi] keV, each represented by its centre energy and weighted by the integral of a smooth
bremsstrahlung-like shape over the bin,

    S(E) = max(E0 - E, 0) / E * exp(-(Ef / E)^3),

with the end-point energy E0 and the filtration knee Ef drawn from the seeded generator.  The
weights are normalised to sum to one.
"""

import numpy as np
from scipy.integrate import simpson


def bremsstrahlung_bins(n_bins, rng, e_lo=60.0, e_hi=160.0, e0_range=(170.0, 220.0),
                        ef_range=(30.0, 50.0), points_per_bin=65):
    """Return (centres_keV, weights) for `n_bins` equal bins of a seeded smooth spectrum.

    `rng` is a numpy Generator; it draws E0 then Ef, in that order.
    """
    if n_bins < 1:
        raise ValueError("n_bins must be >= 1")
    e0 = rng.uniform(*e0_range)
    ef = rng.uniform(*ef_range)
    edges = np.linspace(e_lo, e_hi, n_bins + 1)
    centres = 0.5 * (edges[:-1] + edges[1:])
    weights = np.empty(n_bins)
    for b in range(n_bins):
        e = np.linspace(edges[b], edges[b + 1], points_per_bin)
        s = np.maximum(e0 - e, 0.0) / e * np.exp(-(ef / e) ** 3)
        weights[b] = simpson(s, x=e)
    weights /= weights.sum()
    return centres, weights
