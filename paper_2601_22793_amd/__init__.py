"""Fast eikonal phase retrieval (EPR) on MI355X (gfx950).

The iteration of Mirone et al. (arXiv:2601.22793) -- local O(L^2) closure or non-local ray-map
splat, spectral sum, exact bilinear adjoint, FFT-diagonal Paganin-type preconditioner and
single-thickness projection -- runs in the hand-written HIP kernels of libepr.so behind the C
ABI of include/epr.h.  This package is its torch binding.
"""

from .api import (  # noqa: F401
    Context,
    EPRForward,
    EPRForwardXspec,
    Geometry,
    Material,
    MODELS,
    Spectrum,
    SpectrumProfile,
    epr_forward,
    epr_forward_xspec,
)
from ._lib import EprError, LIB_PATH  # noqa: F401
