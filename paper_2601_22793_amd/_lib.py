"""ctypes declarations of libepr.so (include/epr.h).  Argument marshalling only."""

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# EPR_LIBRARY names another build of the same library (the host AddressSanitizer build the
# ABI tests run against); by default the one in the package directory.
LIB_PATH = os.environ.get("EPR_LIBRARY") or os.path.join(_PKG, "libepr.so")

EPR_OK = 0
EPR_ERR_INVALID_ARG = -1
EPR_ERR_SHAPE = -2
EPR_ERR_NO_DEVICE = -3
EPR_ERR_HIP = -4
EPR_ERR_OOM = -5
EPR_ERR_UNSUPPORTED = -6
EPR_ERR_NONFINITE = -7

EPR_AUTO, EPR_LOCAL_L1, EPR_LOCAL_L2, EPR_NONLOCAL, EPR_NONLOCAL_L2 = 0, 1, 2, 3, 4
EPR_AUTO_MAX_FRACTION = 0.01
EPR_MAX_BINS = 1023
EPR_FLAG_RESIDUALS = 1
EPR_FLAG_BLOCK_PRECOND = 2
EPR_MAX_PRECOND_BLOCKS = 8
EPR_MAX_LINES = 16
EPR_NOALLOC_SCRATCH_BYTES = 128 << 20


class Geometry(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("pixel_m", C.c_double),
                ("distance_m", C.c_double)]


class Spectrum(C.Structure):
    _fields_ = [("n_lines", C.c_int32), ("energy_kev", C.POINTER(C.c_double)),
                ("weight", C.POINTER(C.c_double)), ("energy_ref_kev", C.c_double),
                ("delta_exponent", C.c_double), ("beta_exponent", C.c_double)]


class SpectrumProfile(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("block_x", C.POINTER(C.c_double)),
                ("energy_kev", C.POINTER(C.c_double)), ("weight", C.POINTER(C.c_double))]


class Material(C.Structure):
    _fields_ = [("delta_ref", C.c_double), ("beta_ref", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("model", C.c_int32), ("n_iter", C.c_int32), ("relaxation", C.c_double),
                ("flags", C.c_uint32), ("oversample", C.c_int32)]


class Problem(C.Structure):
    _fields_ = [("geom", Geometry), ("spec", Spectrum), ("mat", Material),
                ("intensity", C.c_void_p), ("thickness", C.c_void_p)]


class Diagnostics(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("n_problems", C.c_int32), ("model", C.c_int32),
                ("max_shift_px", C.c_float),
                ("residual", C.c_float * 256),
                ("nonfinite", C.c_int32), ("first_nonfinite", C.c_int32)]


N_STAGES = 8
STAGE_NAMES = ("maxgrad", "splat", "local", "rowfft", "colfft", "rowinv", "vjp", "binsplit")


class Timing(C.Structure):
    _fields_ = [("ms", C.c_double * N_STAGES), ("launches", C.c_int64 * N_STAGES),
                ("ms_class", (C.c_double * 2) * N_STAGES),
                ("launches_class", (C.c_int64 * 2) * N_STAGES)]


_h = C.c_void_p
_p = C.c_void_p
PROTOTYPES = {
    "epr_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "epr_destroy": (C.c_int, [_h]),
    "epr_status_string": (C.c_char_p, [C.c_int]),
    "epr_last_error": (C.c_char_p, [_h]),
    "epr_forward": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum), C.c_int, _p, _p, _p,
                              _p]),
    "epr_adjoint": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum), C.c_int, _p, _p, _p,
                              _p]),
    "epr_forward_oversampled": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum), C.c_int,
                                          C.c_int32, _p, _p, _p, _p]),
    "epr_adjoint_oversampled": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum), C.c_int,
                                          C.c_int32, _p, _p, _p, _p]),
    "epr_precondition": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum),
                                   C.POINTER(Material), _p, _p, _p]),
    "epr_regime": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum), C.POINTER(Material),
                             _p, C.c_int32, C.c_double, _p, _p]),
    "epr_select_model": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum),
                                   C.POINTER(Material), _p, C.c_double, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_uint32), _p]),
    "epr_solve": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum), C.POINTER(Material),
                            C.POINTER(Opts), _p, _p, _p, _p]),
    "epr_solve_noalloc": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum),
                                    C.POINTER(Material), C.POINTER(Opts), _p, _p, _p, _p]),
    "epr_solve_xspec": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum),
                                  C.POINTER(SpectrumProfile), C.POINTER(Material),
                                  C.POINTER(Opts), _p, _p, _p, _p]),
    "epr_solve_batched": (C.c_int, [_h, C.c_int32, C.POINTER(Problem), C.POINTER(Opts), _p]),
    "epr_solve_batched_xspec": (C.c_int, [_h, C.c_int32, C.POINTER(Problem),
                                          C.POINTER(SpectrumProfile), C.POINTER(Opts), _p]),
    "epr_forward_xspec": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum),
                                    C.POINTER(SpectrumProfile), C.POINTER(Material), C.c_int,
                                    _p, _p, _p]),
    "epr_adjoint_xspec": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum),
                                    C.POINTER(SpectrumProfile), C.POINTER(Material), C.c_int,
                                    _p, _p, _p, _p]),
    "epr_forward_vjp": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum), C.c_int, _p, _p,
                                  _p, _p, _p, _p]),
    "epr_forward_vjp_oversampled": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum),
                                              C.c_int, C.c_int32, _p, _p, _p, _p, _p, _p]),
    "epr_forward_xspec_vjp": (C.c_int, [_h, C.POINTER(Geometry), C.POINTER(Spectrum),
                                        C.POINTER(SpectrumProfile), C.POINTER(Material),
                                        C.c_int, _p, _p, _p, _p]),
    "epr_get_diagnostics": (C.c_int, [_h, C.POINTER(Diagnostics)]),
    "epr_autotune": (C.c_int, [_h, C.c_int32, C.POINTER(Problem), C.POINTER(Opts), C.c_char_p]),
    "epr_set_timing": (C.c_int, [_h, C.c_int]),
    "epr_get_timing": (C.c_int, [_h, C.POINTER(Timing)]),
    "epr_fft_plan": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.c_int32]),
    "epr_check_problem": (C.c_int, [C.POINTER(Geometry), C.POINTER(Spectrum),
                                    C.POINTER(Material), C.POINTER(Opts), C.c_char_p, C.c_size_t]),
}

_lib = None


def load():
    """Load libepr.so (built by paper_2601_22793_amd.build; LIB_PATH)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2601_22793_amd.build` "
            "(the EPR path has no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class EprError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"EPR error {status}: {message}")
        self.status = status
