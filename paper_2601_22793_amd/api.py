"""Thin torch binding of libepr: the same entry points as include/epr.h.

torch supplies device memory and the current HIP stream; every step of the EPR path runs in
the library's kernels.  There is no CPU fallback: without libepr.so or a gfx950 device the
calls raise.
"""

import ctypes as C
from dataclasses import dataclass
from typing import Sequence

import numpy as np
import torch

from . import _lib as L

MODELS = {"auto": L.EPR_AUTO, "local_l1": L.EPR_LOCAL_L1, "local_l2": L.EPR_LOCAL_L2,
          "nonlocal": L.EPR_NONLOCAL, "nonlocal_l2": L.EPR_NONLOCAL_L2}
MODEL_NAMES = {v: k for k, v in MODELS.items()}


@dataclass
class Geometry:
    ny: int
    nx: int
    pixel_m: float
    distance_m: float

    def c(self):
        return L.Geometry(self.ny, self.nx, self.pixel_m, self.distance_m)


@dataclass
class Spectrum:
    energies_kev: Sequence[float]
    weights: Sequence[float]
    energy_ref_kev: float = 60.0
    delta_exponent: float = 2.0
    beta_exponent: float = 3.0

    def c(self):
        e = np.ascontiguousarray(self.energies_kev, dtype=np.float64)
        w = np.ascontiguousarray(self.weights, dtype=np.float64)
        s = L.Spectrum(len(e), e.ctypes.data_as(C.POINTER(C.c_double)),
                       w.ctypes.data_as(C.POINTER(C.c_double)), self.energy_ref_kev,
                       self.delta_exponent, self.beta_exponent)
        s._keep = (e, w)  # keep the host arrays alive with the struct
        return s

    @property
    def n_lines(self):
        return len(self.energies_kev)


@dataclass
class SpectrumProfile:
    """x-dependent effective spectrum: line energies and weights on column blocks centred on
    block_x (detector columns, increasing); energies and weights are [n_blocks][n_lines]."""
    block_x: Sequence[float]
    energies_kev: Sequence[Sequence[float]]
    weights: Sequence[Sequence[float]]

    def c(self):
        x = np.ascontiguousarray(self.block_x, dtype=np.float64)
        e = np.ascontiguousarray(self.energies_kev, dtype=np.float64)
        w = np.ascontiguousarray(self.weights, dtype=np.float64)
        if e.shape != w.shape or e.ndim != 2 or e.shape[0] != x.size:
            raise ValueError("energies and weights must be [n_blocks][n_lines]")
        pr = L.SpectrumProfile(x.size, x.ctypes.data_as(C.POINTER(C.c_double)),
                               e.ctypes.data_as(C.POINTER(C.c_double)),
                               w.ctypes.data_as(C.POINTER(C.c_double)))
        pr._keep = (x, e, w)
        return pr


@dataclass
class Material:
    delta_ref: float
    beta_ref: float

    def c(self):
        return L.Material(self.delta_ref, self.beta_ref)


def _model(m):
    return MODELS[m] if isinstance(m, str) else int(m)


def _dev(t, name, shape=None):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on a HIP device")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


class Context:
    """One library handle on one device.  Its calls share a workspace; each runs on the current
    torch stream, after the previous call's stream (see _st)."""

    _cache = {}

    def __init__(self, device=0):
        self.lib = L.load()
        if isinstance(device, torch.device):
            device = device.index or 0
        self.device = int(device)
        h = C.c_void_p()
        st = self.lib.epr_create(C.byref(h), self.device)
        if st != L.EPR_OK:
            raise L.EprError(st, self.lib.epr_last_error(None).decode())
        self.h = h
        self._last = None   # torch stream of the previous call

    @classmethod
    def get(cls, device=0):
        if isinstance(device, torch.device):
            device = device.index or 0
        if device not in cls._cache:
            cls._cache[device] = cls(device)
        return cls._cache[device]

    def close(self):
        if self.h:
            self.lib.epr_destroy(self.h)
            self.h = None

    def _check(self, st):
        if st != L.EPR_OK:
            raise L.EprError(st, self.lib.epr_last_error(self.h).decode())

    def _tdev(self):
        return torch.device("cuda", self.device)

    def _st(self):
        """The current torch stream, as the call's stream.  The handle's workspace is shared by
        its calls, which the library requires to be ordered on one stream: when the current
        stream differs from the previous call's, it first waits (on the device, no host
        synchronisation) for the work enqueued there."""
        cur = torch.cuda.current_stream(self.device)
        if self._last is not None and self._last != cur:
            cur.wait_stream(self._last)
        self._last = cur
        return C.c_void_p(cur.cuda_stream)

    # -- entry points ---------------------------------------------------------------------------
    def forward(self, phase, absorb, geom: Geometry, spec: Spectrum, model="nonlocal", out=None):
        shape = (geom.ny, geom.nx)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self._tdev())
        g, s = geom.c(), spec.c()
        self._check(self.lib.epr_forward(self.h, C.byref(g), C.byref(s), _model(model),
                                         _dev(phase, "phase", shape), _dev(absorb, "absorb", shape),
                                         _dev(out, "intensity", shape), self._st()))
        return out

    def adjoint(self, phase, resid_lines, geom, spec, model="nonlocal", out=None):
        shape = (spec.n_lines, geom.ny, geom.nx)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self._tdev())
        g, s = geom.c(), spec.c()
        self._check(self.lib.epr_adjoint(self.h, C.byref(g), C.byref(s), _model(model),
                                         _dev(phase, "phase", shape[1:]),
                                         _dev(resid_lines, "resid_lines", shape),
                                         _dev(out, "obj_lines", shape), self._st()))
        return out

    def forward_oversampled(self, phase, absorb, geom: Geometry, spec: Spectrum, oversample,
                            model="nonlocal"):
        """Detector intensity [ny][nx] of maps on the oversampled internal grid
        [f ny][f nx] (geom is the detector)."""
        f = int(oversample)
        ishape = (geom.ny * f, geom.nx * f)
        out = torch.empty((geom.ny, geom.nx), dtype=torch.float32, device=self._tdev())
        g, s = geom.c(), spec.c()
        self._check(self.lib.epr_forward_oversampled(self.h, C.byref(g), C.byref(s), _model(model),
                                                     f, _dev(phase, "phase", ishape),
                                                     _dev(absorb, "absorb", ishape),
                                                     _dev(out, "intensity", (geom.ny, geom.nx)),
                                                     self._st()))
        return out

    def adjoint_oversampled(self, phase, resid_lines, geom: Geometry, spec: Spectrum, oversample,
                            model="nonlocal"):
        """Exact adjoint of forward_oversampled per line: [L][ny][nx] -> [L][f ny][f nx]."""
        f = int(oversample)
        ishape = (geom.ny * f, geom.nx * f)
        out = torch.empty((spec.n_lines,) + ishape, dtype=torch.float32, device=self._tdev())
        g, s = geom.c(), spec.c()
        self._check(self.lib.epr_adjoint_oversampled(
            self.h, C.byref(g), C.byref(s), _model(model), f, _dev(phase, "phase", ishape),
            _dev(resid_lines, "resid_lines", (spec.n_lines, geom.ny, geom.nx)),
            _dev(out, "obj_lines", (spec.n_lines,) + ishape), self._st()))
        return out

    def precondition(self, in_lines, geom, spec, mat: Material, out=None):
        shape = (spec.n_lines, geom.ny, geom.nx)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self._tdev())
        g, s, m = geom.c(), spec.c(), mat.c()
        self._check(self.lib.epr_precondition(self.h, C.byref(g), C.byref(s), C.byref(m),
                                              _dev(in_lines, "in_lines", shape),
                                              _dev(out, "out_lines", shape), self._st()))
        return out

    def regime(self, thickness, geom, spec, mat, n_bins=64, eta_max=4.0, out=None):
        """Per-line histogram of the shift-to-pixel ratio: int32 tensor [n_lines][n_bins + 1]
        (the library writes uint32 counts; a 4096 x 4096 image stays below 2^31)."""
        shape = (geom.ny, geom.nx)
        hshape = (spec.n_lines, int(n_bins) + 1)
        if out is None:
            out = torch.empty(hshape, dtype=torch.int32, device=self._tdev())
        elif out.dtype != torch.int32 or tuple(out.shape) != hshape or not out.is_contiguous():
            raise ValueError(f"counts must be contiguous int32 of shape {hshape}")
        g, s, m = geom.c(), spec.c(), mat.c()
        self._check(self.lib.epr_regime(self.h, C.byref(g), C.byref(s), C.byref(m),
                                        _dev(thickness, "thickness", shape), int(n_bins),
                                        float(eta_max), C.c_void_p(out.data_ptr()),
                                        self._st()))
        return out

    def select_model(self, intensity, geom, spec, mat, max_fraction=L.EPR_AUTO_MAX_FRACTION):
        """Automatic local / non-local choice: (model name, per-line counts of eta >= 1 on the
        Paganin retrieval).  Synchronises the current stream."""
        shape = (geom.ny, geom.nx)
        g, s, m = geom.c(), spec.c(), mat.c()
        model = C.c_int32(-1)
        over = (C.c_uint32 * spec.n_lines)()
        self._check(self.lib.epr_select_model(self.h, C.byref(g), C.byref(s), C.byref(m),
                                              _dev(intensity, "intensity", shape),
                                              float(max_fraction), C.byref(model), over,
                                              self._st()))
        return MODEL_NAMES[model.value], list(over)

    def solve(self, intensity, geom, spec, mat, model="nonlocal", n_iter=30, relaxation=0.4,
              thickness=None, phase_out=None, residuals=False, oversample=1):
        """thickness (and phase_out) live on the internal grid: [f ny][f nx] for oversample
        f; intensity is the detector image [ny][nx]."""
        shape = (geom.ny, geom.nx)
        f = int(oversample)
        ishape = (geom.ny * f, geom.nx * f)
        if thickness is None:
            thickness = torch.zeros(ishape, dtype=torch.float32, device=self._tdev())
        g, s, m = geom.c(), spec.c(), mat.c()
        o = L.Opts(_model(model), int(n_iter), float(relaxation),
                   L.EPR_FLAG_RESIDUALS if residuals else 0, f)
        ph = _dev(phase_out, "phase_out", ishape) if phase_out is not None else None
        self._check(self.lib.epr_solve(self.h, C.byref(g), C.byref(s), C.byref(m), C.byref(o),
                                       _dev(intensity, "intensity", shape),
                                       _dev(thickness, "thickness", ishape), ph,
                                       self._st()))
        return thickness

    def solve_noalloc(self, intensity, geom, spec, mat, model="nonlocal", n_iter=30,
                      relaxation=0.4, thickness=None, phase_out=None, residuals=False,
                      oversample=1):
        """epr_solve_noalloc: as solve, with the workspace in the library's fixed scratch array
        (no device allocation inside the call; `thickness` must then be passed in)."""
        shape = (geom.ny, geom.nx)
        f = int(oversample)
        ishape = (geom.ny * f, geom.nx * f)
        if thickness is None:
            raise ValueError("solve_noalloc needs the thickness buffer (it allocates nothing)")
        g, s, m = geom.c(), spec.c(), mat.c()
        o = L.Opts(_model(model), int(n_iter), float(relaxation),
                   L.EPR_FLAG_RESIDUALS if residuals else 0, f)
        ph = _dev(phase_out, "phase_out", ishape) if phase_out is not None else None
        self._check(self.lib.epr_solve_noalloc(self.h, C.byref(g), C.byref(s), C.byref(m),
                                               C.byref(o), _dev(intensity, "intensity", shape),
                                               _dev(thickness, "thickness", ishape), ph,
                                               self._st()))
        return thickness

    def solve_xspec(self, intensity, geom, spec, profile: SpectrumProfile, mat, model="nonlocal",
                    n_iter=30, relaxation=0.4, thickness=None, phase_out=None, residuals=False,
                    oversample=1, block_precond=False):
        """Solve with an x-dependent spectrum (spec gives n_lines, reference energy and
        exponents; profile the per-block energies and weights).  thickness and phase_out are
        on the internal grid, [f ny][f nx], when oversampling by f."""
        shape = (geom.ny, geom.nx)
        f = int(oversample)
        ishape = (geom.ny * f, geom.nx * f)
        if thickness is None:
            thickness = torch.zeros(ishape, dtype=torch.float32, device=self._tdev())
        g, m, pr = geom.c(), mat.c(), profile.c()
        s = spec.c()
        flags = (L.EPR_FLAG_RESIDUALS if residuals else 0) | \
            (L.EPR_FLAG_BLOCK_PRECOND if block_precond else 0)
        o = L.Opts(_model(model), int(n_iter), float(relaxation), flags, f)
        ph = _dev(phase_out, "phase_out", ishape) if phase_out is not None else None
        self._check(self.lib.epr_solve_xspec(self.h, C.byref(g), C.byref(s), C.byref(pr),
                                             C.byref(m), C.byref(o),
                                             _dev(intensity, "intensity", shape),
                                             _dev(thickness, "thickness", ishape), ph,
                                             self._st()))
        return thickness

    def forward_xspec(self, thickness, geom, spec, profile: SpectrumProfile, mat,
                      model="nonlocal"):
        """Detector intensity of a thickness map under an x-dependent spectrum (the model
        solve_xspec inverts)."""
        shape = (geom.ny, geom.nx)
        out = torch.empty(shape, dtype=torch.float32, device=self._tdev())
        g, s, pr, m = geom.c(), spec.c(), profile.c(), mat.c()
        self._check(self.lib.epr_forward_xspec(self.h, C.byref(g), C.byref(s), C.byref(pr),
                                               C.byref(m), _model(model),
                                               _dev(thickness, "thickness", shape),
                                               _dev(out, "intensity", shape),
                                               self._st()))
        return out

    def adjoint_xspec(self, thickness, resid_lines, geom, spec, profile: SpectrumProfile, mat,
                      model="nonlocal"):
        """Per-line back-transport under an x-dependent spectrum; resid_lines [L][ny][nx]."""
        shape = (geom.ny, geom.nx)
        lshape = (spec.n_lines, geom.ny, geom.nx)
        out = torch.empty(lshape, dtype=torch.float32, device=self._tdev())
        g, s, pr, m = geom.c(), spec.c(), profile.c(), mat.c()
        self._check(self.lib.epr_adjoint_xspec(self.h, C.byref(g), C.byref(s), C.byref(pr),
                                               C.byref(m), _model(model),
                                               _dev(thickness, "thickness", shape),
                                               _dev(resid_lines, "resid_lines", lshape),
                                               _dev(out, "obj_lines", lshape),
                                               self._st()))
        return out

    def _problems(self, problems, oversample=1):
        arr = (L.Problem * len(problems))()
        keep = []
        f = int(oversample)
        for i, (d, tau, geom, spec, mat) in enumerate(problems):
            shape = (geom.ny, geom.nx)
            s = spec.c()
            keep.append(s)
            arr[i] = L.Problem(geom.c(), s, mat.c(), _dev(d, "intensity", shape),
                               _dev(tau, "thickness", (geom.ny * f, geom.nx * f)))
        return arr, keep

    def solve_batched(self, problems, model="nonlocal", n_iter=30, relaxation=0.4,
                      oversample=1, residuals=False):
        """problems: list of (intensity, thickness, Geometry, Spectrum, Material); thickness is
        updated in place (on the internal grid, [f ny][f nx], when oversampling by f).  With
        residuals, the history of problems[0] is recorded (see diagnostics())."""
        arr, keep = self._problems(problems, oversample)
        o = L.Opts(_model(model), int(n_iter), float(relaxation),
                   L.EPR_FLAG_RESIDUALS if residuals else 0, int(oversample))
        self._check(self.lib.epr_solve_batched(self.h, len(problems), arr, C.byref(o),
                                               self._st()))
        del keep
        return [p[1] for p in problems]

    def solve_batched_xspec(self, problems, profiles, model="nonlocal", n_iter=30,
                            relaxation=0.4, oversample=1, residuals=False):
        """solve_batched with an x-dependent spectrum per problem: profiles[i] (a
        SpectrumProfile) for problems[i]; each problem's Spectrum gives the line count,
        reference energy and exponents."""
        if len(profiles) != len(problems):
            raise ValueError("one profile per problem")
        arr, keep = self._problems(problems, oversample)
        prs = (L.SpectrumProfile * len(profiles))()
        cs = [pr.c() for pr in profiles]      # (each holds the arrays its pointers refer to)
        for i, c in enumerate(cs):
            prs[i] = c
        keep.append(cs)
        o = L.Opts(_model(model), int(n_iter), float(relaxation),
                   L.EPR_FLAG_RESIDUALS if residuals else 0, int(oversample))
        self._check(self.lib.epr_solve_batched_xspec(self.h, len(problems), arr, prs,
                                                     C.byref(o), self._st()))
        del keep
        return [p[1] for p in problems]

    def autotune(self, problems, model="nonlocal", n_iter=1, relaxation=0.4, cache_json=None,
                 oversample=1):
        """Time the launch choices (splat tile on a warm state, lines per row-pass workgroup,
        radix order per transform length) on these problems and keep the fastest; returns the
        choices as a dict when a cache file is given (it is read if valid, written otherwise)."""
        arr, _keep = self._problems(problems, oversample)
        o = L.Opts(_model(model), int(n_iter), float(relaxation), 0, int(oversample))
        path = cache_json.encode() if cache_json else None
        self._check(self.lib.epr_autotune(self.h, len(problems), arr, C.byref(o), path))
        if cache_json:
            import json
            with open(cache_json) as fh:
                return json.load(fh)
        return None

    def forward_vjp(self, phase, absorb, grad_intensity, geom, spec, model="nonlocal"):
        shape = (geom.ny, geom.nx)
        gp = torch.empty(shape, dtype=torch.float32, device=self._tdev())
        ga = torch.empty(shape, dtype=torch.float32, device=self._tdev())
        g, s = geom.c(), spec.c()
        self._check(self.lib.epr_forward_vjp(self.h, C.byref(g), C.byref(s), _model(model),
                                             _dev(phase, "phase", shape),
                                             _dev(absorb, "absorb", shape),
                                             _dev(grad_intensity, "grad_intensity", shape),
                                             _dev(gp, "grad_phase", shape),
                                             _dev(ga, "grad_absorb", shape),
                                             self._st()))
        return gp, ga

    def forward_vjp_oversampled(self, phase, absorb, grad_intensity, geom, spec, oversample,
                                model="nonlocal"):
        """dL/d(phase), dL/d(absorb) on the internal grid ([f ny][f nx]) of forward_oversampled
        for grad_intensity = dL/d(intensity) on the detector ([ny][nx])."""
        f = int(oversample)
        shape, ishape = (geom.ny, geom.nx), (geom.ny * f, geom.nx * f)
        gp = torch.empty(ishape, dtype=torch.float32, device=self._tdev())
        ga = torch.empty(ishape, dtype=torch.float32, device=self._tdev())
        g, s = geom.c(), spec.c()
        self._check(self.lib.epr_forward_vjp_oversampled(
            self.h, C.byref(g), C.byref(s), _model(model), f, _dev(phase, "phase", ishape),
            _dev(absorb, "absorb", ishape), _dev(grad_intensity, "grad_intensity", shape),
            _dev(gp, "grad_phase", ishape), _dev(ga, "grad_absorb", ishape), self._st()))
        return gp, ga

    def forward_xspec_vjp(self, thickness, grad_intensity, geom, spec, profile: SpectrumProfile,
                          mat, model="nonlocal"):
        """dL/d(thickness) of forward_xspec for grad_intensity = dL/d(intensity)."""
        shape = (geom.ny, geom.nx)
        gt = torch.empty(shape, dtype=torch.float32, device=self._tdev())
        g, s, pr, m = geom.c(), spec.c(), profile.c(), mat.c()
        self._check(self.lib.epr_forward_xspec_vjp(self.h, C.byref(g), C.byref(s), C.byref(pr),
                                                   C.byref(m), _model(model),
                                                   _dev(thickness, "thickness", shape),
                                                   _dev(grad_intensity, "grad_intensity", shape),
                                                   _dev(gt, "grad_thickness", shape),
                                                   self._st()))
        return gt

    def set_timing(self, enabled=True):
        self._check(self.lib.epr_set_timing(self.h, 1 if enabled else 0))

    def timing(self, by_class=False):
        """{stage: (ms, launches)} since the last set_timing; with by_class, {(stage, size
        class): (ms, launches)} (class 0: up to 2048 x 2048 pixels, 1: larger)."""
        t = L.Timing()
        self._check(self.lib.epr_get_timing(self.h, C.byref(t)))
        if by_class:
            return {(name, c): (t.ms_class[i][c], t.launches_class[i][c])
                    for i, name in enumerate(L.STAGE_NAMES) for c in (0, 1)}
        return {name: (t.ms[i], t.launches[i]) for i, name in enumerate(L.STAGE_NAMES)}

    def diagnostics(self):
        """Diagnostics of the last solve.  A non-finite update (EPR_ERR_NONFINITE) does not
        raise: it is reported as `nonfinite` (problem count) and `first_nonfinite`."""
        d = L.Diagnostics()
        st = self.lib.epr_get_diagnostics(self.h, C.byref(d))
        if st != L.EPR_ERR_NONFINITE:
            self._check(st)
        return {"n_iter": d.n_iter, "n_problems": d.n_problems,
                "model": MODEL_NAMES.get(d.model, d.model), "max_shift_px": d.max_shift_px,
                "residual": list(d.residual[:min(d.n_iter, 256)]), "nonfinite": d.nonfinite,
                "first_nonfinite": d.first_nonfinite}


class EPRForward(torch.autograd.Function):
    """Differentiable forward model (any model but "auto"): (phase, absorb) -> detector
    intensity; with oversample = f > 1 the maps are on the internal grid [f ny][f nx] and the
    intensity is the detector's ([ny][nx], geom is the detector).

    backward is the library's hand-written vector-Jacobian product; the ray maps are
    recomputed from the saved phase, nothing else is kept.
    """

    @staticmethod
    def forward(ctx, phase, absorb, geom, spec, model="nonlocal", oversample=1):
        c = Context.get(phase.device)
        ctx.save_for_backward(phase, absorb)
        ctx.geom, ctx.spec, ctx.model, ctx.f = geom, spec, model, int(oversample)
        ph, ab = phase.detach().contiguous(), absorb.detach().contiguous()
        if ctx.f > 1:
            return c.forward_oversampled(ph, ab, geom, spec, ctx.f, model)
        return c.forward(ph, ab, geom, spec, model)

    @staticmethod
    def backward(ctx, grad):
        phase, absorb = ctx.saved_tensors
        c = Context.get(phase.device)
        ph, ab = phase.detach().contiguous(), absorb.detach().contiguous()
        if ctx.f > 1:
            gp, ga = c.forward_vjp_oversampled(ph, ab, grad.contiguous(), ctx.geom, ctx.spec,
                                               ctx.f, ctx.model)
        else:
            gp, ga = c.forward_vjp(ph, ab, grad.contiguous(), ctx.geom, ctx.spec, ctx.model)
        return gp, ga, None, None, None, None


def epr_forward(phase, absorb, geom, spec, model="nonlocal", oversample=1):
    return EPRForward.apply(phase, absorb, geom, spec, model, oversample)


class EPRForwardXspec(torch.autograd.Function):
    """Differentiable forward model under an x-dependent spectrum (any model but "auto"):
    thickness -> detector intensity; backward is the library's vector-Jacobian product with
    respect to the thickness."""

    @staticmethod
    def forward(ctx, thickness, geom, spec, profile, mat, model="nonlocal"):
        c = Context.get(thickness.device)
        ctx.save_for_backward(thickness)
        ctx.args = (geom, spec, profile, mat, model)
        return c.forward_xspec(thickness.detach().contiguous(), geom, spec, profile, mat, model)

    @staticmethod
    def backward(ctx, grad):
        (thickness,) = ctx.saved_tensors
        c = Context.get(thickness.device)
        geom, spec, profile, mat, model = ctx.args
        gt = c.forward_xspec_vjp(thickness.detach().contiguous(), grad.contiguous(), geom, spec,
                                 profile, mat, model)
        return gt, None, None, None, None, None


def epr_forward_xspec(thickness, geom, spec, profile, mat, model="nonlocal"):
    return EPRForwardXspec.apply(thickness, geom, spec, profile, mat, model)
