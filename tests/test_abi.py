"""The C ABI without a device: the library loads, exports every function include/epr.h declares,
and its host-only logic (status strings, FFT plans, validation) behaves as documented."""

import ctypes as C
import math
import os
import re
import shutil
import subprocess

import pytest

from paper_2601_22793_amd import _lib as L
from tests.helpers import has_gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epr.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(epr_[a-z_]+)\s*\(", src)))


def test_library_loads_and_exports_every_declared_function():
    lib = L.load()
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.PROTOTYPES), "binding and header disagree"


def test_status_strings():
    lib = L.load()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = lib.epr_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.epr_status_string(42).decode() == "unknown status"


@pytest.mark.skipif(has_gpu(), reason="checks the no-device path")
def test_create_without_device_fails_cleanly():
    lib = L.load()
    h = C.c_void_p(123)
    st = lib.epr_create(C.byref(h), 0)
    assert st == L.EPR_ERR_NO_DEVICE
    assert not h.value
    assert "device" in lib.epr_last_error(None).decode()


def test_null_handle_is_rejected():
    lib = L.load()
    g = L.Geometry(64, 64, 1e-5, 1.0)
    assert lib.epr_solve(None, C.byref(g), None, None, None, None, None, None, None) == \
        L.EPR_ERR_INVALID_ARG
    assert lib.epr_destroy(None) == L.EPR_ERR_INVALID_ARG
    assert lib.epr_get_diagnostics(None, None) == L.EPR_ERR_INVALID_ARG
    # every other entry point that takes a handle
    for name in L.PROTOTYPES:
        restype, argtypes = L.PROTOTYPES[name]
        if restype is not C.c_int or not argtypes or \
                argtypes[0] is not L.PROTOTYPES["epr_destroy"][1][0]:
            continue   # (epr_last_error(NULL) is the last error of epr_create)
        args = [None] + [0 if t in (C.c_int, C.c_int32, C.c_uint32, C.c_size_t) else
                         0.0 if t is C.c_double else None for t in argtypes[1:]]
        assert getattr(lib, name)(*args) == L.EPR_ERR_INVALID_ARG, name


@pytest.mark.parametrize("n,expect", [(2048, [16, 16, 8]), (1024, [16, 16, 4]),
                                      (1280, [16, 16, 5]), (2160, [16, 5, 3, 3, 3]),
                                      (1080, [8, 5, 3, 3, 3]), (128, [16, 8]), (8, [8]),
                                      (30, [2, 5, 3]), (4096, [16, 16, 16])])
def test_fft_plan_radices(n, expect):
    lib = L.load()
    buf = (C.c_int32 * 16)()
    k = lib.epr_fft_plan(n, buf, 16)
    assert k == len(expect)
    assert list(buf[:k]) == expect
    assert math.prod(buf[:k]) == n


@pytest.mark.parametrize("n", [7, 14, 4097, 2 * 11])
def test_fft_plan_rejects_other_primes(n):
    lib = L.load()
    assert lib.epr_fft_plan(n, (C.c_int32 * 16)(), 16) == L.EPR_ERR_SHAPE


def _check(geom, energies=(60.0,), weights=(1.0,), mat=(4e-7, 4e-10), opts=(3, 10, 0.4, 0)):
    lib = L.load()
    e = (C.c_double * len(energies))(*energies)
    w = (C.c_double * len(weights))(*weights)
    spec = L.Spectrum(len(energies), e, w, 60.0, 2.0, 3.0)
    g = L.Geometry(*geom)
    m = L.Material(*mat) if mat else None
    o = L.Opts(*opts) if opts else None
    msg = C.create_string_buffer(256)
    st = lib.epr_check_problem(C.byref(g), C.byref(spec), C.byref(m) if m else None,
                               C.byref(o) if o else None, msg, 256)
    return st, msg.value.decode()


def test_check_problem_accepts_the_workload_shapes():
    for shape in [(256, 256), (2048, 2048), (1024, 1024), (2160, 2560), (90, 250), (8, 8)]:
        st, msg = _check((shape[0], shape[1], 1e-5, 20.0))
        assert st == L.EPR_OK, msg
    st, _ = _check((2048, 2048, 1e-5, 20.0), energies=[66.25 + 12.5 * i for i in range(8)],
                   weights=[1 / 8] * 8)
    assert st == L.EPR_OK


@pytest.mark.parametrize("geom,code,word", [
    ((256, 255, 1e-5, 1.0), L.EPR_ERR_SHAPE, "even"),
    ((7 * 32, 256, 1e-5, 1.0), L.EPR_ERR_SHAPE, "products"),
    ((4, 256, 1e-5, 1.0), L.EPR_ERR_SHAPE, "outside"),
    ((5000, 256, 1e-5, 1.0), L.EPR_ERR_SHAPE, "outside"),
    ((256, 256, 0.0, 1.0), L.EPR_ERR_INVALID_ARG, "pixel"),
    ((256, 256, 1e-5, -1.0), L.EPR_ERR_INVALID_ARG, "distance"),
    ((256, 256, float("nan"), 1.0), L.EPR_ERR_INVALID_ARG, "pixel"),
])
def test_check_problem_rejects_bad_geometry(geom, code, word):
    st, msg = _check(geom)
    assert st == code and word in msg


def test_check_problem_rejects_bad_spectrum_material_and_options():
    g = (64, 64, 1e-5, 1.0)
    assert _check(g, weights=(0.9,))[0] == L.EPR_ERR_INVALID_ARG
    assert _check(g, energies=(-1.0,))[0] == L.EPR_ERR_INVALID_ARG
    n = 17
    assert _check(g, energies=[60.0] * n, weights=[1 / n] * n)[0] == L.EPR_ERR_INVALID_ARG
    assert _check(g, mat=(0.0, 1e-9))[0] == L.EPR_ERR_INVALID_ARG
    assert _check(g, opts=(9, 10, 0.4, 0))[0] == L.EPR_ERR_INVALID_ARG
    assert _check(g, opts=(3, -1, 0.4, 0))[0] == L.EPR_ERR_INVALID_ARG
    assert _check(g, opts=(3, 10, 0.0, 0))[0] == L.EPR_ERR_INVALID_ARG
    assert _check(g, opts=(3, 10, 0.4, 8))[0] == L.EPR_ERR_INVALID_ARG
    # material and options may be omitted
    assert _check(g, mat=None, opts=None)[0] == L.EPR_OK
    # EPR_AUTO is valid for the single-problem solve
    assert _check(g, opts=(0, 10, 0.4, 0))[0] == L.EPR_OK


def test_check_problem_oversampling():
    # the internal grid (f ny) x (f nx) must itself satisfy the size rules
    assert _check((1024, 1024, 1e-5, 1.0), opts=(3, 5, 0.4, 0, 4))[0] == L.EPR_OK
    assert _check((2048, 2048, 1e-5, 1.0), opts=(3, 5, 0.4, 0, 2))[0] == L.EPR_OK
    st, msg = _check((2048, 2048, 1e-5, 1.0), opts=(3, 5, 0.4, 0, 4))
    assert st == L.EPR_ERR_SHAPE and "internal grid" in msg
    assert _check((64, 64, 1e-5, 1.0), opts=(3, 5, 0.4, 0, 3))[0] == L.EPR_ERR_INVALID_ARG
    assert _check((64, 64, 1e-5, 1.0), opts=(3, 5, 0.4, 0, 1))[0] == L.EPR_OK


def test_binding_raises_without_device():
    if has_gpu():
        pytest.skip("device present")
    from paper_2601_22793_amd import Context, EprError
    with pytest.raises(EprError):
        Context(0)


STRUCTS = {
    "epr_geometry": L.Geometry, "epr_spectrum": L.Spectrum,
    "epr_spectrum_profile": L.SpectrumProfile, "epr_material": L.Material, "epr_opts": L.Opts,
    "epr_problem": L.Problem, "epr_diagnostics": L.Diagnostics, "epr_timing": L.Timing,
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a C compiler")
def test_struct_layouts_match_the_header(tmp_path):
    """Every struct of include/epr.h as the C compiler lays it out (sizeof, offsetof of each
    field) equals the ctypes declaration of the binding."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "epr.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in filter(None, out):
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in STRUCTS.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
