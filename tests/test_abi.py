"""CPU-side checks of the C-ABI: the library loads, exports every function
the public header declares, its struct layout matches the ctypes binding,
and argument validation rejects bad jobs before any device work (these calls
never reach the GPU, so they run without one)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "toprop.h")


@pytest.fixture(scope="module")
def capi():
    from paper_2411_18591_amd import _capi
    return _capi


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:to_status|const char\*|int32_t)\s+(to_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function(capi):
    lib = capi.lib()
    names = declared_functions()
    assert set(names) >= {"to_propagate", "to_modulate", "to_propagate_backward",
                          "to_coherence_propagate", "to_last_error"}
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(capi.EXPORTED)
    assert lib.to_version().decode().startswith("toprop")


def test_struct_layout_matches_header(capi):
    fields = [f for f, _ in capi.Job._fields_]
    gfields = [f for f, _ in capi.Grad._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){"]
    src.append('printf("%zu %zu %zu %zu %zu\\n", sizeof(to_job), sizeof(to_grad), sizeof(to_plan), '
               'offsetof(to_plan, chunk_mb), offsetof(to_plan, us));')
    for f in fields:
        cf = "in" if f == "in_" else f
        src.append(f'printf("%zu\\n", offsetof(to_job, {cf}));')
    for f in gfields:
        src.append(f'printf("%zu\\n", offsetof(to_grad, {f}));')
    src.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write("\n".join(src))
        subprocess.check_call(["gcc", "-std=c11", "-o", exe, c])
        out = subprocess.check_output([exe]).decode().split()
    sizes = [int(x) for x in out]
    assert sizes[0] == ctypes.sizeof(capi.Job)
    assert sizes[1] == ctypes.sizeof(capi.Grad)
    assert sizes[2:5] == [ctypes.sizeof(capi.Plan), capi.Plan.chunk_mb.offset, capi.Plan.us.offset]
    sizes = sizes[:2] + sizes[5:]
    for f, off in zip(fields, sizes[2:2 + len(fields)]):
        assert getattr(capi.Job, f).offset == off, f
    for f, off in zip(gfields, sizes[2 + len(fields):]):
        assert getattr(capi.Grad, f).offset == off, f


def good_job(capi):
    j = capi.Job()
    j.ny, j.nx, j.py, j.px = 16, 16, 32, 32
    j.method = capi.TO_ASM
    j.ncomp = 1
    j.dy = j.dx = 1e-5
    j.wavelength = 7e-7
    j.z = 0.1
    j.batch = 1
    j.in_ = 0x1000  # never dereferenced: validation fails first in every case below
    j.out = 0x2000
    return j


@pytest.mark.parametrize("mutate,status", [
    (lambda j: setattr(j, "ny", 0), "TO_E_INVAL"),
    (lambda j: setattr(j, "py", 8), "TO_E_INVAL"),          # smaller than the field
    (lambda j: (setattr(j, "nx", 4), setattr(j, "px", 4)), "TO_E_UNSUPPORTED"),  # power of two below 8
    (lambda j: setattr(j, "px", 16384), "TO_E_UNSUPPORTED"),
    (lambda j: (setattr(j, "nx", 16), setattr(j, "px", 5000)), "TO_E_UNSUPPORTED"),  # not a power of two, > 4096
    (lambda j: setattr(j, "dx", 0.0), "TO_E_INVAL"),
    (lambda j: setattr(j, "dy", float("nan")), "TO_E_INVAL"),
    (lambda j: setattr(j, "wavelength", -1.0), "TO_E_INVAL"),
    (lambda j: setattr(j, "z", float("inf")), "TO_E_INVAL"),
    (lambda j: setattr(j, "method", 7), "TO_E_INVAL"),
    (lambda j: setattr(j, "batch", -1), "TO_E_INVAL"),
    (lambda j: setattr(j, "ncomp", 2), "TO_E_INVAL"),
    (lambda j: setattr(j, "el_flags", 8), "TO_E_INVAL"),    # Jones with ncomp 1
    (lambda j: setattr(j, "el_flags", 1), "TO_E_INVAL"),    # phase mask pointer NULL
    (lambda j: setattr(j, "el_flags", 64), "TO_E_INVAL"),
    (lambda j: (setattr(j, "el_flags", 4), setattr(j, "el_f", 0.0)), "TO_E_INVAL"),
    (lambda j: setattr(j, "out", None), "TO_E_INVAL"),
    (lambda j: setattr(j, "epi", 1), "TO_E_INVAL"),         # epilogue buffers NULL
    (lambda j: setattr(j, "epi", 9), "TO_E_INVAL"),
    (lambda j: setattr(j, "epi", 3), "TO_E_INVAL"),         # intensity without epi_out
    (lambda j: (setattr(j, "ncomp", 3), setattr(j, "el_flags", 16)), "TO_E_INVAL"),   # Jones map NULL
    (lambda j: (setattr(j, "ncomp", 3), setattr(j, "el_flags", 24), setattr(j, "el_jones_map", 0x7000)),
     "TO_E_INVAL"),                                         # uniform and mapped Jones together
    (lambda j: (setattr(j, "el_flags", 16), setattr(j, "el_jones_map", 0x7000)), "TO_E_INVAL"),  # ncomp 1
    (lambda j: (setattr(j, "epi", 3), setattr(j, "epi_out", 0x6000), setattr(j, "in_", None)), "TO_E_INVAL"),
    (lambda j: (setattr(j, "epi", 3), setattr(j, "epi_out", 0x6000), setattr(j, "epi_scale", float("nan"))),
     "TO_E_INVAL"),
    (lambda j: (setattr(j, "method", 2), setattr(j, "z", 0.0)), "TO_E_INVAL"),        # DI needs z > 0
    (lambda j: (setattr(j, "method", 2), setattr(j, "z", -0.1)), "TO_E_INVAL"),
    (lambda j: (setattr(j, "method", 2), setattr(j, "py", 16)), "TO_E_UNSUPPORTED"),  # < 2 ny - 1
    (lambda j: (setattr(j, "method", 2), setattr(j, "nx", 17), setattr(j, "px", 32)), "TO_E_UNSUPPORTED"),
    (lambda j: (setattr(j, "method", 3), setattr(j, "z", 10.0), setattr(j, "px", 16)), "TO_E_UNSUPPORTED"),
])
def test_validation_rejects_bad_jobs(capi, mutate, status):
    j = good_job(capi)
    mutate(j)
    arr = capi.jobs_array([j])
    rc = capi.lib().to_propagate(arr, 1, capi.TO_C64, None)
    assert rc == getattr(capi, status)
    assert len(capi.lib().to_last_error()) > 0


def test_validation_other_entry_points(capi):
    lib = capi.lib()
    assert lib.to_propagate(None, 1, capi.TO_C64, None) == capi.TO_E_INVAL
    assert lib.to_propagate(None, -1, capi.TO_C64, None) == capi.TO_E_INVAL
    assert lib.to_propagate(None, 0, capi.TO_C64, None) == capi.TO_OK
    j = good_job(capi)
    assert lib.to_propagate(capi.jobs_array([j]), 1, 5, None) == capi.TO_E_INVAL  # dtype
    g = capi.Grad()
    assert lib.to_propagate_backward(capi.jobs_array([j]), capi.grads_array([g]), 1,
                                     capi.TO_C64, None) == capi.TO_E_INVAL  # grad_out NULL
    g.grad_out = 0x3000
    g.grad_phase = 0x4000
    j.el_flags = capi.TO_EL_PHASE
    j.el_phase = 0x5000
    assert lib.to_propagate_backward(capi.jobs_array([j]), capi.grads_array([g]), 1,
                                     capi.TO_C64, None) == capi.TO_E_INVAL  # saved_in NULL
    assert lib.to_coherence_propagate(None, capi.TO_C64, 0, None, None) == capi.TO_E_INVAL
    j2 = good_job(capi)
    j2.batch = 2
    assert lib.to_coherence_propagate(ctypes.byref(j2), capi.TO_C64, 0, None, None) == capi.TO_E_INVAL


def test_missing_library_fails_loudly(capi, monkeypatch, tmp_path):
    monkeypatch.setattr(capi, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(capi, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        capi.lib()


def test_grid_layout_matches_header(capi):
    src = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){",
           'printf("%zu", sizeof(to_grid));']
    for f, _ in capi.Grid._fields_:
        src.append(f'printf(" %zu", offsetof(to_grid, {f}));')
    src.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "grid.c")
        exe = os.path.join(d, "grid")
        open(c, "w").write("\n".join(src))
        subprocess.check_call(["gcc", "-std=c11", "-o", exe, c])
        vals = [int(x) for x in subprocess.check_output([exe]).decode().split()]
    assert vals[0] == ctypes.sizeof(capi.Grid)
    assert vals[1:] == [getattr(capi.Grid, f).offset for f, _ in capi.Grid._fields_]


def _grid(capi, ny=8, nx=9, dy=1e-6, dx=2e-6):
    g = capi.Grid()
    g.ny, g.nx, g.dy, g.dx = ny, nx, dy, dx
    return g


@pytest.mark.parametrize("case,status", [
    (dict(gin=None), "TO_E_INVAL"),
    (dict(interp=5), "TO_E_INVAL"),
    (dict(batch=-1), "TO_E_INVAL"),
    (dict(dtype=7), "TO_E_INVAL"),
    (dict(gin_ny=0), "TO_E_INVAL"),
    (dict(gout_dx=0.0), "TO_E_INVAL"),
    (dict(gout_dy=float("nan")), "TO_E_INVAL"),
    (dict(src=None), "TO_E_INVAL"),
    (dict(dst=0x1000 + 64), "TO_E_INVAL"),   # overlaps src
    (dict(batch=0, src=None, dst=None), "TO_OK"),
])
def test_resample_validation(capi, case, status):
    gin, gout = _grid(capi), _grid(capi, 5, 6, 1.5e-6, 2.5e-6)
    if "gin_ny" in case:
        gin.ny = case["gin_ny"]
    if "gout_dx" in case:
        gout.dx = case["gout_dx"]
    if "gout_dy" in case:
        gout.dy = case["gout_dy"]
    src = case.get("src", 0x1000)
    dst = case.get("dst", 0x9000000)
    gp = None if case.get("gin", 1) is None else ctypes.byref(gin)
    rc = capi.lib().to_resample(src, dst, gp, ctypes.byref(gout), case.get("batch", 2), case.get("interp", 1), 0,
                                case.get("dtype", capi.TO_C64), None)
    assert rc == getattr(capi, status)


def _resolve(capi, j):
    m = ctypes.c_int32(-1)
    rc = capi.lib().to_resolve_method(ctypes.byref(j), ctypes.byref(m))
    return rc, m.value


def test_resolve_method_matches_the_oracle(capi):
    """The automatic choice (Eq. (sampling_condition)) in the library's host
    code against the oracle's, over random geometries around the critical
    distance, both signs of z, and unequal axes."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(31)
    for _ in range(400):
        j = good_job(capi)
        j.ny, j.nx = int(rng.integers(1, 600)), int(rng.integers(1, 600))
        j.py, j.px = 2048, 2048
        j.dy, j.dx = float(rng.uniform(1e-6, 2e-5)), float(rng.uniform(1e-6, 2e-5))
        j.wavelength = float(rng.uniform(4e-7, 8e-7))
        zc = oracle.critical_distance(j.ny, j.nx, j.dy, j.dx, j.wavelength)
        j.z = float(zc * rng.choice([-1.5, 0.0, 0.5, 0.999999, 1.0, 1.000001, 3.0]))
        j.method = capi.TO_AUTO
        rc, m = _resolve(capi, j)
        assert rc == capi.TO_OK
        assert m == oracle.resolve_method(j.ny, j.nx, j.dy, j.dx, j.wavelength, j.z), (j.ny, j.nx, j.z / zc)
    j = good_job(capi)
    for meth in (capi.TO_ASM, capi.TO_FRESNEL, capi.TO_DI):
        j.method = meth
        assert _resolve(capi, j) == (capi.TO_OK, meth)
    j.method = 7
    assert _resolve(capi, j)[0] == capi.TO_E_INVAL
    assert capi.lib().to_resolve_method(None, None) == capi.TO_E_INVAL


def test_transfer_table_validation(capi):
    lib = capi.lib()
    j = good_job(capi)
    assert lib.to_transfer_table(ctypes.byref(j), capi.TO_C64, None, None) == capi.TO_E_INVAL
    assert lib.to_transfer_table(None, capi.TO_C64, 0x1000, None) == capi.TO_E_INVAL
    j.method = capi.TO_DI
    j.py = 16
    assert lib.to_transfer_table(ctypes.byref(j), capi.TO_C64, 0x1000, None) == capi.TO_E_UNSUPPORTED


def test_next_smooth_padding():
    """round_smooth padding: the least length >= max(n, 3) with no prime
    factor above 7, checked by brute force up to 5000."""
    import paper_2411_18591_amd as tp

    def smooth(m):
        for q in (2, 3, 5, 7):
            while m % q == 0:
                m //= q
        return m == 1

    for n in range(1, 5001):
        m = tp.next_smooth(n)
        assert m >= max(n, 3) and smooth(m)
        assert not any(smooth(k) for k in range(max(n, 3), m))
    o = tp.Optics(dy=1e-5, dx=1e-5, wavelength=7e-7, z=0.1, pad=2, round_pow2=False, round_smooth=True)
    assert o.padded_shape(1001, 1000) == (2016, 2000)


@pytest.mark.parametrize("mutate,status,words", [
    (lambda j: setattr(j, "ny", 0), "TO_E_INVAL", ">= 1"),            # the checks of to_propagate
    (lambda j: (setattr(j, "nx", 20), setattr(j, "px", 48)), "TO_E_UNSUPPORTED", "powers of two"),
    (lambda j: (setattr(j, "ny", 4096), setattr(j, "nx", 4096), setattr(j, "py", 8192), setattr(j, "px", 8192)),
     "TO_E_UNSUPPORTED", "static area"),                               # 256 MiB for one field
    (lambda j: setattr(j, "method", 2), "TO_E_UNSUPPORTED", "direct integration"),  # DI without a table
])
def test_noalloc_rejects_before_any_gpu_work(capi, mutate, status, words):
    """The entry point that allocates nothing rejects jobs beyond its static
    area (and everything to_propagate rejects) on the host, before it looks
    up the array or enqueues anything, so these run without a GPU."""
    j = good_job(capi)
    mutate(j)
    rc = capi.lib().to_propagate_noalloc(capi.jobs_array([j]), 1, capi.TO_C64, None)
    assert rc == getattr(capi, status)
    assert words in capi.lib().to_last_error().decode()
    assert capi.lib().to_propagate_noalloc(None, -1, capi.TO_C64, None) == capi.TO_E_INVAL
    assert capi.lib().to_propagate_noalloc(None, 0, capi.TO_C64, None) == capi.TO_OK


def test_jones_elements_match_the_oracle(capi):
    """The library's element matrices (host-only entry points) against the
    oracle's, whose polarizer and waveplate are pinned by the paper's
    transmitted powers and Malus's law; composition order: the first
    argument acts first."""
    import math

    import numpy as np

    import oracle
    for th in (0.0, 0.3, math.pi / 6, math.pi / 4, 2.0):
        got = np.array(capi.jones_linear_polarizer(th))
        assert np.abs(got - oracle.embed_jones(oracle.linear_polarizer(th))).max() <= 1e-15
        for gam in (math.pi / 2, math.pi, 1.1):
            got = np.array(capi.jones_waveplate(th, gam))
            assert np.abs(got - oracle.embed_jones(oracle.waveplate(th, gam))).max() <= 1e-15
    qwp, lp = capi.jones_waveplate(math.pi / 4, math.pi / 2), capi.jones_linear_polarizer(math.pi / 6)
    got = np.array(capi.jones_compose(qwp, lp))
    exp = oracle.embed_jones(oracle.linear_polarizer(math.pi / 6) @ oracle.waveplate(math.pi / 4, math.pi / 2))
    assert np.abs(got - exp).max() <= 1e-15
    with pytest.raises(capi.ToError):
        capi.jones_linear_polarizer(float("nan"))
