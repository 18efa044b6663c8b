"""ctypes view of the C-ABI declared in include/toprop.h.

Argument marshalling only: every computation happens in libtoprop.so.  The
library is loaded from this package directory; if it is missing the loader
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtoprop.so")

TO_OK = 0
TO_E_INVAL = -1
TO_E_UNSUPPORTED = -2
TO_E_NOMEM = -3
TO_E_HIP = -4

TO_ASM = 0
TO_FRESNEL = 1
TO_DI = 2
TO_AUTO = 3
TO_NEAREST = 0
TO_BILINEAR = 1
TO_C64 = 0
TO_C128 = 1

TO_EL_PHASE = 1
TO_EL_COMPLEX = 2
TO_EL_LENS = 4
TO_EL_JONES = 8
TO_EL_JONES_MAP = 16
TO_GRAD_IN_TRANSIENT = 1

TO_EPI_NONE = 0
TO_EPI_MSE = 1
TO_EPI_WEIGHTED = 2
TO_EPI_INTENSITY = 3

EXPORTED = (
    "to_jones_linear_polarizer",
    "to_jones_waveplate",
    "to_jones_compose",
    "to_propagate",
    "to_propagate_noalloc",
    "to_graph_create",
    "to_graph_launch",
    "to_graph_destroy",
    "to_resample",
    "to_transfer_table",
    "to_resolve_method",
    "to_modulate",
    "to_propagate_backward",
    "to_coherence_propagate",
    "to_last_error",
    "to_release",
    "to_version",
    "to_profile_begin",
    "to_profile_end",
    "to_profile_count",
    "to_profile_entry",
    "to_propagate_plain",
    "to_propagate_backward_plain",
    "to_autotune",
    "to_plan_get",
    "to_plan_set",
    "to_plan_clear",
    "to_plan_load",
    "to_plan_save",
)


class Job(ctypes.Structure):
    _fields_ = [
        ("ny", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("py", ctypes.c_int32),
        ("px", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("ncomp", ctypes.c_int32),
        ("dy", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("wavelength", ctypes.c_double),
        ("z", ctypes.c_double),
        ("y0", ctypes.c_double),
        ("x0", ctypes.c_double),
        ("batch", ctypes.c_int64),
        ("el_flags", ctypes.c_uint32),
        ("epi", ctypes.c_int32),
        ("el_phase", ctypes.c_void_p),
        ("el_complex", ctypes.c_void_p),
        ("el_f", ctypes.c_double),
        ("el_jones", ctypes.c_double * 18),
        ("epi_ref", ctypes.c_void_p),
        ("epi_scale", ctypes.c_double),
        ("epi_grad", ctypes.c_void_p),
        ("epi_loss", ctypes.c_void_p),
        ("in_", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("epi_out", ctypes.c_void_p),
        ("el_jones_map", ctypes.c_void_p),
        ("tf_table", ctypes.c_void_p),
    ]


class Grid(ctypes.Structure):
    _fields_ = [
        ("ny", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("dy", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("y0", ctypes.c_double),
        ("x0", ctypes.c_double),
    ]


class Grad(ctypes.Structure):
    _fields_ = [
        ("grad_out", ctypes.c_void_p),
        ("grad_in", ctypes.c_void_p),
        ("saved_in", ctypes.c_void_p),
        ("grad_phase", ctypes.c_void_p),
        ("grad_f", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
    ]


class Plan(ctypes.Structure):
    _fields_ = [
        ("col_variant", ctypes.c_int32),
        ("chunk_mb", ctypes.c_int32),
        ("row_fpb", ctypes.c_int32),
        ("us", ctypes.c_double),
    ]


def _plan_dict(p) -> dict:
    return {"col_variant": p.col_variant, "chunk_mb": p.chunk_mb, "row_fpb": p.row_fpb, "us": p.us}


class ToError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"toprop error {status}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libtoprop.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2411_18591_amd.build` "
                "(hipcc, gfx950). There is no fallback implementation.")
        L = ctypes.CDLL(LIB_PATH)
        c_int = ctypes.c_int32
        JP = ctypes.POINTER(Job)
        GP = ctypes.POINTER(Grad)
        L.to_propagate.argtypes = [JP, c_int, c_int, ctypes.c_void_p]
        L.to_propagate.restype = c_int
        L.to_propagate_noalloc.argtypes = [JP, c_int, c_int, ctypes.c_void_p]
        L.to_propagate_noalloc.restype = c_int
        L.to_graph_create.argtypes = [JP, GP, c_int, c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
        L.to_graph_create.restype = c_int
        L.to_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.to_graph_launch.restype = c_int
        L.to_graph_destroy.argtypes = [ctypes.c_void_p]
        L.to_graph_destroy.restype = c_int
        L.to_modulate.argtypes = [JP, c_int, c_int, c_int, ctypes.c_void_p]
        L.to_modulate.restype = c_int
        L.to_propagate_backward.argtypes = [JP, GP, c_int, c_int, ctypes.c_void_p]
        L.to_propagate_backward.restype = c_int
        L.to_coherence_propagate.argtypes = [JP, c_int, c_int, GP, ctypes.c_void_p]
        L.to_coherence_propagate.restype = c_int
        L.to_last_error.argtypes = []
        L.to_last_error.restype = ctypes.c_char_p
        L.to_release.argtypes = []
        L.to_release.restype = c_int
        L.to_version.argtypes = []
        L.to_version.restype = ctypes.c_char_p
        L.to_profile_begin.argtypes = []
        L.to_profile_begin.restype = c_int
        L.to_profile_end.argtypes = []
        L.to_profile_end.restype = c_int
        L.to_profile_count.argtypes = []
        L.to_profile_count.restype = c_int
        L.to_profile_entry.argtypes = [c_int, ctypes.c_char_p, c_int, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double)]
        L.to_profile_entry.restype = c_int
        L.to_propagate_plain.argtypes = [JP, c_int, c_int, ctypes.c_void_p]
        L.to_propagate_plain.restype = c_int
        L.to_propagate_backward_plain.argtypes = [JP, GP, c_int, c_int, ctypes.c_void_p]
        L.to_propagate_backward_plain.restype = c_int
        PP = ctypes.POINTER(Plan)
        L.to_autotune.argtypes = [JP, c_int, ctypes.c_void_p, PP]
        L.to_autotune.restype = c_int
        L.to_plan_get.argtypes = [c_int, c_int, c_int, PP, ctypes.POINTER(c_int)]
        L.to_plan_get.restype = c_int
        L.to_plan_set.argtypes = [c_int, c_int, c_int, PP]
        L.to_plan_set.restype = c_int
        L.to_plan_clear.argtypes = []
        L.to_plan_clear.restype = c_int
        L.to_plan_load.argtypes = [ctypes.c_char_p]
        L.to_plan_load.restype = c_int
        L.to_plan_save.argtypes = [ctypes.c_char_p]
        L.to_plan_save.restype = c_int
        L.to_transfer_table.argtypes = [JP, c_int, ctypes.c_void_p, ctypes.c_void_p]
        L.to_transfer_table.restype = c_int
        L.to_resolve_method.argtypes = [JP, ctypes.POINTER(c_int)]
        L.to_resolve_method.restype = c_int
        GR = ctypes.POINTER(Grid)
        L.to_resample.argtypes = [ctypes.c_void_p, ctypes.c_void_p, GR, GR, ctypes.c_int64, c_int, c_int, c_int,
                                  ctypes.c_void_p]
        L.to_resample.restype = c_int
        DP = ctypes.POINTER(ctypes.c_double)
        L.to_jones_linear_polarizer.argtypes = [ctypes.c_double, DP]
        L.to_jones_linear_polarizer.restype = c_int
        L.to_jones_waveplate.argtypes = [ctypes.c_double, ctypes.c_double, DP]
        L.to_jones_waveplate.restype = c_int
        L.to_jones_compose.argtypes = [DP, DP, DP]
        L.to_jones_compose.restype = c_int
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != TO_OK:
        raise ToError(status, lib().to_last_error().decode())


def _jones_out():
    return (ctypes.c_double * 18)()


def _jones_list(buf):
    return [[complex(buf[6 * r + 2 * c], buf[6 * r + 2 * c + 1]) for c in range(3)] for r in range(3)]


def _jones_buf(J):
    buf = _jones_out()
    for r in range(3):
        for c in range(3):
            buf[6 * r + 2 * c] = complex(J[r][c]).real
            buf[6 * r + 2 * c + 1] = complex(J[r][c]).imag
    return buf


def jones_linear_polarizer(theta: float):
    out = _jones_out()
    check(lib().to_jones_linear_polarizer(float(theta), out))
    return _jones_list(out)


def jones_waveplate(theta: float, retardance: float):
    out = _jones_out()
    check(lib().to_jones_waveplate(float(theta), float(retardance), out))
    return _jones_list(out)


def jones_compose(first, then):
    out = _jones_out()
    check(lib().to_jones_compose(_jones_buf(first), _jones_buf(then), out))
    return _jones_list(out)


def jobs_array(jobs):
    arr = (Job * len(jobs))(*jobs)
    return arr


def grads_array(grads):
    return (Grad * len(grads))(*grads)


def propagate(jobs, dtype: int, stream: int, plain: bool = False) -> None:
    arr = jobs_array(jobs)
    fn = lib().to_propagate_plain if plain else lib().to_propagate
    check(fn(arr, len(jobs), dtype, ctypes.c_void_p(stream)))


def propagate_noalloc(jobs, dtype: int, stream: int) -> None:
    check(lib().to_propagate_noalloc(jobs_array(jobs), len(jobs), dtype, ctypes.c_void_p(stream)))


def modulate(jobs, dtype: int, adjoint: bool, stream: int) -> None:
    arr = jobs_array(jobs)
    check(lib().to_modulate(arr, len(jobs), dtype, 1 if adjoint else 0, ctypes.c_void_p(stream)))


def graph_create(jobs, grads, dtype: int, stream: int) -> int:
    """to_graph_create: run the call once, capture it; returns the handle."""
    h = ctypes.c_void_p()
    g = grads_array(grads) if grads is not None else None
    check(lib().to_graph_create(jobs_array(jobs), g, len(jobs), dtype, ctypes.c_void_p(stream), ctypes.byref(h)))
    return h.value


def graph_launch(handle: int, stream: int) -> None:
    check(lib().to_graph_launch(ctypes.c_void_p(handle), ctypes.c_void_p(stream)))


def graph_destroy(handle: int) -> None:
    check(lib().to_graph_destroy(ctypes.c_void_p(handle)))


def propagate_backward(jobs, grads, dtype: int, stream: int, plain: bool = False) -> None:
    fn = lib().to_propagate_backward_plain if plain else lib().to_propagate_backward
    check(fn(jobs_array(jobs), grads_array(grads), len(jobs), dtype, ctypes.c_void_p(stream)))


def coherence_propagate(job, dtype: int, adjoint: bool, grad, stream: int) -> None:
    jp = ctypes.byref(job)
    gp = ctypes.byref(grad) if grad is not None else None
    check(lib().to_coherence_propagate(jp, dtype, 1 if adjoint else 0, gp, ctypes.c_void_p(stream)))


def autotune(job, dtype: int, stream: int) -> dict:
    p = Plan()
    check(lib().to_autotune(ctypes.byref(job), dtype, ctypes.c_void_p(stream), ctypes.byref(p)))
    return _plan_dict(p)


def transfer_table(job, dtype: int, table: int, stream: int) -> None:
    check(lib().to_transfer_table(ctypes.byref(job), dtype, ctypes.c_void_p(table), ctypes.c_void_p(stream)))


def resample(src: int, dst: int, grid_in, grid_out, batch: int, interp: int, adjoint: bool, dtype: int,
             stream: int) -> None:
    check(lib().to_resample(ctypes.c_void_p(src), ctypes.c_void_p(dst), ctypes.byref(grid_in),
                            ctypes.byref(grid_out), batch, interp, 1 if adjoint else 0, dtype,
                            ctypes.c_void_p(stream)))


def resolve_method(job) -> int:
    m = ctypes.c_int32()
    check(lib().to_resolve_method(ctypes.byref(job), ctypes.byref(m)))
    return m.value


def plan_get(py: int, px: int, dtype: int):
    p = Plan()
    found = ctypes.c_int32()
    check(lib().to_plan_get(py, px, dtype, ctypes.byref(p), ctypes.byref(found)))
    return _plan_dict(p) if found.value else None


def plan_set(py: int, px: int, dtype: int, col_variant: int, chunk_mb: int, us: float = 0.0,
             row_fpb: int = 0) -> None:
    p = Plan(col_variant, chunk_mb, row_fpb, us)
    check(lib().to_plan_set(py, px, dtype, ctypes.byref(p)))


def plan_clear() -> None:
    check(lib().to_plan_clear())


def plan_load(path: str) -> None:
    check(lib().to_plan_load(os.fsencode(path)))


def plan_save(path: str) -> None:
    check(lib().to_plan_save(os.fsencode(path)))


def profile_begin() -> None:
    check(lib().to_profile_begin())


def profile_end() -> dict:
    """Stop kernel timing; returns {kernel name: (launches, total GPU ms)}."""
    L = lib()
    check(L.to_profile_end())
    out = {}
    buf = ctypes.create_string_buffer(128)
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    for i in range(L.to_profile_count()):
        check(L.to_profile_entry(i, buf, 128, ctypes.byref(n), ctypes.byref(ms)))
        out[buf.value.decode()] = (int(n.value), float(ms.value))
    return out
