"""MI355X-native batched free-space propagation (angular spectrum, Fresnel
transfer function, direct integration of the Rayleigh-Sommerfeld integral,
or the automatic choice between AS and DI by the critical distance) with
fused element modulation, after the TorchOptics paper (Filipovich &
Lvovsky, arXiv 2411.18591).

This module is a thin PyTorch binding of the C-ABI in ``include/toprop.h``:
it marshals tensor pointers, shapes and physical parameters into ``to_job``
records and calls ``libtoprop.so`` on the current HIP stream.  Every step of
the computation runs in the library's HIP kernels; PyTorch only provides
device memory and streams.

Fields are complex64 (FP32 arithmetic, FP64 transfer-function phases) or
complex128 tensors of shape ``[..., ny, nx]`` (scalar) or ``[..., 3, ny, nx]``
(polarized, ``ncomp=3``), contiguous, on a GPU.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _capi
from ._capi import ToError  # noqa: F401

__all__ = [
    "Optics", "propagate", "modulate", "propagate_backward", "coherence_propagate",
    "propagate_ad", "propagate_intensity", "propagate_jobs", "propagate_backward_jobs", "linear_polarizer", "waveplate",
    "jones3", "version", "autotune", "plan_get", "plan_set", "plan_clear", "plan_load", "plan_save",
    "transfer_table", "resolve_method", "Grid", "resample", "propagate_to",
]

ASM = "asm"
FRESNEL = "fresnel"
DI = "di"
AUTO = "auto"
_METHODS = {ASM: _capi.TO_ASM, FRESNEL: _capi.TO_FRESNEL, DI: _capi.TO_DI, AUTO: _capi.TO_AUTO}
_METHOD_NAMES = {v: k for k, v in _METHODS.items()}


def version() -> str:
    return _capi.lib().to_version().decode()


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.complex64:
        return _capi.TO_C64
    if t.dtype == torch.complex128:
        return _capi.TO_C128
    raise TypeError(f"fields must be complex64 or complex128, got {t.dtype}")


def _real_dtype(t: torch.Tensor):
    return torch.float32 if t.dtype == torch.complex64 else torch.float64


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _need(t: torch.Tensor, name: str, dtype, like: torch.Tensor, shape=None) -> torch.Tensor:
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != like.device:
        raise ValueError(f"{name} must be on {like.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


# ---------------------------------------------------------------------------
# Jones matrices of standard elements (section "Polarization")
# ---------------------------------------------------------------------------

def linear_polarizer(theta: float):
    """3x3 Jones matrix (the 2x2 matrix on (Ex, Ey), J_zz = 1) of a linear
    polarizer whose axis is at angle theta from x (to_jones_linear_polarizer)."""
    return _capi.jones_linear_polarizer(theta)


def waveplate(theta: float, retardance: float):
    """3x3 Jones matrix of a waveplate, fast axis at theta, retardance Gamma
    (to_jones_waveplate)."""
    return _capi.jones_waveplate(theta, retardance)


def jones3(*mats):
    """Product of 3x3 Jones matrices applied left to right (the first
    argument acts first), composed by to_jones_compose; no argument gives
    the identity."""
    J = [[1 + 0j if r == c else 0j for c in range(3)] for r in range(3)]
    for M in mats:
        J = _capi.jones_compose(J, M)
    return J


# ---------------------------------------------------------------------------
# Job marshalling
# ---------------------------------------------------------------------------

def next_pow2(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p


def next_smooth(n: int) -> int:
    """The least m >= max(n, 3) whose prime factors are all at most 7."""
    m = max(int(n), 3)
    while True:
        r = m
        for q in (2, 3, 5, 7):
            while r % q == 0:
                r //= q
        if r == 1:
            return m
        m += 1


@dataclass
class Optics:
    """Geometry and free-space parameters of one propagation.

    The padded grid is ``padded`` = (py, px) if given, else each extent is
    ``pad`` times the field, rounded up to a power of two unless
    ``round_pow2`` is False (extents that are not powers of two, up to 4096,
    run through the unfused path with mixed-radix or Bluestein transforms);
    with ``round_pow2=False`` and ``round_smooth=True`` it is rounded up to
    the next length of the form 2^a 3^b 5^c 7^d instead (2002 -> 2016), which
    keeps it on the mixed-radix transforms.  ``method`` is
    "asm", "fresnel", "di" (direct integration; needs pad >= 2 and z > 0) or
    "auto" (DI at or beyond the critical distance, AS below it)."""
    dy: float
    dx: float
    wavelength: float
    z: float
    method: str = ASM
    pad: int = 2
    y0: float = 0.0
    x0: float = 0.0
    padded: Optional[tuple] = None
    round_pow2: bool = True
    round_smooth: bool = False

    def padded_shape(self, ny: int, nx: int):
        if self.padded is not None:
            return int(self.padded[0]), int(self.padded[1])
        if not self.round_pow2:
            if self.round_smooth:
                return next_smooth(self.pad * ny), next_smooth(self.pad * nx)
            return self.pad * ny, self.pad * nx
        return next_pow2(self.pad * ny), next_pow2(self.pad * nx)


def _field_dims(u: torch.Tensor, ncomp: int):
    if u.dim() < 2 + (1 if ncomp == 3 else 0):
        raise ValueError("field tensor has too few dimensions")
    ny, nx = u.shape[-2], u.shape[-1]
    lead = u.shape[:-3] if ncomp == 3 else u.shape[:-2]
    if ncomp == 3 and u.shape[-3] != 3:
        raise ValueError("polarized fields need a component axis of size 3")
    batch = 1
    for d in lead:
        batch *= int(d)
    return int(ny), int(nx), batch


def make_job(u: torch.Tensor, opt: Optics, *, out: Optional[torch.Tensor] = None, ncomp: int = 1,
             phase=None, cmask=None, lens_f=None, jones=None, jones_map=None, epi: int = _capi.TO_EPI_NONE,
             epi_ref=None, epi_scale: float = 1.0, epi_grad=None, epi_loss=None, epi_out=None,
             tf_table=None):
    """Fill a to_job record for field tensor u (and the given element /
    epilogue tensors; ``tf_table``: a direct-integration table from
    :func:`transfer_table`, reused instead of being rebuilt in the call).
    Returns the record; the caller keeps the tensors alive until the stream
    work is done."""
    if not u.is_contiguous():
        raise ValueError("field must be contiguous")
    _dtype_code(u)
    rdt = _real_dtype(u)
    ny, nx, batch = _field_dims(u, ncomp)
    j = _capi.Job()
    j.ny, j.nx = ny, nx
    j.py, j.px = opt.padded_shape(ny, nx)
    if opt.method not in _METHODS:
        raise ValueError(f"method must be one of {list(_METHODS)}")
    j.method = _METHODS[opt.method]
    j.dy, j.dx, j.wavelength, j.z = float(opt.dy), float(opt.dx), float(opt.wavelength), float(opt.z)
    j.y0, j.x0 = float(opt.y0), float(opt.x0)
    j.batch = batch
    j.ncomp = ncomp
    flags = 0
    if phase is not None:
        _need(phase, "phase", rdt, u, (ny, nx))
        j.el_phase = _ptr(phase)
        flags |= _capi.TO_EL_PHASE
    if cmask is not None:
        _need(cmask, "cmask", u.dtype, u, (ny, nx))
        j.el_complex = _ptr(cmask)
        flags |= _capi.TO_EL_COMPLEX
    if lens_f is not None:
        j.el_f = float(lens_f)
        flags |= _capi.TO_EL_LENS
    if jones is not None:
        flat = []
        for r in range(3):
            for c in range(3):
                v = complex(jones[r][c])
                flat += [v.real, v.imag]
        j.el_jones[:] = flat
        flags |= _capi.TO_EL_JONES
    if jones_map is not None:
        _need(jones_map, "jones_map", u.dtype, u, (3, 3, ny, nx))
        j.el_jones_map = _ptr(jones_map)
        flags |= _capi.TO_EL_JONES_MAP
    j.el_flags = flags
    j.epi = int(epi)
    if epi in (_capi.TO_EPI_MSE, _capi.TO_EPI_WEIGHTED):
        _need(epi_ref, "epi_ref", rdt, u, (ny, nx))
        _need(epi_grad, "epi_grad", u.dtype, u, tuple(u.shape))
        _need(epi_loss, "epi_loss", torch.float64, u)
        j.epi_ref, j.epi_grad, j.epi_loss = _ptr(epi_ref), _ptr(epi_grad), _ptr(epi_loss)
    elif epi == _capi.TO_EPI_INTENSITY:
        _need(epi_out, "epi_out", rdt, u)
        if epi_out.numel() != batch * ny * nx:
            raise ValueError(f"epi_out must hold {batch} x {ny} x {nx} intensities")
        j.epi_out = _ptr(epi_out)
    elif epi != _capi.TO_EPI_NONE:
        raise ValueError(f"unknown epilogue {epi}")
    j.epi_scale = float(epi_scale)
    j.in_ = _ptr(u)
    if out is not None:
        _need(out, "out", u.dtype, u, tuple(u.shape))
        j.out = _ptr(out)
    if tf_table is not None:
        _need(tf_table, "tf_table", u.dtype, u, (j.py, j.px))
        j.tf_table = _ptr(tf_table)
    return j


def _geometry_job(opt: Optics, ny: int, nx: int):
    if opt.method not in _METHODS:
        raise ValueError(f"method must be one of {list(_METHODS)}")
    j = _capi.Job()
    j.ny, j.nx = int(ny), int(nx)
    j.py, j.px = opt.padded_shape(ny, nx)
    j.method = _METHODS[opt.method]
    j.dy, j.dx, j.wavelength, j.z = float(opt.dy), float(opt.dx), float(opt.wavelength), float(opt.z)
    j.y0, j.x0 = float(opt.y0), float(opt.x0)
    j.ncomp = 1
    return j


def transfer_table(opt: Optics, ny: int, nx: int, dtype=torch.complex64, device=None) -> torch.Tensor:
    """The transfer function ``[py, px]`` (FFT order) the library applies to
    ny x nx fields under ``opt``; for direct integration, the DFT of the
    sampled impulse response, which a job may carry (``make_job(...,
    tf_table=...)``) so that calls with the same geometry skip building it.
    Computed on the GPU, on the current stream."""
    j = _geometry_job(opt, ny, nx)
    dev = torch.device("cuda") if device is None else torch.device(device)
    H = torch.empty((j.py, j.px), dtype=dtype, device=dev)
    code = _dtype_code(H)
    _capi.transfer_table(j, code, H.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
    return H


@dataclass
class Grid:
    """A sampling grid: ny x nx samples of spacing (dy, dx), offset (y0, x0)
    from the optical axis (sample ny//2, nx//2 on it when the offset is 0)."""
    ny: int
    nx: int
    dy: float
    dx: float
    y0: float = 0.0
    x0: float = 0.0

    def _rec(self):
        g = _capi.Grid()
        g.ny, g.nx = int(self.ny), int(self.nx)
        g.dy, g.dx, g.y0, g.x0 = float(self.dy), float(self.dx), float(self.y0), float(self.x0)
        return g


_INTERP = {"nearest": _capi.TO_NEAREST, "bilinear": _capi.TO_BILINEAR}


def resample(u: torch.Tensor, grid_in: Grid, grid_out: Grid, interp: str = "bilinear", *,
             adjoint: bool = False, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Interpolate fields ``[..., ny, nx]`` on ``grid_in`` onto ``grid_out``
    (``adjoint``: the transpose map, from a gradient on grid_out to one on
    grid_in).  Zero outside the input window."""
    if interp not in _INTERP:
        raise ValueError(f"interp must be one of {list(_INTERP)}")
    src_g, dst_g = (grid_out, grid_in) if adjoint else (grid_in, grid_out)
    if tuple(u.shape[-2:]) != (src_g.ny, src_g.nx):
        raise ValueError(f"field must end in ({src_g.ny}, {src_g.nx})")
    if not u.is_contiguous():
        raise ValueError("field must be contiguous")
    batch = u.numel() // (src_g.ny * src_g.nx)
    shape = tuple(u.shape[:-2]) + (dst_g.ny, dst_g.nx)
    if out is None:
        out = torch.empty(shape, dtype=u.dtype, device=u.device)
    _need(out, "out", u.dtype, u, shape)
    _capi.resample(u.data_ptr(), out.data_ptr(), grid_in._rec(), grid_out._rec(), batch, _INTERP[interp], adjoint,
                   _dtype_code(u), _stream(u))
    return out


def propagate_to(u: torch.Tensor, opt: Optics, grid_out: Grid, interp: str = "bilinear", **element) -> torch.Tensor:
    """Propagation onto a grid of other spacing (section "Computational
    Fourier optics"): propagate on the input grid (spacing and window of u),
    then interpolate onto ``grid_out``; the output window reads zero beyond
    the input window."""
    ny, nx = u.shape[-2], u.shape[-1]
    mid = propagate(u, opt, **element)
    return resample(mid, Grid(ny, nx, opt.dy, opt.dx, opt.y0, opt.x0), grid_out, interp)


def resolve_method(opt: Optics, ny: int, nx: int) -> str:
    """The method the library runs for ny x nx fields under ``opt`` ("auto"
    resolved by the critical distance)."""
    return _METHOD_NAMES[_capi.resolve_method(_geometry_job(opt, ny, nx))]


# ---------------------------------------------------------------------------
# Entry points
# ---------------------------------------------------------------------------

def propagate(u: torch.Tensor, opt: Optics, *, out: Optional[torch.Tensor] = None, ncomp: int = 1,
              plain: bool = False, **element) -> torch.Tensor:
    """out = P_z(M u): modulation by the element (phase=, cmask=, lens_f=,
    jones=) fused into the first pass, then zero-padded propagation."""
    if out is None:
        out = torch.empty_like(u)
    job = make_job(u, opt, out=out, ncomp=ncomp, **element)
    _capi.propagate([job], _dtype_code(u), _stream(u), plain=plain)
    return out


def propagate_loss(u: torch.Tensor, opt: Optics, *, kind: str, ref: torch.Tensor, scale: float,
                   out: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None,
                   loss: Optional[torch.Tensor] = None, ncomp: int = 1, plain: bool = False,
                   **element):
    """Forward propagation with a fused intensity-loss epilogue ("mse" or
    "weighted").  Returns (out, dL/d(out), loss) where loss is a float64
    device scalar (accumulated into `loss` if given)."""
    epi = {"mse": _capi.TO_EPI_MSE, "weighted": _capi.TO_EPI_WEIGHTED}[kind]
    out = torch.empty_like(u) if out is None else out
    grad = torch.empty_like(u) if grad is None else grad
    loss = torch.zeros((), dtype=torch.float64, device=u.device) if loss is None else loss
    job = make_job(u, opt, out=out, ncomp=ncomp, epi=epi, epi_ref=ref, epi_scale=scale,
                   epi_grad=grad, epi_loss=loss, **element)
    _capi.propagate([job], _dtype_code(u), _stream(u), plain=plain)
    return out, grad, loss


def propagate_intensity(u: torch.Tensor, opt: Optics, *, intensity: Optional[torch.Tensor] = None,
                        weight: float = 1.0, out: Optional[torch.Tensor] = None, ncomp: int = 1,
                        **element) -> torch.Tensor:
    """Detected intensity after propagation: ``intensity[b] += weight *
    sum_c |P_z(M u)_c|^2`` (shape [batch, ny, nx], real, accumulated; zeros
    if not given).  Called once per wavelength with a shared ``intensity``
    and the wavelength's weight, this is the incoherent polychromatic sum of
    Eq. (I_poly).  The propagated field is stored only if ``out`` is given."""
    ny, nx, batch = _field_dims(u, ncomp)
    if intensity is None:
        intensity = torch.zeros((batch, ny, nx), dtype=_real_dtype(u), device=u.device)
    job = make_job(u, opt, out=out, ncomp=ncomp, epi=_capi.TO_EPI_INTENSITY, epi_out=intensity,
                   epi_scale=weight, **element)
    _capi.propagate([job], _dtype_code(u), _stream(u))
    return intensity


def modulate(u: torch.Tensor, *, dy: float, dx: float, wavelength: float, y0: float = 0.0,
             x0: float = 0.0, adjoint: bool = False, out: Optional[torch.Tensor] = None,
             ncomp: int = 1, **element) -> torch.Tensor:
    """out = M u (or M^H u), Eq. (field_modulation) / the Jones product."""
    if out is None:
        out = torch.empty_like(u)
    opt = Optics(dy=dy, dx=dx, wavelength=wavelength, z=0.0, pad=1, y0=y0, x0=x0, padded=(8, 8))
    job = make_job(u, opt, out=out, ncomp=ncomp, **element)
    _capi.modulate([job], _dtype_code(u), adjoint, _stream(u))
    return out


def propagate_backward(grad_out: torch.Tensor, opt: Optics, *, saved_in=None, want_grad_in=True,
                       grad_in=None, grad_phase=None, grad_f=None, ncomp: int = 1, plain: bool = False,
                       **element):
    """Backward of :func:`propagate`: returns dL/d(in) (or None); element
    gradients are accumulated into grad_phase / grad_f (device tensors)."""
    job = make_job(grad_out, opt, ncomp=ncomp, **element)
    job.in_ = None
    g = _capi.Grad()
    g.grad_out = _ptr(grad_out)
    if want_grad_in:
        grad_in = torch.empty_like(grad_out) if grad_in is None else grad_in
        g.grad_in = _ptr(grad_in)
    else:
        grad_in = None
    if saved_in is not None:
        _need(saved_in, "saved_in", grad_out.dtype, grad_out, tuple(grad_out.shape))
        g.saved_in = _ptr(saved_in)
    if grad_phase is not None:
        g.grad_phase = _ptr(_need(grad_phase, "grad_phase", _real_dtype(grad_out), grad_out,
                                  grad_out.shape[-2:]))
    if grad_f is not None:
        g.grad_f = _ptr(_need(grad_f, "grad_f", torch.float64, grad_out))
    _capi.propagate_backward([job], [g], _dtype_code(grad_out), _stream(grad_out), plain=plain)
    return grad_in


def _common_dtype(tensors) -> int:
    codes = {_dtype_code(t) for t in tensors}
    devs = {t.device for t in tensors}
    if len(codes) != 1 or len(devs) != 1:
        raise ValueError("all jobs of one call must share the dtype and the device")
    return codes.pop()


class Graph:
    """A library call captured into a HIP graph owned by the library
    (`to_graph_create`): :meth:`launch` replays it on a stream, reading and
    writing the tensors the call named (keep them alive; refill them in
    place).  Returned by ``propagate_jobs(..., graph=True)`` and
    ``propagate_backward_jobs(..., graph=True)``."""

    def __init__(self, handle: int, tensors, device):
        self._h = handle
        self._keep = list(tensors)  # the captured addresses stay valid
        self._device = device

    def launch(self, stream: Optional[torch.cuda.Stream] = None) -> None:
        if self._h is None:
            raise RuntimeError("graph was closed")
        s = stream if stream is not None else torch.cuda.current_stream(self._device)
        _capi.graph_launch(self._h, s.cuda_stream)

    def close(self) -> None:
        if self._h is not None:
            _capi.graph_destroy(self._h)
            self._h = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def propagate_jobs(fields: Sequence[torch.Tensor], opts: Sequence[Optics], *, outs=None, elements=None,
                   ncomp: int = 1, plain: bool = False, graph: bool = False):
    """One library call over several independent propagations, each with its
    own grid, optics and element (the uneven batch).  Independent jobs run
    concurrently on the library's lanes; a job that reads what an earlier job
    of the call writes runs after it.  Returns the output tensors; with
    ``graph=True`` the call also is captured (after running once) and
    ``(outs, Graph)`` is returned."""
    n = len(fields)
    if len(opts) != n:
        raise ValueError("one Optics per field")
    outs = [torch.empty_like(u) for u in fields] if outs is None else list(outs)
    elements = [{}] * n if elements is None else list(elements)
    if n == 0:
        return outs
    dt = _common_dtype(fields)
    jobs = [make_job(u, o, out=y, ncomp=ncomp, **el) for u, o, y, el in zip(fields, opts, outs, elements)]
    if graph:
        if plain:
            raise ValueError("graph=True captures the fused call")
        h = _capi.graph_create(jobs, None, dt, _stream(fields[0]))
        kept = list(fields) + list(outs) + [v for el in elements for v in el.values() if isinstance(v, torch.Tensor)]
        return outs, Graph(h, kept, fields[0].device)
    _capi.propagate(jobs, dt, _stream(fields[0]), plain=plain)
    return outs


def propagate_backward_jobs(grads_out: Sequence[torch.Tensor], opts: Sequence[Optics], *, saved_ins=None,
                            grad_ins=None, grad_phases=None, grad_fs=None, elements=None, ncomp: int = 1,
                            plain: bool = False, transient=None, graph: bool = False):
    """Backward of :func:`propagate_jobs` in one call: returns dL/d(in) per
    job (``grad_ins[i]`` None: not formed); element gradients accumulate
    into ``grad_phases[i]`` / ``grad_fs[i]`` (jobs that share a gradient
    tensor are run in call order on one lane).  ``transient[i]`` True:
    ``grad_ins[i]`` only links job i to job i + 1 (its grad_out), and may be
    left unwritten where the library fuses the two layers."""
    n = len(grads_out)
    if len(opts) != n:
        raise ValueError("one Optics per gradient")
    grad_ins = [torch.empty_like(g) for g in grads_out] if grad_ins is None else list(grad_ins)
    saved_ins = [None] * n if saved_ins is None else list(saved_ins)
    grad_phases = [None] * n if grad_phases is None else list(grad_phases)
    grad_fs = [None] * n if grad_fs is None else list(grad_fs)
    elements = [{}] * n if elements is None else list(elements)
    transient = [False] * n if transient is None else list(transient)
    if n == 0:
        return grad_ins
    dt = _common_dtype(grads_out)
    jobs, grs = [], []
    for go, o, gi, si, gp, gf, el, tr in zip(grads_out, opts, grad_ins, saved_ins, grad_phases, grad_fs, elements,
                                             transient):
        j = make_job(go, o, ncomp=ncomp, **el)
        j.in_ = None
        g = _capi.Grad()
        g.grad_out = _ptr(go)
        if gi is not None:
            g.grad_in = _ptr(_need(gi, "grad_in", go.dtype, go, tuple(go.shape)))
        if si is not None:
            g.saved_in = _ptr(_need(si, "saved_in", go.dtype, go, tuple(go.shape)))
        if gp is not None:
            g.grad_phase = _ptr(_need(gp, "grad_phase", _real_dtype(go), go, go.shape[-2:]))
        if gf is not None:
            g.grad_f = _ptr(_need(gf, "grad_f", torch.float64, go))
        g.flags = _capi.TO_GRAD_IN_TRANSIENT if tr else 0
        jobs.append(j)
        grs.append(g)
    if graph:
        if plain:
            raise ValueError("graph=True captures the fused call")
        h = _capi.graph_create(jobs, grs, dt, _stream(grads_out[0]))
        kept = [t for t in list(grads_out) + grad_ins + saved_ins + grad_phases + grad_fs if isinstance(t, torch.Tensor)]
        kept += [v for el in elements for v in el.values() if isinstance(v, torch.Tensor)]
        return grad_ins, Graph(h, kept, grads_out[0].device)
    _capi.propagate_backward(jobs, grs, dt, _stream(grads_out[0]), plain=plain)
    return grad_ins


def autotune(u: torch.Tensor, opt: Optics, *, out: Optional[torch.Tensor] = None, ncomp: int = 1,
             **element):
    """Time the launch schedules for this field's padded grid and dtype,
    keep the fastest in the library's plan table (used by every later call
    of that shape), and propagate u once with it.  Returns (out, plan)."""
    if out is None:
        out = torch.empty_like(u)
    job = make_job(u, opt, out=out, ncomp=ncomp, **element)
    plan = _capi.autotune(job, _dtype_code(u), _stream(u))
    return out, plan


def _dtype_of(dtype) -> int:
    if dtype in (torch.complex64, "c64"):
        return _capi.TO_C64
    if dtype in (torch.complex128, "c128"):
        return _capi.TO_C128
    raise TypeError("dtype must be torch.complex64 or torch.complex128")


def plan_get(py: int, px: int, dtype=torch.complex64):
    """The plan stored for a padded grid and dtype, or None."""
    return _capi.plan_get(py, px, _dtype_of(dtype))


def plan_set(py: int, px: int, col_variant: int, chunk_mb: int, dtype=torch.complex64, us: float = 0.0,
             row_fpb: int = 0):
    _capi.plan_set(py, px, _dtype_of(dtype), col_variant, chunk_mb, us, row_fpb)


def plan_clear():
    _capi.plan_clear()


def plan_load(path: str):
    """Merge a plan file into the table (rejected whole if any line is bad)."""
    _capi.plan_load(path)


def plan_save(path: str):
    _capi.plan_save(path)


def coherence_propagate(gamma: torch.Tensor, opt: Optics, *, adjoint: bool = False,
                        out: Optional[torch.Tensor] = None, saved_in=None, grad_phase=None,
                        loss_kind: Optional[str] = None, loss_ref=None, loss_scale: float = 1.0,
                        loss=None, loss_grad=None, **element):
    """Propagate a mutual coherence function [ny, nx, ny, nx] (section
    "Spatial coherence"): P (M G M^H) P^H, or its adjoint M^H P^H G P M.

    With ``loss_kind`` ("mse" or "weighted", forward only) the loss of the
    output intensity Re Gamma(r, r) against ``loss_ref`` is accumulated into
    ``loss`` and its gradient dL/dGamma_out written to ``loss_grad``; the
    call then returns (out, loss_grad, loss).  With ``loss_kind="intensity"``
    the call returns (out, I) with I[y, x] += loss_scale * Re Gamma(r, r)
    (I = ``loss_grad`` if given, else a new zero tensor).  With ``adjoint`` and
    ``grad_phase``, dL/dphi of the phase element is accumulated using
    ``saved_in`` (the forward input)."""
    ny, nx = int(gamma.shape[0]), int(gamma.shape[1])
    if gamma.dim() != 4 or tuple(gamma.shape) != (ny, nx, ny, nx):
        raise ValueError("gamma must be [ny, nx, ny, nx]")
    if not gamma.is_contiguous():
        raise ValueError("gamma must be contiguous")
    if out is None:
        out = torch.empty_like(gamma)
    _need(out, "out", gamma.dtype, gamma, tuple(gamma.shape))
    epi = {}
    if loss_kind == "intensity":
        # time-averaged intensity Re Gamma(r, r), accumulated (scaled) into loss_grad
        inten = torch.zeros((ny, nx), dtype=_real_dtype(gamma), device=gamma.device) if loss_grad is None \
            else loss_grad
        _need(inten, "intensity", _real_dtype(gamma), gamma, (ny, nx))
        job = make_job(gamma[0, 0], opt, ncomp=1, **element)
        job.epi = _capi.TO_EPI_INTENSITY
        job.epi_scale = float(loss_scale)
        job.epi_out = _ptr(inten)
        job.batch = 1
        job.in_ = _ptr(gamma)
        job.out = _ptr(out)
        _capi.coherence_propagate(job, _dtype_code(gamma), adjoint, None, _stream(gamma))
        return out, inten
    if loss_kind is not None:
        loss_grad = torch.empty_like(gamma) if loss_grad is None else loss_grad
        loss = torch.zeros((), dtype=torch.float64, device=gamma.device) if loss is None else loss
        _need(loss_grad, "loss_grad", gamma.dtype, gamma, tuple(gamma.shape))
        epi = dict(epi={"mse": _capi.TO_EPI_MSE, "weighted": _capi.TO_EPI_WEIGHTED}[loss_kind],
                   epi_ref=loss_ref, epi_scale=loss_scale, epi_grad=loss_grad[0, 0], epi_loss=loss)
    job = make_job(gamma[0, 0], opt, ncomp=1, **element, **epi)  # grid, element, epilogue
    job.batch = 1
    job.in_ = _ptr(gamma)
    job.out = _ptr(out)
    if loss_kind is not None:
        job.epi_grad = _ptr(loss_grad)
    g = None
    if adjoint and (saved_in is not None or grad_phase is not None):
        g = _capi.Grad()
        if saved_in is not None:
            g.saved_in = _ptr(_need(saved_in, "saved_in", gamma.dtype, gamma, tuple(gamma.shape)))
        if grad_phase is not None:
            g.grad_phase = _ptr(_need(grad_phase, "grad_phase", _real_dtype(gamma), gamma, (ny, nx)))
    _capi.coherence_propagate(job, _dtype_code(gamma), adjoint, g, _stream(gamma))
    if loss_kind is not None:
        return out, loss_grad, loss
    return out


# ---------------------------------------------------------------------------
# Autograd
# ---------------------------------------------------------------------------

class _Propagate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, phase, lens_f, opt, ncomp, jones, cmask):
        ctx.opt, ctx.ncomp, ctx.jones, ctx.lens_f_value = opt, ncomp, jones, None
        el = {}
        if phase is not None:
            el["phase"] = phase.detach().contiguous()
        if lens_f is not None:
            ctx.lens_f_value = float(lens_f)
            el["lens_f"] = ctx.lens_f_value
        if jones is not None:
            el["jones"] = jones
        if cmask is not None:
            el["cmask"] = cmask.detach().contiguous()
        ctx.el = el
        u = u.detach().contiguous()
        out = propagate(u, opt, ncomp=ncomp, **el)
        ctx.save_for_backward(u)
        ctx.has_phase = phase is not None
        ctx.has_lens = lens_f is not None
        ctx.lens_requires = lens_f is not None and isinstance(lens_f, torch.Tensor) and lens_f.requires_grad
        ctx.phase_requires = phase is not None and phase.requires_grad
        return out

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        g = g.contiguous()
        gp = torch.zeros_like(ctx.el["phase"]) if ctx.phase_requires else None
        gf = torch.zeros((), dtype=torch.float64, device=g.device) if ctx.lens_requires else None
        need_param = gp is not None or gf is not None
        gin = propagate_backward(g, ctx.opt, saved_in=u if need_param else None,
                                 want_grad_in=ctx.needs_input_grad[0], grad_phase=gp, grad_f=gf,
                                 ncomp=ctx.ncomp, **ctx.el)
        gf_out = None
        if gf is not None:
            gf_out = gf.to(torch.float64)
        return gin, gp, gf_out, None, None, None, None


def propagate_ad(u: torch.Tensor, opt: Optics, *, phase=None, lens_f=None, jones=None, cmask=None,
                 ncomp: int = 1) -> torch.Tensor:
    """Differentiable P_z(M u) with respect to u, the phase mask and the lens
    focal length (pass lens_f as a 0-d float64 tensor with requires_grad)."""
    return _Propagate.apply(u, phase, lens_f, opt, ncomp, jones, cmask)
