"""Seeded synthetic inputs for the propagation workloads.

This module is shared by the GPU path's tests/benchmark and by the FP64
oracle, and therefore holds NONE of the method's arithmetic: no transfer
functions, no modulation, no Fourier transforms.  It only draws random
numbers and builds input profiles (beam amplitudes, blurred noise, a
Gaussian Schell-model coherence function, per-job parameters).

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64), drawn in
float64, and are cast to the workload's storage type at the end so that both
sides receive bit-identical inputs (the oracle promotes them to float64).

The paper's own inputs (``input_data.pt``, ``target.pt``) are not available;
the workloads below replace them with seeded stand-ins of the same kind
(beam profiles, random phase masks, smooth random targets).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def grid_axis(n: int, d: float, offset: float = 0.0) -> np.ndarray:
    """Sample positions ``(k - n // 2) * d + offset`` of a length-n axis."""
    return (np.arange(n) - n // 2) * float(d) + float(offset)


def gaussian_kernel1d(sigma: float) -> np.ndarray:
    r = int(math.ceil(4.0 * sigma))
    t = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-0.5 * (t / sigma) ** 2)
    return k / k.sum()


def gaussian_blur(a: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur over the last two axes (taps |k| <= 4 sigma,
    normalised, reflect boundary)."""
    k = gaussian_kernel1d(sigma)
    r = (k.size - 1) // 2
    out = np.asarray(a, dtype=np.float64)
    for axis in (-1, -2):
        n = out.shape[axis]
        pad = [(0, 0)] * out.ndim
        pad[axis] = (r, r)
        p = np.pad(out, pad, mode="symmetric")
        acc = np.zeros_like(out)
        for i, w in enumerate(k):
            sl = [slice(None)] * out.ndim
            sl[axis] = slice(i, i + n)
            acc += w * p[tuple(sl)]
        out = acc
    return out


def blurred_uniform(seed: int, shape, sigma: float) -> np.ndarray:
    """U[0,1) noise (float64) of the given shape, Gaussian-blurred."""
    rng = np.random.default_rng(seed)
    return gaussian_blur(rng.random(shape), sigma)


def uniform_phase(seed: int, shape) -> np.ndarray:
    """U[0, 2 pi) phases, float64."""
    return np.random.default_rng(seed).random(shape) * (2.0 * math.pi)


def gaussian_amplitude(ny: int, nx: int, dy: float, dx: float, w0: float) -> np.ndarray:
    """Gaussian beam amplitude ``exp(-r^2 / w0^2)`` (w0 = 1/e^2 intensity
    radius) on the integer-centred grid, float64."""
    y = grid_axis(ny, dy)[:, None]
    x = grid_axis(nx, dx)[None, :]
    return np.exp(-(x * x + y * y) / (w0 * w0))


def gaussian_schell(n: int, d: float, w0: float, sigma_c: float) -> np.ndarray:
    """Gaussian Schell-model mutual coherence ``[n, n, n, n]`` (float64):
    ``exp(-(|r1|^2 + |r2|^2) / w0^2) * exp(-|r1 - r2|^2 / (2 sigma_c^2))``."""
    a = grid_axis(n, d)
    y1 = a[:, None, None, None]
    x1 = a[None, :, None, None]
    y2 = a[None, None, :, None]
    x2 = a[None, None, None, :]
    inten = np.exp(-(x1 * x1 + y1 * y1 + x2 * x2 + y2 * y2) / (w0 * w0))
    mu = np.exp(-((x1 - x2) ** 2 + (y1 - y2) ** 2) / (2.0 * sigma_c * sigma_c))
    return inten * mu


# ---------------------------------------------------------------------------
# Workload definitions
# ---------------------------------------------------------------------------

@dataclass
class GaussianLensWorkload:
    """Single scalar field 256x256 (complex128), spacing 10 um, 700 nm,
    Gaussian waist 200 um; AS propagation 5 cm (2x padding), thin lens
    f = 10 cm, AS propagation 10 cm."""
    n: int = 256
    d: float = 10e-6
    wavelength: float = 700e-9
    w0: float = 200e-6
    z1: float = 0.05
    f: float = 0.10
    z2: float = 0.10
    pad: int = 2

    def field(self) -> np.ndarray:
        return gaussian_amplitude(self.n, self.n, self.d, self.d, self.w0).astype(np.complex128)


@dataclass
class DiffractiveNetWorkload:
    """Batch of input fields through L trainable phase masks, AS propagation
    between layers, MSE loss of output intensity against a target.

    Default: 64 fields of 1024^2 complex64, amplitude = U[0,1) noise blurred
    with sigma 4 px (seeds 2001..), zero phase; 5 masks U[0, 2 pi) (seeds
    2011..2015); z = 10 cm, spacing 8 um, 700 nm, 2x padding; target =
    blurred U[0,1) squared (seed 2021)."""
    batch: int = 64
    n: int = 1024
    layers: int = 5
    d: float = 8e-6
    wavelength: float = 700e-9
    z: float = 0.10
    pad: int = 2
    sigma: float = 4.0

    def fields(self, count: int | None = None) -> np.ndarray:
        """complex64 [count, n, n]; field b uses seed 2001 + b, so any
        subset can be regenerated on its own."""
        count = self.batch if count is None else count
        out = np.empty((count, self.n, self.n), dtype=np.complex64)
        for b in range(count):
            out[b] = blurred_uniform(2001 + b, (self.n, self.n), self.sigma).astype(np.complex64)
        return out

    def masks(self) -> np.ndarray:
        return np.stack([uniform_phase(2011 + l, (self.n, self.n)) for l in range(self.layers)]
                        ).astype(np.float32)

    def target(self) -> np.ndarray:
        t = blurred_uniform(2021, (self.n, self.n), self.sigma)
        return (t * t).astype(np.float32)


@dataclass
class Polychromatic4fWorkload:
    """Wide-band light through a 4f imaging system (the polychromatic
    example of the paper's "Polychromatic fields" section, on the 4f system
    of its first listing): 1000^2 grid, 10 um spacing, lenses f = 200 mm at
    z = f and z = 3f, image at z = 4f; 251 wavelengths evenly spaced over
    575-825 nm with Gaussian spectral weights (mean 700 nm, FWHM 10, 20, 40
    or 80 nm, normalised to unit sum); the detected image is the
    weight-summed intensity (Eq. (I_poly)).

    The paper's input file is not available: the input is a stand-in with
    uniform phase and the amplitude of U[0,1) noise blurred with sigma 6 px
    (seed 6001), squared for contrast, complex64.  Padding 2x (1000 ->
    2048, the next power of two)."""
    n: int = 1000
    d: float = 10e-6
    f: float = 0.2
    count: int = 251
    lam_lo: float = 575e-9
    lam_hi: float = 825e-9
    mean: float = 700e-9
    fwhm: float = 10e-9
    pad: int = 2

    def wavelengths(self) -> np.ndarray:
        return np.linspace(self.lam_lo, self.lam_hi, self.count)

    def weights(self) -> np.ndarray:
        """Gaussian spectrum exp(-4 ln 2 (lambda - mean)^2 / FWHM^2),
        normalised to unit sum (float64)."""
        lam = self.wavelengths()
        w = np.exp(-4.0 * math.log(2.0) * ((lam - self.mean) / self.fwhm) ** 2)
        return w / w.sum()

    def field(self, n: int | None = None) -> np.ndarray:
        n = self.n if n is None else n
        a = blurred_uniform(6001, (n, n), 6.0)
        a = (a - a.min()) / (a.max() - a.min())
        return (a * a).astype(np.complex64)


@dataclass
class PolarizedWorkload:
    """3-component field x W wavelengths, Fresnel propagation after a
    quarter-wave plate (fast axis 45 deg), a linear polarizer (30 deg) and a
    thin lens; weighted-intensity loss, gradient to the focal length."""
    n: int = 2048
    d: float = 4e-6
    wavelengths: tuple = tuple(np.linspace(450e-9, 700e-9, 8))
    w0: float = 1e-3
    f: float = 0.20
    z: float = 0.20
    pad: int = 2
    qwp_angle: float = math.pi / 4
    lp_angle: float = math.pi / 6
    sigma: float = 8.0

    def field(self) -> np.ndarray:
        """complex64 [W, 3, n, n]: x-polarised Gaussian for every wavelength."""
        g = gaussian_amplitude(self.n, self.n, self.d, self.d, self.w0).astype(np.complex64)
        E = np.zeros((len(self.wavelengths), 3, self.n, self.n), dtype=np.complex64)
        E[:, 0] = g
        return E

    def weight(self) -> np.ndarray:
        return blurred_uniform(3001, (self.n, self.n), self.sigma).astype(np.float32)


@dataclass
class CoherenceWorkload:
    """Gaussian Schell-model source (waist 150 um, coherence length 50 um),
    64^2 grid, 10 um, 633 nm; phase mask (seed 4001) and lens f = 5 cm at
    z = 0, AS propagation 5 cm, diagonal intensity, MSE to a target (seed
    4002)."""
    n: int = 64
    d: float = 10e-6
    wavelength: float = 633e-9
    w0: float = 150e-6
    sigma_c: float = 50e-6
    f: float = 0.05
    z: float = 0.05
    pad: int = 2

    def gamma(self) -> np.ndarray:
        return gaussian_schell(self.n, self.d, self.w0, self.sigma_c).astype(np.complex64)

    def mask(self) -> np.ndarray:
        return uniform_phase(4001, (self.n, self.n)).astype(np.float32)

    def target(self) -> np.ndarray:
        t = blurred_uniform(4002, (self.n, self.n), 2.0)
        return (t * t).astype(np.float32)


@dataclass
class UnevenJob:
    n: int
    wavelength: float
    z: float
    d: float
    seed_field: int
    seed_grad: int

    def field(self) -> np.ndarray:
        """Unit-amplitude random-phase field exp(i phi), complex64."""
        phi = uniform_phase(self.seed_field, (self.n, self.n))
        return (np.cos(phi) + 1j * np.sin(phi)).astype(np.complex64)

    def upstream_grad(self) -> np.ndarray:
        rng = np.random.default_rng(self.seed_grad)
        g = rng.standard_normal((self.n, self.n)) + 1j * rng.standard_normal((self.n, self.n))
        return g.astype(np.complex64)


def uneven_jobs(count: int = 128, sizes=(256, 512, 1024, 2048, 4096), seed: int = 5001):
    """Jobs with square sizes drawn uniformly from ``sizes``, wavelength
    U[400, 800] nm, distance log-uniform in [1 mm, 50 cm], spacing
    U[2, 20] um; field seeds 5100 + j, gradient seeds 5300 + j."""
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(count):
        n = int(sizes[rng.integers(len(sizes))])
        lam = float(rng.uniform(400e-9, 800e-9))
        z = float(math.exp(rng.uniform(math.log(1e-3), math.log(0.5))))
        d = float(rng.uniform(2e-6, 20e-6))
        jobs.append(UnevenJob(n, lam, z, d, 5100 + j, 5300 + j))
    return jobs
