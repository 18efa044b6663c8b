"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these tests touches the GPU.  Each check is chosen so that a
plausible slip in the oracle (a sign, a dropped term, a transposed operand,
a wrong frequency ordering or window) fails at least one of them:

* DFT/FFT: closed-form transforms, the naive DFT, numpy's FFT.
* Transfer function and frequency grid: plane waves at grid frequencies are
  eigenfunctions with the physical phase k z cos(theta); evanescent waves
  are removed.
* Pad / crop / DFT chain: brute-force circular convolution.
* Identities: z = 0, adjoint, P(-z) = P^H, Parseval, pad placement, group law.
* Physics: Gaussian-beam q-parameter closed form, the exact discrete lens
  Fourier-transform identity, the Dirichlet (discrete sinc) pattern of a
  square aperture, brute-force Rayleigh-Sommerfeld integration.
* Direct integration: the brute-force sum's impulse response against the z
  derivative of the free-space Green's function; the FFT form of the DI
  method against the brute-force sum (forward and adjoint, ragged and
  non-square grids), invariance under extra padding, the critical distance
  as the Nyquist limit of the Fresnel chirp.
* Polarization: the powers printed in the paper's polarizer listing, Malus's
  law, a quarter-wave plate plus polarizer.
* Coherence: reductions to the field propagator.
* Gradients: central finite differences.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def exact_cycles_frac(num: float, den: float) -> float:
    """frac(num / den) of two doubles, computed exactly in rationals."""
    c = Fraction(num) / Fraction(den)
    return float(c - math.floor(c))


# --------------------------------------------------------------------------
# DFT / FFT
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 3, 8, 13])
def test_dft_closed_forms(n):
    for n0 in range(n):
        x = np.zeros(n, complex)
        x[n0] = 1.0
        k = np.arange(n)
        assert np.abs(oracle.dft(x) - np.exp(-2j * np.pi * n0 * k / n)).max() < 1e-14
        tone = np.exp(2j * np.pi * n0 * k / n)
        expect = np.zeros(n, complex)
        expect[n0] = n
        assert np.abs(oracle.dft(tone) - expect).max() < 1e-12


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_matches_naive_dft(n, sign):
    x = crandn(np.random.default_rng(n), n)
    assert np.abs(oracle.fft(x, sign) - oracle.dft(x, sign)).max() < 1e-13 * max(1, n)


def test_fft_matches_numpy():
    rng = np.random.default_rng(7)
    x = crandn(rng, 1024)
    assert rel(oracle.fft(x), np.fft.fft(x)) < 1e-14
    assert rel(oracle.fft(x, +1), np.fft.ifft(x) * 1024) < 1e-14
    a = crandn(rng, 32, 16)
    assert rel(oracle.fft2(a), np.fft.fft2(a)) < 1e-14


def test_fft_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft(np.ones(12))


# --------------------------------------------------------------------------
# Transfer function and frequency convention
# --------------------------------------------------------------------------

def plane_wave(n, mx, my):
    k = np.arange(n)
    return np.exp(2j * np.pi * (my * k[:, None] + mx * k[None, :]) / n)


@pytest.mark.parametrize("method", [oracle.ASM, oracle.FRESNEL])
@pytest.mark.parametrize("mx,my", [(0, 0), (3, 0), (-5, 2), (7, -11), (-16, 4)])
def test_plane_wave_eigenfunction(method, mx, my):
    n, d, lam, z = 32, 1.0e-6, 0.7e-6, 1.0e-4
    u = plane_wave(n, mx, my)
    out = oracle.propagate(u, d, d, lam, z, method, pad=1)
    # direction cosines of the plane wave: alpha = lambda fx, beta = lambda fy
    alpha, beta = lam * mx / (n * d), lam * my / (n * d)
    k = 2 * np.pi / lam
    if method == oracle.ASM:
        gamma = math.cos(math.asin(math.hypot(alpha, beta)))  # propagation angle
        phase = k * z * gamma
    else:
        phase = k * z * (1.0 - 0.5 * (alpha * alpha + beta * beta))
    assert np.abs(out - np.exp(1j * phase) * u).max() < 1e-12


@pytest.mark.parametrize("method", [oracle.ASM, oracle.FRESNEL])
@pytest.mark.parametrize("n,mx,my", [(48, 7, -11), (48, -24, 5), (45, 22, -22), (45, -3, 17), (20, 10, -9)])
def test_plane_wave_eigenfunction_any_length(method, n, mx, my):
    """The eigenfunction pin on grids whose extent is not a power of two
    (the naive DFT path), odd lengths included: bin (n-1)/2 of an odd grid
    is the positive frequency, as in numpy's fftfreq."""
    d, lam, z = 1.0e-6, 0.7e-6, 1.0e-4
    u = plane_wave(n, mx, my)
    out = oracle.propagate(u, d, d, lam, z, method, padded=(n, n))
    alpha, beta = lam * mx / (n * d), lam * my / (n * d)
    k = 2 * np.pi / lam
    if method == oracle.ASM:
        phase = k * z * math.cos(math.asin(math.hypot(alpha, beta)))
    else:
        phase = k * z * (1.0 - 0.5 * (alpha * alpha + beta * beta))
    assert np.abs(out - np.exp(1j * phase) * u).max() < 1e-11
    assert np.allclose(oracle.fftfreq(n, d) * n * d, np.fft.fftfreq(n) * n)


def test_any_length_padding_invariants():
    """Non-power-of-two padded grids (1000-like 2x padding of a 25 x 15
    field: 50 x 30, and an odd 49 x 31): the window position does not
    matter, the adjoint identity holds, and DI equals the brute-force sum on
    the smallest admissible odd padding (2n - 1)."""
    rng = np.random.default_rng(760)
    u = crandn(rng, 25, 15)
    v = crandn(rng, 25, 15)
    args = (4e-6, 3e-6, 0.6e-6, 2e-3)
    for py, px in ((50, 30), (49, 31)):
        a = oracle.propagate(u, *args, oracle.ASM, padded=(py, px))
        for oy, ox in ((0, 0), (py - 25, px - 15), (7, 3)):
            b = oracle.propagate_offset(u, *args, oracle.ASM, 0, oy, ox, padded=(py, px))
            assert rel(b, a) < 1e-13, (py, px, oy, ox)
        lhs = np.vdot(v, a)
        rhs = np.vdot(oracle.propagate(v, *args, oracle.ASM, padded=(py, px), adjoint=True), u)
        assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(a) * np.linalg.norm(v)
    ny, nx = 6, 5
    uu = crandn(rng, ny, nx)
    dy, dx, lam, z = 1.5e-6, 2e-6, 0.6e-6, 2.5e-5
    di = oracle.propagate(uu, dy, dx, lam, z, oracle.DI, padded=(2 * ny - 1, 2 * nx - 1))
    assert rel(di, oracle.rs_direct(uu, dy, dx, lam, z)) < 1e-12


def test_evanescent_plane_wave_is_removed():
    n, d, lam = 32, 0.4e-6, 0.7e-6
    u = plane_wave(n, 14, 14)  # fx^2 + fy^2 > 1/lambda^2
    out = oracle.propagate(u, d, d, lam, 1e-5, oracle.ASM, pad=1)
    assert np.abs(out).max() < 1e-14
    # the same wave under the Fresnel transfer function is not removed
    out_f = oracle.propagate(u, d, d, lam, 1e-5, oracle.FRESNEL, pad=1)
    assert abs(np.abs(out_f).max() - 1.0) < 1e-12


# --------------------------------------------------------------------------
# Pad / crop / DFT chain against brute-force circular convolution
# --------------------------------------------------------------------------

def naive_dft2(a, sign):
    ny, nx = a.shape
    rows = np.stack([oracle.dft(a[r], sign) for r in range(ny)])
    return np.stack([oracle.dft(rows[:, c], sign) for c in range(nx)], axis=1)


@pytest.mark.parametrize("method", [oracle.ASM, oracle.FRESNEL])
def test_propagation_is_circular_convolution(method):
    n, pad, d, lam, z = 16, 2, 2e-6, 0.6e-6, 3e-4
    P = n * pad
    u = crandn(np.random.default_rng(3), n, n)
    H = oracle.transfer(P, P, d, d, lam, z, method)
    h = naive_dft2(H, +1) / (P * P)            # impulse response of the padded grid
    upad = np.zeros((P, P), complex)
    o = (P - n) // 2
    upad[o:o + n, o:o + n] = u
    out_full = np.zeros((P, P), complex)
    idx = np.arange(P)
    for my in range(P):
        for mx in range(P):
            out_full[my, mx] = np.sum(h[(my - idx)[:, None] % P, (mx - idx)[None, :] % P] * upad)
    expect = out_full[o:o + n, o:o + n]
    got = oracle.propagate(u, d, d, lam, z, method, pad)
    assert rel(got, expect) < 1e-12


# --------------------------------------------------------------------------
# Identities
# --------------------------------------------------------------------------

@pytest.mark.parametrize("method", [oracle.ASM, oracle.FRESNEL])
def test_zero_distance_is_identity(method):
    u = crandn(np.random.default_rng(4), 24, 40)
    out = oracle.propagate(u[:16, :32], 3e-6, 5e-6, 0.8e-6, 0.0, method, pad=2)
    assert np.abs(out - u[:16, :32]).max() < 1e-14


@pytest.mark.parametrize("method", [oracle.ASM, oracle.FRESNEL])
def test_adjoint_identity(method):
    rng = np.random.default_rng(5)
    u, v = crandn(rng, 32, 32), crandn(rng, 32, 32)
    args = (8e-6, 8e-6, 0.7e-6, 0.1, method, 2)
    Pu = oracle.propagate(u, *args)
    PHv = oracle.propagate(v, *args, adjoint=True)
    lhs, rhs = np.vdot(v, Pu), np.vdot(PHv, u)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    # conj(H(z)) = H(-z): the adjoint is propagation over -z
    dy, dx, lam, z, m, p = args
    assert rel(PHv, oracle.propagate(v, dy, dx, lam, -z, m, p)) < 1e-12


def test_adjoint_is_conjugate_transpose_matrix():
    n = 4
    args = (1e-6, 1e-6, 0.5e-6, 2e-5, oracle.ASM, 2)
    eye = np.eye(n * n).reshape(n * n, n, n)
    P = oracle.propagate(eye, *args).reshape(n * n, n * n).T
    PH = oracle.propagate(eye, *args, adjoint=True).reshape(n * n, n * n).T
    assert np.abs(PH - P.conj().T).max() < 1e-14


def test_parseval_without_padding():
    u = crandn(np.random.default_rng(6), 64, 64)
    out = oracle.propagate(u, 8e-6, 8e-6, 0.7e-6, 0.2, oracle.ASM, pad=1)
    assert abs(np.linalg.norm(out) / np.linalg.norm(u) - 1.0) < 1e-13


def test_pad_placement_invariance():
    u = crandn(np.random.default_rng(8), 16, 16)
    args = (4e-6, 4e-6, 0.6e-6, 0.01, oracle.ASM, 2)
    ref = oracle.propagate(u, *args)
    for oy, ox in [(0, 0), (3, 5), (16, 16), (9, 0)]:
        got = oracle.propagate_offset(u, *args, oy, ox)
        assert rel(got, ref) < 1e-13


def test_group_law_without_padding():
    u = crandn(np.random.default_rng(9), 32, 32)
    args = (6e-6, 6e-6, 0.55e-6)
    a = oracle.propagate(oracle.propagate(u, *args, 0.03, oracle.ASM, 1), *args, 0.05, oracle.ASM, 1)
    b = oracle.propagate(u, *args, 0.08, oracle.ASM, 1)
    assert rel(a, b) < 1e-12


# --------------------------------------------------------------------------
# Physics closed forms
# --------------------------------------------------------------------------

def gaussian_lens_closed_form(w):
    """Paraxial Gaussian beam through z1, lens f, z2 with q-parameters
    (field ~ (q0/q) exp(i k r^2 / (2 q)) exp(i k z), q = z - i zR)."""
    lam = w.wavelength
    k = 2 * math.pi / lam
    zR = math.pi * w.w0 ** 2 / lam
    q0 = -1j * zR
    q1 = q0 + w.z1
    q2 = 1.0 / (1.0 / q1 - 1.0 / w.f)
    q3 = q2 + w.z2
    x = (np.arange(w.n) - w.n // 2) * w.d
    r2 = x[:, None] ** 2 + x[None, :] ** 2
    ph = Fraction(w.z1) / Fraction(lam) + Fraction(w.z2) / Fraction(lam)
    ph = float(ph - math.floor(ph))
    U = (q0 / q1) * (q2 / q3) * np.exp(1j * k * r2 / (2 * q3)) * np.exp(2j * np.pi * ph)
    w_out = math.sqrt(2.0 / (k * (1.0 / q3).imag))
    return U, w_out


def run_gaussian_lens(w, method):
    u = w.field()
    v = oracle.propagate(u, w.d, w.d, w.wavelength, w.z1, method, w.pad)
    v = oracle.modulate(v, oracle.lens(w.n, w.n, w.d, w.d, w.wavelength, w.f))
    return oracle.propagate(v, w.d, w.d, w.wavelength, w.z2, method, w.pad)


def test_gaussian_beam_fresnel_exact():
    w = workloads.GaussianLensWorkload()
    U, w_out = gaussian_lens_closed_form(w)
    assert abs(w_out - 111.408e-6) < 1e-9
    v = run_gaussian_lens(w, oracle.FRESNEL)
    assert rel(v, U) < 1e-12
    I = (w.w0 / w_out) ** 2 * np.exp(-2 * ((np.arange(w.n) - w.n // 2)[:, None] ** 2 +
                                           (np.arange(w.n) - w.n // 2)[None, :] ** 2) * w.d ** 2 / w_out ** 2)
    assert rel(np.abs(v) ** 2, I) < 1e-12


def test_gaussian_beam_asm_within_paraxial_error():
    w = workloads.GaussianLensWorkload()
    U, _ = gaussian_lens_closed_form(w)
    v = run_gaussian_lens(w, oracle.ASM)
    e = rel(np.abs(v) ** 2, np.abs(U) ** 2)
    assert 1e-8 < e < 1e-5  # non-paraxial correction, small but present


def ff_chain(u, n, d, lam, f):
    v = oracle.propagate(u, d, d, lam, f, oracle.FRESNEL, pad=1)
    v = oracle.modulate(v, oracle.lens(n, n, d, d, lam, f))
    return oracle.propagate(v, d, d, lam, f, oracle.FRESNEL, pad=1)


def test_lens_ff_is_discrete_fourier_transform():
    n, d, lam = 64, 10e-6, 700e-9
    f = n * d * d / lam
    u = crandn(np.random.default_rng(10), n, n)
    v = ff_chain(u, n, d, lam, f)
    centred_dft = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(u)))
    expect = (-1j / n) * np.exp(2j * np.pi * exact_cycles_frac(2 * f, lam)) * centred_dft
    assert rel(v, expect) < 1e-13


def test_square_aperture_dirichlet_pattern():
    n, d, lam, M = 64, 10e-6, 700e-9, 9
    f = n * d * d / lam
    u = np.zeros((n, n), complex)
    s = slice(n // 2 - M // 2, n // 2 + M // 2 + 1)
    u[s, s] = 1.0
    v = ff_chain(u, n, d, lam, f)
    m = np.arange(n) - n // 2
    with np.errstate(all="ignore"):
        D = np.where(m == 0, M, np.sin(np.pi * M * m / n) / np.sin(np.pi * m / n))
    expect = (-1j / n) * np.exp(2j * np.pi * exact_cycles_frac(2 * f, lam)) * D[:, None] * D[None, :]
    assert rel(v, expect) < 1e-13


def test_rayleigh_sommerfeld_brute_force_converges():
    lam, width, w0, z = 1.0e-6, 8e-6, 1.5e-6, 4e-6
    errs = []
    for n in (16, 32):
        d = width / n
        x = (np.arange(n) - n // 2) * d
        u = np.exp(-(x[:, None] ** 2 + x[None, :] ** 2) / w0 ** 2).astype(complex)
        a = oracle.propagate(u, d, d, lam, z, oracle.ASM, pad=8)
        r = oracle.rs_direct(u, d, d, lam, z)
        errs.append(rel(a, r))
    assert errs[0] < 3e-5
    assert errs[1] < errs[0] and errs[1] < 1e-5


# --------------------------------------------------------------------------
# Direct integration (DI) and the choice of method
# --------------------------------------------------------------------------

def _green(oy, ox, z, lam):
    d = np.sqrt(oy * oy + ox * ox + z * z)
    return np.exp(2j * np.pi * (d / lam)) / d


@pytest.mark.parametrize("geom", [(20e-6, 1.0e-6, 2e-6, 1.5e-6), (3e-4, 0.6e-6, 4e-6, 4e-6)])
def test_rs_impulse_response_is_green_derivative(geom):
    """A single-pixel input returns the sampled impulse response times dx dy;
    Eq. (impulse_response) equals -(1/2 pi) d/dz of exp(i k d)/d.  The
    derivative is taken by a fourth-order central difference in z (an
    independent evaluation: a dropped 1/(kd) term, a wrong sign of i or a
    missing z/d factor each change the result by more than the bound)."""
    z, lam, dy, dx = geom
    ny, nx = 6, 5
    u = np.zeros((ny, nx), complex)
    r0, c0 = 2, 1
    u[r0, c0] = 1.0
    out = oracle.rs_direct(u, dy, dx, lam, z)
    oy = (np.arange(ny)[:, None] - r0) * dy
    ox = (np.arange(nx)[None, :] - c0) * dx
    h = 1e-3 * lam
    deriv = (-_green(oy, ox, z + 2 * h, lam) + 8 * _green(oy, ox, z + h, lam)
             - 8 * _green(oy, ox, z - h, lam) + _green(oy, ox, z - 2 * h, lam)) / (12 * h)
    expect = -deriv / (2 * np.pi) * dx * dy
    assert rel(out, expect) < 1e-8
    # the 1/(kd) correction is well above the bound in the first geometry
    k = 2 * np.pi / lam
    d = np.sqrt(oy ** 2 + ox ** 2 + z ** 2)
    if geom[0] < 1e-4:
        assert float(np.max(1.0 / (k * d))) > 1e-3


@pytest.mark.parametrize("shape", [(8, 8, 16, 16), (5, 7, 16, 16), (6, 10, 16, 32), (3, 9, 8, 32), (1, 6, 8, 16)])
def test_di_equals_brute_force_sum(shape):
    """DI through the zero-padded DFT equals the direct Riemann sum of
    Eq. (field_propagation) on the same grid: the dense operator of the
    brute-force sum, built column by column, against the FFT form applied to
    random fields, forward and adjoint."""
    ny, nx, py, px = shape
    dy, dx, lam, z = 1.5e-6, 2.0e-6, 0.6e-6, 2.5e-5
    rng = np.random.default_rng(700 + ny * nx)
    n = ny * nx
    A = np.empty((n, n), complex)
    for p in range(n):
        e = np.zeros(n, complex)
        e[p] = 1.0
        A[:, p] = oracle.rs_direct(e.reshape(ny, nx), dy, dx, lam, z).ravel()
    u = crandn(rng, 3, ny, nx)
    fwd = oracle.propagate(u, dy, dx, lam, z, oracle.DI, padded=(py, px))
    adj = oracle.propagate(u, dy, dx, lam, z, oracle.DI, padded=(py, px), adjoint=True)
    ur = u.reshape(3, n)
    assert rel(fwd.reshape(3, n), ur @ A.T) < 1e-12
    assert rel(adj.reshape(3, n), ur @ A.conj()) < 1e-12


def test_di_invariant_under_extra_padding():
    """Beyond 2 n - 1 samples per axis, padding adds only offsets no pair of
    samples has: the result does not change, and the window's position in
    the padded grid does not matter."""
    rng = np.random.default_rng(711)
    u = crandn(rng, 12, 20)
    args = (3e-6, 2e-6, 0.5e-6, 4e-4, oracle.DI)
    a = oracle.propagate(u, *args, padded=(32, 64))
    b = oracle.propagate(u, *args, padded=(128, 64))
    c = oracle.propagate(u, *args, padded=(32, 256))
    assert rel(b, a) < 1e-13 and rel(c, a) < 1e-13
    H = oracle.di_transfer(12, 20, 32, 64, 3e-6, 2e-6, 0.5e-6, 4e-4)
    assert np.allclose(H, H[np.r_[0, 31:0:-1]][:, np.r_[0, 63:0:-1]], rtol=0, atol=1e-15 * np.abs(H).max())


def test_di_needs_linear_convolution_padding():
    u = np.ones((8, 8), complex)
    with pytest.raises(ValueError):
        oracle.propagate(u, 1e-6, 1e-6, 0.5e-6, 1e-4, oracle.DI, padded=(8, 16))
    with pytest.raises(ValueError):
        oracle.di_transfer(9, 8, 16, 16, 1e-6, 1e-6, 0.5e-6, 1e-4)
    assert oracle.di_transfer(8, 8, 16, 16, 1e-6, 1e-6, 0.5e-6, 1e-4).shape == (16, 16)


@pytest.mark.parametrize("n", [64, 250])
def test_critical_distance_is_the_fresnel_chirp_nyquist_limit(n):
    """Eq. (sampling_condition): at z = L dx / lambda the phase of the
    transfer function's chirp advances by pi (N-1)/N between the last two
    bins of the unpadded grid, i.e. it reaches the Nyquist rate; a shorter
    distance stays below it.  Evaluated from the oracle's Fresnel transfer
    function (power-of-two length) and from the closed-form chirp."""
    d, lam = 8e-6, 0.7e-6
    zc = oracle.critical_distance(n, n, d, d, lam)
    f = (np.arange(n) - n // 2) / (n * d)
    steps = np.abs(np.diff(-np.pi * lam * zc * f ** 2))
    assert abs(steps.max() - np.pi * (n - 1) / n) < 1e-9
    if n == 64:
        H = oracle.transfer(1, n, d, d, lam, zc, oracle.FRESNEL)[0]
        Hs = np.fft.fftshift(H)
        ang = np.abs(np.angle(Hs[1:] / Hs[:-1]))
        assert abs(ang.max() - np.pi * (n - 1) / n) < 1e-9
        H2 = oracle.transfer(1, n, d, d, lam, 0.9 * zc, oracle.FRESNEL)[0]
        Hs2 = np.fft.fftshift(H2)
        assert np.abs(np.angle(Hs2[1:] / Hs2[:-1])).max() < 0.9 * np.pi


def test_resolve_method():
    zc = oracle.critical_distance(128, 256, 4e-6, 2e-6, 0.5e-6)
    assert zc == pytest.approx(min(128 * 16e-12, 256 * 4e-12) / 0.5e-6, rel=1e-15)
    assert oracle.resolve_method(128, 256, 4e-6, 2e-6, 0.5e-6, 0.999 * zc) == oracle.ASM
    assert oracle.resolve_method(128, 256, 4e-6, 2e-6, 0.5e-6, zc) == oracle.DI
    assert oracle.resolve_method(128, 256, 4e-6, 2e-6, 0.5e-6, 10 * zc) == oracle.DI
    assert oracle.resolve_method(128, 256, 4e-6, 2e-6, 0.5e-6, 0.0) == oracle.ASM
    assert oracle.resolve_method(128, 256, 4e-6, 2e-6, 0.5e-6, -10 * zc) == oracle.ASM


# --------------------------------------------------------------------------
# Resampling onto another grid
# --------------------------------------------------------------------------

def test_bilinear_reproduces_bilinear_functions():
    """Bilinear interpolation is exact for f = a + b x + c y + d x y at every
    output sample inside the input grid's hull (a closed form independent of
    the interpolation code)."""
    gin = (12, 17, 3e-6, 2e-6, 1e-6, -2e-6)
    gout = (23, 19, 1.3e-6, 1.7e-6, 0.4e-6, 0.5e-6)
    yi = oracle.coords(12, 3e-6, 1e-6)[:, None]
    xi = oracle.coords(17, 2e-6, -2e-6)[None, :]
    f = lambda y, x: (0.3 - 0.2j) + 1e5 * x * (1 + 2j) - 2e5 * y + 3e10 * x * y * 1j
    out = oracle.resample(f(yi, xi), gin, gout, oracle.BILINEAR)
    Y = oracle.coords(23, 1.3e-6, 0.4e-6)[:, None]
    X = oracle.coords(19, 1.7e-6, 0.5e-6)[None, :]
    inside = (Y >= yi.min()) & (Y <= yi.max()) & (X >= xi.min()) & (X <= xi.max())
    assert inside.sum() > 100
    exp = f(Y, X) * np.ones_like(out)
    assert np.max(np.abs(out - exp)[inside]) < 1e-13 * np.max(np.abs(exp))
    assert np.all(out[~((Y >= yi.min() - 3e-6) & (Y <= yi.max() + 3e-6) & (X >= xi.min() - 2e-6) & (X <= xi.max() + 2e-6))] == 0)


def test_nearest_is_the_closest_sample():
    """Nearest neighbour against a brute-force search for the closest input
    sample of every output sample (distances not within 1e-9 of a tie);
    zero outside the input window."""
    gin = (9, 14, 5e-6, 4e-6, 2e-6, 1e-6)
    gout = (21, 25, 2.1e-6, 2.9e-6, -1.1e-6, 3.3e-6)
    rng = np.random.default_rng(751)
    u = crandn(rng, 2, 9, 14)
    out = oracle.resample(u, gin, gout, oracle.NEAREST)
    yi, xi = oracle.coords(9, 5e-6, 2e-6), oracle.coords(14, 4e-6, 1e-6)
    Y, X = oracle.coords(21, 2.1e-6, -1.1e-6), oracle.coords(25, 2.9e-6, 3.3e-6)
    for q in range(21):
        for r in range(25):
            ky = int(np.argmin(np.abs(yi - Y[q])))
            kx = int(np.argmin(np.abs(xi - X[r])))
            iny = abs(yi[ky] - Y[q]) < 0.5 * 5e-6
            inx = abs(xi[kx] - X[r]) < 0.5 * 4e-6
            exp = u[:, ky, kx] if (iny and inx) else 0
            assert np.all(out[:, q, r] == exp), (q, r)


def test_resample_identity_and_adjoint():
    rng = np.random.default_rng(752)
    gin = (7, 10, 2e-6, 3e-6, 0.0, 1e-6)
    u = crandn(rng, 3, 7, 10)
    for mode in (oracle.NEAREST, oracle.BILINEAR):
        assert np.array_equal(oracle.resample(u, gin, gin, mode), u)
    gout = (11, 6, 1.1e-6, 4.7e-6, 0.3e-6, -0.6e-6)
    for mode in (oracle.NEAREST, oracle.BILINEAR):
        A = np.empty((66, 70), complex)
        for p in range(70):
            e = np.zeros(70, complex)
            e[p] = 1.0
            A[:, p] = oracle.resample(e.reshape(7, 10), gin, gout, mode).ravel()
        g = crandn(rng, 3, 11, 6)
        adj = oracle.resample_adjoint(g, gin, gout, mode)
        assert rel(adj.reshape(3, 70), g.reshape(3, 66) @ A.conj()) < 1e-14


# --------------------------------------------------------------------------
# Polarization
# --------------------------------------------------------------------------

def test_polarizer_listing_powers():
    with open(os.path.join(GOLDEN, "polarizer_powers.json")) as fh:
        gold = json.load(fh)
    n, d = 32, 10e-6
    E = np.zeros((3, n, n), complex)
    E[0] = 1.0
    E /= math.sqrt(oracle.power(E, d, d))
    for case in gold["cases"]:
        F = E
        for deg in case["elements_applied_in_order_deg"]:
            F = oracle.jones_apply(F, oracle.embed_jones(oracle.linear_polarizer(math.radians(deg))))
        assert abs(oracle.power(F, d, d) - case["power"]) < 1e-14


def test_malus_law_and_waveplate():
    E = np.zeros((3, 4, 4), complex)
    E[0] = 1.0
    for th in np.linspace(0, math.pi, 7):
        F = oracle.jones_apply(E, oracle.embed_jones(oracle.linear_polarizer(th)))
        assert abs(np.sum(np.abs(F) ** 2) / 16 - math.cos(th) ** 2) < 1e-14
    # quarter-wave plate at 45 deg turns x into circular light: any linear
    # polarizer then passes half the power
    qwp = oracle.embed_jones(oracle.waveplate(math.pi / 4, math.pi / 2))
    for th in (0.0, math.pi / 6, 1.0):
        F = oracle.jones_apply(oracle.jones_apply(E, qwp),
                               oracle.embed_jones(oracle.linear_polarizer(th)))
        assert abs(np.sum(np.abs(F) ** 2) / 16 - 0.5) < 1e-14
    W = oracle.waveplate(0.3, 1.1)
    assert np.abs(W @ W.conj().T - np.eye(2)).max() < 1e-15


def test_jones_apply_is_matrix_vector_product():
    rng = np.random.default_rng(11)
    J = crandn(rng, 3, 3)
    E = crandn(rng, 2, 3, 3, 5)
    got = oracle.jones_apply(E, J)
    gotH = oracle.jones_apply(E, J, conj_transpose=True)
    for b in range(2):
        for y in range(3):
            for x in range(5):
                v = E[b, :, y, x]
                assert np.abs(got[b, :, y, x] - J.dot(v)).max() < 1e-14
                assert np.abs(gotH[b, :, y, x] - J.conj().T.dot(v)).max() < 1e-14
    Jp = crandn(rng, 3, 3, 3, 5)
    got = oracle.jones_apply(E, Jp)
    assert np.abs(got[1, :, 2, 4] - Jp[:, :, 2, 4].dot(E[1, :, 2, 4])).max() < 1e-14


# --------------------------------------------------------------------------
# Coherence
# --------------------------------------------------------------------------

COH = (10e-6, 10e-6, 633e-9, 0.02, oracle.ASM, 2)


def test_coherence_rank_one_reduces_to_field():
    n = 8
    u = crandn(np.random.default_rng(12), n, n)
    G = np.einsum("ab,cd->abcd", u, np.conj(u))
    Pu = oracle.propagate(u, *COH)
    expect = np.einsum("ab,cd->abcd", Pu, np.conj(Pu))
    assert rel(oracle.coherence_propagate(G, *COH), expect) < 1e-13
    assert rel(oracle.coherence_intensity(oracle.coherence_propagate(G, *COH)), np.abs(Pu) ** 2) < 1e-13


def test_coherence_sum_of_modes_and_hermiticity():
    n, modes = 8, 3
    rng = np.random.default_rng(13)
    us = [crandn(rng, n, n) for _ in range(modes)]
    G = sum(np.einsum("ab,cd->abcd", u, np.conj(u)) for u in us)
    out = oracle.coherence_propagate(G, *COH)
    expect = sum(np.einsum("ab,cd->abcd", p, np.conj(p)) for p in (oracle.propagate(u, *COH) for u in us))
    assert rel(out, expect) < 1e-13
    M = out.reshape(n * n, n * n)
    assert np.abs(M - M.conj().T).max() < 1e-13 * np.abs(M).max()


def test_coherence_trace_and_adjoint():
    n = 8
    rng = np.random.default_rng(14)
    A = crandn(rng, n * n, n * n)
    G = (A @ A.conj().T).reshape(n, n, n, n)
    out = oracle.coherence_propagate(G, 10e-6, 10e-6, 633e-9, 0.02, oracle.ASM, 1)
    tr = lambda X: np.trace(X.reshape(n * n, n * n))
    assert abs(tr(out) - tr(G)) / abs(tr(G)) < 1e-13
    X, Y = crandn(rng, n, n, n, n), crandn(rng, n, n, n, n)
    lhs = np.vdot(Y, oracle.coherence_propagate(X, *COH))
    rhs = np.vdot(oracle.coherence_propagate(Y, *COH, adjoint=True), X)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_coherence_modulation_matches_modes():
    n = 8
    rng = np.random.default_rng(15)
    u = crandn(rng, n, n)
    m = np.exp(1j * rng.random((n, n)) * 6)
    G = np.einsum("ab,cd->abcd", u, np.conj(u))
    mu = m * u
    assert rel(oracle.coherence_modulate(G, m), np.einsum("ab,cd->abcd", mu, np.conj(mu))) < 1e-14


# --------------------------------------------------------------------------
# Gradients against central finite differences
# --------------------------------------------------------------------------

STACK = dict(dy=6e-6, dx=6e-6, wavelength=0.7e-6, z=0.004, method=oracle.ASM, pad=2)


def stack_loss(u0, phis, target):
    us = oracle.stack_forward(u0, phis, **STACK)
    return oracle.mse_intensity(us[-1], target)[0]


def test_stack_gradient_finite_differences():
    rng = np.random.default_rng(16)
    B, n, L = 2, 16, 3
    u0 = crandn(rng, B, n, n) * 0.5
    phis = [rng.random((n, n)) * 2 * np.pi for _ in range(L)]
    target = rng.random((n, n))
    us = oracle.stack_forward(u0, phis, **STACK)
    loss, g = oracle.mse_intensity(us[-1], target)
    g0, grads = oracle.stack_backward(us, phis, g, **STACK)
    h = 1e-5
    # directional derivatives along random directions in mask space
    for _ in range(4):
        dirs = [rng.standard_normal((n, n)) for _ in range(L)]
        lp = stack_loss(u0, [p + h * q for p, q in zip(phis, dirs)], target)
        lm = stack_loss(u0, [p - h * q for p, q in zip(phis, dirs)], target)
        fd = (lp - lm) / (2 * h)
        an = sum(float(np.sum(gr * q)) for gr, q in zip(grads, dirs))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    # single pixels
    for (l, y, x) in [(0, 3, 4), (1, 8, 8), (2, 15, 0)]:
        pp = [p.copy() for p in phis]
        pm = [p.copy() for p in phis]
        pp[l][y, x] += h
        pm[l][y, x] -= h
        fd = (stack_loss(u0, pp, target) - stack_loss(u0, pm, target)) / (2 * h)
        assert abs(fd - grads[l][y, x]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10
    # gradient with respect to the input field (complex convention)
    du = crandn(rng, B, n, n)
    fd = (stack_loss(u0 + h * du, phis, target) - stack_loss(u0 - h * du, phis, target)) / (2 * h)
    an = float(np.real(np.vdot(g0, du)))
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_lens_gradient_finite_differences():
    rng = np.random.default_rng(17)
    n, d, lam, f, z = 32, 5e-6, 0.6e-6, 0.05, 0.05
    E = crandn(rng, 2, n, n)
    W = rng.random((n, n))

    def loss_of(fv):
        um = oracle.modulate(E, oracle.lens(n, n, d, d, lam, fv))
        out = oracle.propagate(um, d, d, lam, z, oracle.FRESNEL, 2)
        return oracle.weighted_intensity(out, W, d, d)

    L0, g = loss_of(f)
    um = oracle.modulate(E, oracle.lens(n, n, d, d, lam, f))
    g_mod = oracle.propagate(g, d, d, lam, z, oracle.FRESNEL, 2, adjoint=True)
    an = oracle.grad_lens_f(g_mod, um, n, n, d, d, lam, f)
    h = 1e-6 * f
    fd = (loss_of(f + h)[0] - loss_of(f - h)[0]) / (2 * h)
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_coherence_mask_gradient_finite_differences():
    rng = np.random.default_rng(18)
    n = 8
    A = crandn(rng, n * n, n * n)
    G0 = (A @ A.conj().T).reshape(n, n, n, n) / (n * n)
    phi = rng.random((n, n)) * 2 * np.pi
    T = rng.random((n, n))
    args = (10e-6, 10e-6, 633e-9, 0.01, oracle.ASM, 2)

    def loss_of(p):
        Gm = oracle.coherence_modulate(G0, np.exp(1j * p))
        I = oracle.coherence_intensity(oracle.coherence_propagate(Gm, *args))
        return float(np.mean((I - T) ** 2)), Gm, I

    L0, Gm, I = loss_of(phi)
    Gout = np.zeros((n * n, n * n), complex)
    np.fill_diagonal(Gout, (2.0 / (n * n)) * (I - T).ravel())
    Gmod = oracle.coherence_propagate(Gout.reshape(n, n, n, n), *args, adjoint=True)
    grad = oracle.coherence_grad_phase(Gmod, Gm)
    h = 1e-6
    for (y, x) in [(0, 0), (2, 3), (5, 7)]:
        pp, pm = phi.copy(), phi.copy()
        pp[y, x] += h
        pm[y, x] -= h
        fd = (loss_of(pp)[0] - loss_of(pm)[0]) / (2 * h)
        assert abs(fd - grad[y, x]) <= 1e-6 * max(abs(fd), 1e-6)


def test_intensity_malus_law_components():
    """Intensity of a 3-component field is the sum over components: an
    x-polarized unit field behind a linear polarizer at theta carries
    cos^2(theta) (Malus's law, closed form)."""
    E = np.zeros((3, 4, 4), complex)
    E[0] = 1.0
    for th in (0.0, 0.3, np.pi / 4, 1.2, np.pi / 2):
        J = oracle.embed_jones(oracle.linear_polarizer(th))
        I = oracle.intensity(oracle.jones_apply(E, J), ncomp=3)
        assert np.allclose(I, np.cos(th) ** 2, atol=1e-15)
    rng = np.random.default_rng(61)
    u = rng.standard_normal((2, 5, 6)) + 1j * rng.standard_normal((2, 5, 6))
    assert np.allclose(oracle.intensity(u), u.real ** 2 + u.imag ** 2, rtol=1e-14, atol=0)


def test_incoherent_sum_has_no_cross_terms():
    """Eq. (I_poly): mutually incoherent wavelengths add in intensity.  The
    coherent superposition differs from it by exactly the interference term
    2 Re(u1 conj(u2)); the weights scale linearly."""
    rng = np.random.default_rng(62)
    u1 = rng.standard_normal((6, 7)) + 1j * rng.standard_normal((6, 7))
    u2 = rng.standard_normal((6, 7)) + 1j * rng.standard_normal((6, 7))
    inc = oracle.incoherent_sum([u1, u2], [1.0, 1.0])
    coh = np.abs(u1 + u2) ** 2
    assert np.allclose(coh - inc, 2 * np.real(u1 * np.conj(u2)), atol=1e-12)
    w = oracle.incoherent_sum([u1, u2], [0.25, 2.0])
    assert np.allclose(w, 0.25 * np.abs(u1) ** 2 + 2.0 * np.abs(u2) ** 2, atol=1e-12)


def test_incoherent_sum_equals_coherence_diagonal():
    """A partially coherent field given as incoherent modes, Gamma = sum_k
    w_k u_k u_k^H, has the time-averaged intensity Re Gamma(r, r) =
    sum_k w_k |u_k|^2 (section "Spatial coherence")."""
    rng = np.random.default_rng(63)
    n = 4
    modes = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for _ in range(3)]
    w = [0.5, 1.5, 0.25]
    G = sum(wk * np.einsum("ab,cd->abcd", u, np.conj(u)) for wk, u in zip(w, modes))
    assert np.allclose(oracle.coherence_intensity(G), oracle.incoherent_sum(modes, w), atol=1e-12)


# --------------------------------------------------------------------------
# Overlap integral of Eq. (loss_func) and the sign of a phase modulator
# --------------------------------------------------------------------------

def test_inner_gaussian_overlap_closed_form():
    """Eq. (loss_func)'s overlap integral of two Gaussians of amplitude
    exp(-r^2/w0^2), the second displaced by a and tilted by exp(i k0 x):

        int u conj(v) dA = (pi w0^2 / 2) exp(-|a|^2 / (2 w0^2))
                           exp(-k0^2 w0^2 / 8) exp(-i k0 a_x / 2)

    (complete the square: r^2 + |r - a|^2 = 2 |r - a/2|^2 + |a|^2 / 2).  The
    Riemann sum of a well-sampled Gaussian equals its integral far below
    rounding, so this fixes the conjugated operand (the sign of the
    imaginary part), the area element and the normalisation."""
    n, d, w0 = 160, 10e-6, 150e-6
    ax, ay, k0 = 30e-6, -20e-6, 2 * math.pi / 400e-6
    x = oracle.coords(n, d)[None, :]
    y = oracle.coords(n, d)[:, None]
    u = np.exp(-(x ** 2 + y ** 2) / w0 ** 2)
    v = np.exp(-((x - ax) ** 2 + (y - ay) ** 2) / w0 ** 2) * np.exp(1j * k0 * x)
    expect = (math.pi * w0 ** 2 / 2) * math.exp(-(ax ** 2 + ay ** 2) / (2 * w0 ** 2)) \
        * math.exp(-k0 ** 2 * w0 ** 2 / 8) * np.exp(-1j * k0 * ax / 2)
    got = oracle.inner(u, v, d, d)
    assert abs(got - expect) < 1e-12 * abs(expect)
    assert got.imag < 0  # k0 ax > 0
    # Hermitian symmetry, and the self-overlap is the power
    assert abs(oracle.inner(v, u, d, d) - np.conj(got)) < 1e-15 * abs(got)
    assert abs(oracle.inner(u, u, d, d) - oracle.power(u, d, d)) < 1e-15 * oracle.power(u, d, d)
    assert abs(oracle.power(u, d, d) - math.pi * w0 ** 2 / 2) < 1e-12 * math.pi * w0 ** 2
    # Eq. (loss_func) for normalised fields: 1 - |<u, v>|^2 / (|u|^2 |v|^2)
    loss = 1 - abs(got) ** 2 / (oracle.power(u, d, d) * oracle.power(v, d, d))
    assert abs(loss - (1 - math.exp(-(ax ** 2 + ay ** 2) / w0 ** 2) * math.exp(-k0 ** 2 * w0 ** 2 / 4))) < 1e-12


def test_phase_mask_equals_pinned_lens():
    """A phase modulator with the thin-lens phase -pi r^2 / (lambda f) is the
    thin lens, whose sign the Gaussian-beam closed form pins (f > 0
    converges to the q-parameter waist).  exp(-i phi) would give the
    diverging lens."""
    ny, nx, d, lam, f = 48, 40, 7e-6, 0.6e-6, 0.03
    phi = 2 * math.pi * oracle.lens_phase_cycles(ny, nx, d, d, lam, f)
    assert rel(oracle.phase_mask(phi), oracle.lens(ny, nx, d, d, lam, f)) < 1e-12


def test_phase_ramp_steers_towards_positive_x():
    """A phase ramp phi = 2 pi g x tilts the beam toward +x under the
    exp(+i k z) convention of Eq. (transfer_function): after Fresnel
    propagation over z the field is, exactly on the padded grid,

        P[e^{2 pi i g x} u](x) = e^{2 pi i g x} e^{-i pi lambda z g^2} (P u)(x - lambda z g)

    for g a frequency of the padded grid and lambda z g a whole number s of
    samples (the spectrum of the beam vanishes at the wrap).  A modulator
    applying exp(-i phi) would move the beam to -s.  Tolerance: z / lambda
    is 1e5 cycles here, so the two propagations' FP64 phase rounding
    reaches ~1e-11 relative (the wrong sign is an O(1) error)."""
    n, d, lam, w0 = 256, 5e-6, 0.5e-6, 100e-6
    k0, s = 10, 20
    g = k0 / (2 * n * d)
    z = s * d / (lam * g)
    x = oracle.coords(n, d)[None, :]
    y = oracle.coords(n, d)[:, None]
    u = np.exp(-(x ** 2 + y ** 2) / w0 ** 2) * np.ones((n, n))
    ramp = 2 * math.pi * g * x * np.ones((n, 1))
    tilted = oracle.propagate(oracle.modulate(u, oracle.phase_mask(ramp)), d, d, lam, z, oracle.FRESNEL, pad=2)
    plain = oracle.propagate(u, d, d, lam, z, oracle.FRESNEL, pad=2)
    shifted = np.zeros_like(plain)
    shifted[:, s:] = plain[:, :-s]
    expect = np.exp(2j * math.pi * g * x) * np.exp(-1j * math.pi * lam * z * g * g) * shifted
    assert rel(tilted, expect) < 1e-10
    # the intensity centroid sits at +lambda z g
    I = np.abs(tilted) ** 2
    cx_ = float(np.sum(I * x) / np.sum(I))
    assert abs(cx_ - lam * z * g) < 1e-6 * d
