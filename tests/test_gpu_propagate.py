"""GPU parity of the propagation library against the FP64 oracle.

Every case runs the HIP path through the C-ABI (the Python binding only
marshals arguments) and compares with the oracle on the same seeded inputs,
element by element:
  complex64 fields: relative L2 error <= 2e-5,
  complex128 fields: relative L2 error <= 1e-12.
Sizes span several column tiles and transform passes; ragged grids (the
field smaller than half the padded extent) exercise the masked loads.
"""
import math

import numpy as np
import pytest

import oracle
from tests._util import announce, crandn, rel, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {np.complex64: 2e-5, np.complex128: 1e-12}


def _tp():
    import paper_2411_18591_amd as tp
    return tp


def run_case(ny, nx, py, px, method, dtype, *, batch=2, seed=0, z=0.05, d=(6e-6, 8e-6), lam=0.6e-6,
             phase=False, lens=None, cmask=False):
    tp = _tp()
    announce(f"propagate {ny}x{nx} pad {py}x{px} method={method} dtype={dtype.__name__} b={batch}")
    rng = np.random.default_rng(seed)
    u = crandn(rng, batch, ny, nx, dtype=dtype)
    rdt = np.float32 if dtype == np.complex64 else np.float64
    el_np = {}
    el_gpu = {}
    M = np.ones((ny, nx), complex)
    if phase:
        phi = (rng.random((ny, nx)) * 2 * np.pi).astype(rdt)
        el_gpu["phase"] = to_gpu(phi, torch)
        M = M * oracle.phase_mask(phi)
    if cmask:
        cm = crandn(rng, ny, nx, dtype=dtype)
        el_gpu["cmask"] = to_gpu(cm, torch)
        M = M * cm
    if lens is not None:
        el_gpu["lens_f"] = lens
        M = M * oracle.lens(ny, nx, d[0], d[1], lam, lens)
    meth = oracle.ASM if method == "asm" else oracle.FRESNEL
    expect = oracle.propagate(oracle.modulate(u, M), d[0], d[1], lam, z, meth, padded=(py, px))
    opt = tp.Optics(dy=d[0], dx=d[1], wavelength=lam, z=z, method=method, padded=(py, px))
    ug = to_gpu(u, torch)
    out = tp.propagate(ug, opt, **el_gpu)
    torch.cuda.synchronize()
    return rel(to_np(out), expect)


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("shape", [
    (4, 4, 8, 8), (8, 8, 16, 16), (16, 32, 32, 64), (32, 16, 64, 32), (64, 64, 128, 128),
    (128, 64, 256, 128), (256, 256, 512, 512), (100, 60, 256, 128), (5, 300, 16, 1024),
    (24, 24, 32, 32), (32, 32, 32, 32),
])
def test_asm_parity(shape, dtype):
    ny, nx, py, px = shape
    e = run_case(ny, nx, py, px, "asm", dtype)
    assert e <= TOL[dtype], e


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("L", [1024, 2048, 4096, 8192])
def test_large_transform_lengths(L, dtype):
    # one field row/column long enough for every transform length
    e = run_case(8, L // 2, 16, L, "asm", dtype, batch=1, z=0.02)
    assert e <= TOL[dtype], e
    e = run_case(L // 2, 8, L, 16, "asm", dtype, batch=1, z=0.02)
    assert e <= TOL[dtype], e


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_fresnel_parity(dtype):
    e = run_case(64, 128, 128, 256, "fresnel", dtype, z=0.1)
    assert e <= TOL[dtype], e


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_elements_parity(dtype):
    e = run_case(64, 64, 128, 128, "asm", dtype, phase=True)
    assert e <= TOL[dtype], e
    e = run_case(64, 64, 128, 128, "asm", dtype, lens=0.08)
    assert e <= TOL[dtype], e
    e = run_case(48, 40, 128, 128, "fresnel", dtype, phase=True, cmask=True, lens=-0.05)
    assert e <= TOL[dtype], e


def test_zero_distance_identity():
    e = run_case(64, 64, 128, 128, "asm", np.complex128, z=0.0)
    assert e <= 1e-14, e


def test_gaussian_beam_config_c128():
    """Gaussian waist 200 um through 5 cm, lens f = 10 cm, 10 cm (256^2,
    complex128, 2x padding) against the oracle, plus the closed-form waist."""
    import workloads
    tp = _tp()
    w = workloads.GaussianLensWorkload()
    announce("gaussian lens workload 256^2 c128")
    u = w.field()
    for method, m_or in (("asm", oracle.ASM), ("fresnel", oracle.FRESNEL)):
        o1 = tp.Optics(dy=w.d, dx=w.d, wavelength=w.wavelength, z=w.z1, method=method, pad=2)
        o2 = tp.Optics(dy=w.d, dx=w.d, wavelength=w.wavelength, z=w.z2, method=method, pad=2)
        ug = to_gpu(u, torch)
        v = tp.propagate(ug, o1)
        v = tp.propagate(v, o2, lens_f=w.f)
        torch.cuda.synchronize()
        r = oracle.propagate(u, w.d, w.d, w.wavelength, w.z1, m_or, 2)
        r = oracle.propagate(oracle.modulate(r, oracle.lens(w.n, w.n, w.d, w.d, w.wavelength, w.f)),
                             w.d, w.d, w.wavelength, w.z2, m_or, 2)
        assert rel(to_np(v), r) <= 1e-12
        I = np.abs(to_np(v)) ** 2
        x = (np.arange(w.n) - w.n // 2) * w.d
        r2 = x[:, None] ** 2 + x[None, :] ** 2
        w_out = math.sqrt(np.sum(I * r2) / np.sum(I) * 2)  # second moment: w^2 = 2 <r^2>
        assert abs(w_out - 111.408e-6) < (2e-9 if method == "fresnel" else 2e-8)


def test_in_place_and_multiple_jobs():
    tp = _tp()
    announce("in-place propagation")
    rng = np.random.default_rng(3)
    u = crandn(rng, 3, 32, 32, dtype=np.complex64)
    opt = tp.Optics(dy=5e-6, dx=5e-6, wavelength=0.5e-6, z=0.01, pad=2)
    ug = to_gpu(u, torch)
    tp.propagate(ug, opt, out=ug)
    torch.cuda.synchronize()
    expect = oracle.propagate(u, 5e-6, 5e-6, 0.5e-6, 0.01, oracle.ASM, 2)
    assert rel(to_np(ug), expect) <= 2e-5


def test_polarizer_listing_on_gpu():
    """The paper's polarizer listing: powers 1, 0.5, 0, 0.25."""
    import json
    import os
    tp = _tp()
    announce("polarizer listing (modulate, Jones)")
    with open(os.path.join(os.path.dirname(__file__), "golden", "polarizer_powers.json")) as fh:
        gold = json.load(fh)
    n, d = 32, 10e-6
    E = np.zeros((1, 3, n, n), np.complex128)
    E[0, 0] = 1.0 / math.sqrt(n * n * d * d)
    for case in gold["cases"]:
        F = to_gpu(E, torch)
        for deg in case["elements_applied_in_order_deg"]:
            J = tp.jones3(tp.linear_polarizer(math.radians(deg)))
            F = tp.modulate(F, dy=d, dx=d, wavelength=700e-9, ncomp=3, jones=J)
        torch.cuda.synchronize()
        p = float(np.sum(np.abs(to_np(F)) ** 2) * d * d)
        assert abs(p - case["power"]) < 1e-14


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_evanescent_cutoff(dtype):
    """Spacing below lambda / sqrt(2): the outer spectrum is evanescent and
    cut (H = 0); the library takes its per-bin FP64 transfer path.  Parity
    with the oracle, and a plane wave at an evanescent grid frequency is
    removed entirely."""
    # spacings chosen so that no bin lies within 5e-4 of the cutoff circle
    # (a bin on it in exact arithmetic is a floating-point tie: the FP64
    # kernel and the long-double oracle may round it to either side)
    e = run_case(48, 40, 128, 128, "asm", dtype, d=(0.37e-6, 0.43e-6), lam=0.8e-6, z=2e-6)
    assert e <= TOL[dtype], e
    tp = _tp()
    n, d, lam = 32, 0.4e-6, 0.8e-6
    k = 12  # grid frequency f = k / (n d) on both axes: lambda^2 (2 f^2) = 1.125 > 1
    y = np.arange(n)[:, None]
    x = np.arange(n)[None, :]
    u = np.exp(2j * np.pi * (k * x + k * y) / n).astype(dtype)[None]
    opt = tp.Optics(dy=d, dx=d, wavelength=lam, z=1e-6, pad=1, padded=(n, n))
    out = to_np(tp.propagate(to_gpu(u, torch), opt))
    torch.cuda.synchronize()
    fx = k / (n * d)
    assert lam * lam * 2 * fx * fx > 1.0  # the wave is evanescent
    assert np.abs(out).max() <= 1e-6 * np.abs(u).max()
