"""Padded grids whose extents are not powers of two (the paper's own
examples pad 1000, 250 and 50 samples to 2000, 500 and 100): the library
runs them through its unfused path, transforming each line with the
mixed-radix passes (lengths 2^a 3^b 5^c 7^d) or with Bluestein's chirp-z
method on its power-of-two FFTs (any other length).  Against the FP64 oracle
(whose transform of such lengths is the naive DFT, pinned on the CPU): even
and odd lengths, every radix (2, 3, 4, 5, 7, 8, 16), both line methods in
one job, a line of 2100 points (256 threads per line), the lengths with
compile-time kernels (50, 100, 250, 500, 1000, 2000), AS / Fresnel / DI (at
the smallest admissible DI padding, 2n - 1), forward and adjoint, elements,
the MSE epilogue and the mask gradient, mixed with power-of-two jobs in one
call; at the paper's 1000^2 -> 2000^2 scale (and 2002^2, a Bluestein
length), a separable Fresnel Gaussian against the oracle's 1-D
transforms."""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests._util import announce, crandn, rel, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {np.complex64: 2e-5, np.complex128: 1e-12}
METH = {"asm": oracle.ASM, "fresnel": oracle.FRESNEL, "di": oracle.DI}


def _tp():
    import paper_2411_18591_amd as tp
    return tp


def _oracle(u, opt, adjoint=False):
    ny, nx = u.shape[-2:]
    return oracle.propagate(u, opt.dy, opt.dx, opt.wavelength, opt.z, METH[opt.method], adjoint=adjoint,
                            padded=opt.padded_shape(ny, nx))


CASES = [
    # (ny, nx, py, px, method); line methods: M mixed-radix, B Bluestein
    (25, 15, 50, 30, "asm"),      # even, 2x padding (M 2*5*5, M 2*5*3)
    (24, 40, 49, 81, "fresnel"),  # odd extents (M 7*7, M 3^4)
    (50, 50, 100, 100, "asm"),    # the paper's 50^2 example, padded 2x (M 4*5*5)
    (30, 17, 59, 33, "di"),       # DI at 2n - 1 (odd; B 59, B 33)
    (20, 13, 40, 25, "di"),       # DI at 2n - 1 and 2n (M 8*5, M 5*5)
    (2, 3, 3, 5, "asm"),          # the smallest lengths (M 3, M 5)
    (20, 36, 20, 64, "fresnel"),  # one extent unpadded and not a power of two, the other a power of two
    (26, 20, 53, 40, "asm"),      # B 53 columns, M 8*5 rows
    (105, 9, 210, 18, "fresnel"), # every odd radix (M 2*5*3*7, M 2*3*3)
    (2, 1050, 3, 2100, "asm"),    # long mixed-radix rows, 256 threads per line (M 3, M 4*5*5*3*7)
    (250, 7, 500, 14, "asm"),     # compile-time length 500 in the column launch (the paper's 250^2 padded)
    (3, 500, 6, 1000, "fresnel"), # compile-time length 1000 in the row launches
    (125, 7, 250, 14, "asm"),     # compile-time length 250 (the paper's 250^2 grid without padding)
    (7, 25, 14, 50, "fresnel"),   # compile-time length 50 (the paper's 50^2 grid without padding)
]


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("case", CASES)
def test_forward_and_adjoint(case, dtype):
    tp = _tp()
    ny, nx, py, px, method = case
    announce(f"any-length {case} {dtype.__name__}")
    rng = np.random.default_rng(1200 + ny * nx)
    u = crandn(rng, 1 if px > 1000 else 3, ny, nx, dtype=dtype)
    z = 1.5 * oracle.critical_distance(ny, nx, 4e-6, 5e-6, 0.6e-6) if method == "di" else 3e-4
    opt = tp.Optics(dy=4e-6, dx=5e-6, wavelength=0.6e-6, z=z, method=method, padded=(py, px))
    ug = to_gpu(u, torch)
    out = tp.propagate(ug, opt)
    gin = tp.propagate_backward(ug, opt)
    torch.cuda.synchronize()
    assert rel(to_np(out), _oracle(u, opt)) <= TOL[dtype]
    assert rel(to_np(gin), _oracle(u, opt, adjoint=True)) <= TOL[dtype]


@pytest.mark.parametrize("shape", [(40, 30), (50, 50)])
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_elements_loss_and_mask_gradient(dtype, shape):
    """Phase mask + lens, the MSE epilogue (loss and dL/du), and the
    backward pass with the mask gradient, on a 2x padded field: 40 x 30
    (80 x 60, the run-time-length kernels) and 50 x 50 (100 x 100, the
    compile-time-length kernels, the elements applied in the row launch)."""
    tp = _tp()
    announce(f"any-length elements + loss {shape} {dtype.__name__}")
    rng = np.random.default_rng(1210)
    ny, nx = shape
    rdt = np.float32 if dtype == np.complex64 else np.float64
    u = crandn(rng, 2, ny, nx, dtype=dtype)
    phi = (rng.random((ny, nx)) * 6).astype(rdt)
    T = rng.random((ny, nx)).astype(rdt)
    opt = tp.Optics(dy=5e-6, dx=5e-6, wavelength=0.7e-6, z=2e-3, pad=2, round_pow2=False)
    assert opt.padded_shape(ny, nx) == (2 * ny, 2 * nx)
    ug, pg = to_gpu(u, torch), to_gpu(phi, torch)
    out, grad, loss = tp.propagate_loss(ug, opt, kind="mse", ref=to_gpu(T, torch), scale=0.5, phase=pg,
                                        lens_f=0.05)
    gphi = torch.zeros_like(pg)
    gin = tp.propagate_backward(grad, opt, saved_in=ug, grad_phase=gphi, phase=pg, lens_f=0.05)
    torch.cuda.synchronize()
    M = oracle.phase_mask(phi) * oracle.lens(ny, nx, 5e-6, 5e-6, 0.7e-6, 0.05)
    um = oracle.modulate(u, M)
    v = _oracle(um, opt)
    assert rel(to_np(out), v) <= TOL[dtype]
    Ie = np.abs(v) ** 2 - T
    assert abs(float(loss.item()) - 0.5 * float((Ie ** 2).sum())) <= 1e-4 * 0.5 * float((Ie ** 2).sum())
    g = 4 * 0.5 * Ie * v
    # the loss gradient 2 (|v|^2 - T) v is a derived quantity: the error of
    # v enters |v|^2 - T relative to that difference, not to |v|^2, so its
    # bar carries the factor 4 (measured and justified with the other
    # derived bars); the input gradient is one adjoint propagation of the
    # library's own loss gradient and takes the field bar
    assert rel(to_np(grad), g) <= 4 * TOL[dtype]
    gmod = _oracle(to_np(grad).astype(np.complex128), opt, adjoint=True)
    e_in = rel(to_np(gin), oracle.modulate(gmod, M, conj=True))
    announce(f"any-length loss chain: input-gradient error {e_in:.2e}")
    assert e_in <= TOL[dtype], e_in
    assert rel(to_np(gphi), oracle.grad_phase(gmod, um)) <= (1e-4 if dtype == np.complex64 else 1e-10)


def test_mixed_with_power_of_two_jobs():
    """Non-power-of-two jobs (the plain path, kept on one lane) and fused
    power-of-two jobs in one call: every output bitwise equal to its solo
    run."""
    tp = _tp()
    announce("any-length mixed call")
    rng = np.random.default_rng(1220)
    shapes = [(25, 15, False), (32, 32, True), (24, 40, False), (48, 16, True), (25, 15, False)]
    fields, opts = [], []
    for ny, nx, p2 in shapes:
        fields.append(to_gpu(crandn(rng, 2, ny, nx, dtype=np.complex64), torch))
        opts.append(tp.Optics(dy=4e-6, dx=4e-6, wavelength=0.6e-6, z=3e-4, pad=2, round_pow2=p2))
    outs = tp.propagate_jobs(fields, opts)
    solo = [tp.propagate(f, o) for f, o in zip(fields, opts)]
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(outs, solo)):
        assert torch.equal(a, b), i
    assert rel(to_np(outs[2]), _oracle(to_np(fields[2]), opts[2])) <= TOL[np.complex64]


def _prop1d(v, h, n):
    """1-D zero-padded propagation with the oracle's naive DFT (any length)."""
    x = np.zeros(h.size, dtype=np.complex128)
    x[: v.size] = v
    return oracle.dft(oracle.dft(x, -1) * h, +1)[:n] / h.size


@pytest.mark.parametrize("P", [2000, 2002])
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_paper_scale_separable(dtype, P):
    """1000^2 Gaussian through a lens, Fresnel, padded to P^2 (2000: the
    paper's 4f grid at 2x padding, mixed-radix lines; 2002 = 2*7*11*13:
    Bluestein lines): the field is separable, so every output pixel is
    H(0,0) a(y) a(x) with a the 1-D propagation computed with the oracle's
    naive DFT of length P and its Fresnel transfer function."""
    tp = _tp()
    n, d, lam, z, f, w0 = 1000, 10e-6, 700e-9, 0.05, 0.2, 1.5e-3
    announce(f"any-length 1000^2 -> {P}^2 {dtype.__name__}")
    g1 = workloads.gaussian_amplitude(n, 1, d, d, w0)[:, 0]
    l1 = oracle.lens(n, 1, d, d, lam, f)[:, 0]
    col = oracle.transfer(P, 1, d, d, lam, z, oracle.FRESNEL)[:, 0]
    a = _prop1d(g1 * l1, col / col[0], n)
    opt = tp.Optics(dy=d, dx=d, wavelength=lam, z=z, method="fresnel", padded=(P, P))
    u = workloads.gaussian_amplitude(n, n, d, d, w0).astype(dtype)[None]
    out = tp.propagate(to_gpu(u, torch), opt, lens_f=f)
    rows = np.array([0, 1, n // 3, n // 2, n - 1])
    got = to_np(out[0][torch.from_numpy(rows).cuda()])
    torch.cuda.synchronize()
    exp = col[0] * a[rows, None] * a[None, :]
    assert rel(got, exp) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_intensity_epilogue(dtype):
    """The intensity epilogue on a padded 30 x 25 -> 60 x 50 grid: a batch of
    two 3-component fields (no Jones element) through a lens, accumulated
    with weight 0.75 into an image that already holds values, the field not
    stored; then a scalar batch with the field stored too."""
    tp = _tp()
    announce(f"any-length intensity {dtype.__name__}")
    rng = np.random.default_rng(1230)
    ny, nx, d, lam, z = 30, 25, 4e-6, 500e-9, 0.004
    rdt = np.float32 if dtype == np.complex64 else np.float64
    E = crandn(rng, 2, 3, ny, nx, dtype=dtype)
    I0 = rng.random((2, ny, nx)).astype(rdt)
    opt = tp.Optics(dy=d, dx=d, wavelength=lam, z=z, padded=(60, 50))
    I = to_gpu(I0.copy(), torch)
    tp.propagate_intensity(to_gpu(E, torch), opt, intensity=I, ncomp=3, weight=0.75, lens_f=0.03)
    u = crandn(rng, 3, ny, nx, dtype=dtype)
    out = to_gpu(np.zeros_like(u), torch)
    Is = tp.propagate_intensity(to_gpu(u, torch), opt, out=out)
    torch.cuda.synchronize()
    m = oracle.modulate(E, oracle.lens(ny, nx, d, d, lam, 0.03))
    field = oracle.propagate(m, d, d, lam, z, oracle.ASM, padded=(60, 50))
    assert rel(to_np(I), I0 + 0.75 * oracle.intensity(field, ncomp=3)) <= TOL[dtype]
    fs = oracle.propagate(u, d, d, lam, z, oracle.ASM, padded=(60, 50))
    assert rel(to_np(out), fs) <= TOL[dtype]
    assert rel(to_np(Is), oracle.intensity(fs)) <= 2 * TOL[dtype]


@pytest.mark.parametrize("padded", [(120, 100), (127, 100)])
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_lens_gradient(dtype, padded):
    """dL/df of the lens focal length with a phase mask in front, on 60 x 50
    fields padded to 120 x 100 (mixed radix) and 127 x 100 (a Bluestein
    column length), Fresnel: against the oracle's grad_lens_f with the
    oracle's adjoint propagation, and grad_in against M^H P^H g."""
    tp = _tp()
    announce(f"any-length lens gradient {padded} {dtype.__name__}")
    rng = np.random.default_rng(1240)
    ny, nx, d, lam, f, z = 60, 50, 5e-6, 0.6e-6, 0.05, 0.02
    rdt = np.float32 if dtype == np.complex64 else np.float64
    u = crandn(rng, 2, ny, nx, dtype=dtype)
    g = crandn(rng, 2, ny, nx, dtype=dtype)
    phi = (rng.random((ny, nx)) * 6).astype(rdt)
    M = oracle.phase_mask(phi) * oracle.lens(ny, nx, d, d, lam, f)
    um = oracle.modulate(u, M)
    g_mod = oracle.propagate(g, d, d, lam, z, oracle.FRESNEL, adjoint=True, padded=padded)
    exp_f = oracle.grad_lens_f(g_mod, um, ny, nx, d, d, lam, f)
    opt = tp.Optics(dy=d, dx=d, wavelength=lam, z=z, method="fresnel", padded=padded)
    gf = torch.zeros((), dtype=torch.float64, device="cuda")
    pg = to_gpu(phi, torch)
    gphi = torch.zeros_like(pg)
    gin = tp.propagate_backward(to_gpu(g, torch), opt, saved_in=to_gpu(u, torch), grad_f=gf, grad_phase=gphi,
                                phase=pg, lens_f=f)
    torch.cuda.synchronize()
    assert rel(to_np(gin), oracle.modulate(g_mod, M, conj=True)) <= TOL[dtype]
    assert abs(float(gf.item()) - exp_f) <= (1e-4 if dtype == np.complex64 else 1e-11) * abs(exp_f)
    assert rel(to_np(gphi), oracle.grad_phase(g_mod, um)) <= (1e-4 if dtype == np.complex64 else 1e-10)


@pytest.mark.parametrize("padded", [(50, 60), (53, 60)])
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_jones_forward_backward(dtype, padded):
    """Polarized fields on 25 x 30 grids padded to 50 x 60 (mixed radix) and
    53 x 60 (Bluestein columns): a uniform Jones matrix (quarter-wave plate
    then a polarizer) with a phase mask and a lens, Fresnel, the
    weighted-intensity loss, gradients to the input, the mask and the focal
    length; then the same element with a per-pixel Jones map into the
    intensity epilogue."""
    tp = _tp()
    announce(f"any-length jones {padded} {dtype.__name__}")
    rng = np.random.default_rng(1250)
    ny, nx, d, lam, f, z = 25, 30, 6e-6, 0.55e-6, 0.04, 0.03
    rdt = np.float32 if dtype == np.complex64 else np.float64
    E = crandn(rng, 2, 3, ny, nx, dtype=dtype)
    Wt = rng.random((ny, nx)).astype(rdt)
    phi = (rng.random((ny, nx)) * 6).astype(rdt)
    Jo = oracle.embed_jones(oracle.linear_polarizer(math.pi / 6) @ oracle.waveplate(math.pi / 4, math.pi / 2))
    Jg = tp.jones3(tp.waveplate(math.pi / 4, math.pi / 2), tp.linear_polarizer(math.pi / 6))
    M = oracle.phase_mask(phi) * oracle.lens(ny, nx, d, d, lam, f)
    Em = oracle.modulate(oracle.jones_apply(E, Jo), M)
    out = oracle.propagate(Em, d, d, lam, z, oracle.FRESNEL, padded=padded)
    loss, gout = oracle.weighted_intensity(out, Wt, d, d)
    g_mod = oracle.propagate(gout, d, d, lam, z, oracle.FRESNEL, adjoint=True, padded=padded)
    exp_f = oracle.grad_lens_f(g_mod, Em, ny, nx, d, d, lam, f)
    exp_phi = oracle.grad_phase(g_mod, Em, reduce_axes=(0, 1))
    exp_gin = oracle.jones_apply(oracle.modulate(g_mod, M, conj=True), Jo, conj_transpose=True)

    opt = tp.Optics(dy=d, dx=d, wavelength=lam, z=z, method="fresnel", padded=padded)
    Eg, pg = to_gpu(E, torch), to_gpu(phi, torch)
    o, go, lo = tp.propagate_loss(Eg, opt, kind="weighted", ref=to_gpu(Wt, torch), scale=d * d,
                                  ncomp=3, jones=Jg, phase=pg, lens_f=f)
    gf = torch.zeros((), dtype=torch.float64, device="cuda")
    gphi = torch.zeros_like(pg)
    gin = tp.propagate_backward(go, opt, saved_in=Eg, grad_f=gf, grad_phase=gphi, ncomp=3, jones=Jg, phase=pg,
                                lens_f=f)
    torch.cuda.synchronize()
    assert rel(to_np(o), out) <= TOL[dtype]
    assert rel(to_np(go), gout) <= TOL[dtype]
    assert abs(float(lo.item()) - loss) <= (1e-4 if dtype == np.complex64 else 1e-11) * abs(loss)
    assert rel(to_np(gin), exp_gin) <= TOL[dtype]
    assert abs(float(gf.item()) - exp_f) <= (1e-4 if dtype == np.complex64 else 1e-11) * abs(exp_f)
    assert rel(to_np(gphi), exp_phi) <= (1e-4 if dtype == np.complex64 else 1e-10)

    Jmap = crandn(rng, 3, 3, ny, nx, dtype=dtype)
    I = tp.propagate_intensity(Eg, opt, ncomp=3, weight=0.5, jones_map=to_gpu(Jmap, torch))
    torch.cuda.synchronize()
    fm = oracle.propagate(oracle.jones_apply(E, Jmap), d, d, lam, z, oracle.FRESNEL, padded=padded)
    assert rel(to_np(I), 0.5 * oracle.intensity(fm, ncomp=3)) <= 2 * TOL[dtype]


@pytest.mark.parametrize("method", ["asm", "fresnel"])
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_transfer_formed_in_launch_equals_table(dtype, method):
    """Jobs of one or two fields form the AS / Fresnel transfer function in
    the column launch; larger jobs read a table built per call from the same
    function: the two agree to a few ulps (the compiler may contract the
    complex product with H differently when H is formed in place), forward
    and adjoint, at a compile-time length (50 x 50 -> 100 x 100) and a
    run-time one (25 x 15 -> 50 x 30), and both match the oracle."""
    tp = _tp()
    announce(f"any-length transfer in launch vs table {method} {dtype.__name__}")
    rng = np.random.default_rng(1260)
    for ny, nx in ((50, 50), (25, 15)):
        u = to_gpu(crandn(rng, 4, ny, nx, dtype=dtype), torch)
        opt = tp.Optics(dy=4e-6, dx=5e-6, wavelength=0.6e-6, z=3e-4, method=method, pad=2, round_pow2=False)
        big = tp.propagate(u, opt)
        adj = tp.propagate_backward(u, opt)
        ulps = 1e-6 if dtype == np.complex64 else 1e-14
        for k in range(4):
            one = tp.propagate(u[k:k + 1].contiguous(), opt)
            adj1 = tp.propagate_backward(u[k:k + 1].contiguous(), opt)
            torch.cuda.synchronize()
            assert rel(to_np(one[0]), to_np(big[k])) <= ulps, (ny, k)
            assert rel(to_np(adj1[0]), to_np(adj[k])) <= ulps, (ny, k)
        torch.cuda.synchronize()
        assert rel(to_np(big), _oracle(to_np(u), opt)) <= TOL[dtype]


def test_round_smooth_padding():
    """round_smooth rounds 2n up to the next 2/3/5/7-smooth length (11 x 13
    -> 24 x 27, instead of the Bluestein lengths 22 x 26): against the oracle
    on the same padded grid."""
    tp = _tp()
    announce("any-length round_smooth padding")
    rng = np.random.default_rng(1270)
    u = crandn(rng, 2, 11, 13, dtype=np.complex128)
    opt = tp.Optics(dy=4e-6, dx=4e-6, wavelength=0.6e-6, z=3e-4, pad=2, round_pow2=False, round_smooth=True)
    assert opt.padded_shape(11, 13) == (24, 27)
    out = tp.propagate(to_gpu(u, torch), opt)
    torch.cuda.synchronize()
    assert rel(to_np(out), _oracle(u, opt)) <= 1e-12
