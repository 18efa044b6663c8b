"""Polychromatic 4f imaging on the GPU (section "Polychromatic fields" on the
paper's 4f system): per wavelength P_f, lens, P_2f, lens, P_f and the
weighted incoherent sum of Eq. (I_poly), one library call for the whole
spectrum.  Checks: the FP64 oracle's composition of the same steps on small
grids (AS and the automatic AS/DI choice, both dtypes); the exact discrete
imaging identity of a Fresnel 4f system without padding at N dx^2 =
lambda f (the image is the input intensity with inverted coordinates, two
applications of the pinned lens f-f Fourier identity); and, at the paper's
scale (1000^2 padded to 2048^2, 251 wavelengths), the one-call image against
one call per wavelength (bitwise) and against the oracle on a three-line
spectrum."""
import numpy as np
import pytest

import oracle
import workloads
from tests._util import announce, crandn, rel, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _fourf():
    from paper_2411_18591_amd.fourf import FourF
    return FourF


def _pow2(n):
    p = 1
    while p < n:
        p *= 2
    return p


def _oracle_image(u, d, f, lams, wts, method, padded=None):
    """The oracle's 4f image: the same steps, one wavelength at a time, on
    the padded grid the library uses (2x, rounded up to a power of two)."""
    ny, nx = u.shape[-2:]
    if padded is None:
        padded = (_pow2(2 * ny), _pow2(2 * nx))
    pad = 2
    fields = []
    for lam in lams:
        def prop(v, z):
            meth = method
            if meth == "auto":
                meth = oracle.resolve_method(ny, nx, d, d, lam, z)
            return oracle.propagate(v, d, d, lam, z, meth, pad, padded=padded)
        L = oracle.lens(ny, nx, d, d, lam, f)
        v = prop(u, f)
        v = prop(oracle.modulate(v, L), 2 * f)
        v = prop(oracle.modulate(v, L), f)
        fields.append(v)
    return oracle.incoherent_sum(fields, wts)


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("method", [oracle.ASM, "auto"])
def test_small_4f_against_oracle(method, dtype):
    """48 x 40 fields (batch 2), 11 wavelengths over 575-825 nm with
    Gaussian weights; f chosen so that, with the automatic choice, f is
    below the critical distance (AS) at the shorter wavelengths and beyond
    it (DI) at the longest, and 2f is beyond it everywhere."""
    FourF = _fourf()
    name = "asm" if method == oracle.ASM else "auto"
    announce(f"4f small {name} {dtype.__name__}")
    rng = np.random.default_rng(990)
    ny, nx, d = 48, 40, 10e-6
    wl = workloads.Polychromatic4fWorkload(count=11, fwhm=80e-9)
    lams, wts = wl.wavelengths(), wl.weights()
    zc = [oracle.critical_distance(ny, nx, d, d, lam) for lam in lams]
    f = 0.75 * max(zc)
    u = crandn(rng, 2, ny, nx, dtype=dtype)
    sys = FourF(f, d, d, method=name)
    I = sys.image(to_gpu(u, torch), lams, wts)
    torch.cuda.synchronize()
    exp = _oracle_image(u, d, f, lams, wts, method)
    if name == "auto":
        meths = {oracle.resolve_method(ny, nx, d, d, lam, z) for lam in lams for z in (f, 2 * f)}
        assert meths == {oracle.ASM, oracle.DI}
    assert rel(to_np(I), exp) <= (4e-5 if dtype == np.complex64 else 1e-12)


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_fresnel_4f_inverts_the_image(dtype):
    """Fresnel transfer function, no padding (P(2f) = P(f) P(f) exactly),
    N dx^2 = lambda f: each f-lens-f stage is the centred DFT times
    (-i/N) exp(2 i k f), so the 4f image is |u(-r)|^2 exactly."""
    FourF = _fourf()
    announce(f"4f Fresnel inversion {dtype.__name__}")
    n, d, lam = 128, 10e-6, 640e-9
    f = n * d * d / lam
    rng = np.random.default_rng(991)
    u = crandn(rng, n, n, dtype=dtype)
    sys = FourF(f, d, d, method="fresnel", padded=(n, n))
    I = sys.image(to_gpu(u, torch), [lam], [1.0])
    torch.cuda.synchronize()
    idx = (-(np.arange(n) - n // 2)) % n  # centred index -m, wrapped
    idx = (idx + n // 2) % n
    exp = np.abs(u.astype(np.complex128)[np.ix_(idx, idx)]) ** 2
    assert rel(to_np(I), exp) <= (4e-5 if dtype == np.complex64 else 1e-12)


def test_paper_scale_spectrum():
    """1000^2 (padded 2048^2), 251 wavelengths, FWHM 10 nm, AS: the one-call
    image with one set of buffers (call-order sum) equals one call per
    wavelength bitwise; with four sets (chains concurrent on the lanes,
    private accumulators combined in lane order) it is deterministic
    (bitwise over repeats) and equal to the call-order sum to rounding; a
    three-line spectrum against the oracle."""
    FourF = _fourf()
    announce("4f 1000^2 x 251 wavelengths")
    wl = workloads.Polychromatic4fWorkload()
    u = to_gpu(wl.field(), torch)
    sys = FourF(wl.f, wl.d, wl.d, method="asm")
    lams, wts = wl.wavelengths(), wl.weights()
    I1 = sys.image(u, lams, wts, sets=1)
    I2 = torch.zeros_like(I1)
    for lam, w in zip(lams, wts):
        sys.image(u, [lam], [w], out=I2)
    I = sys.image(u, lams, wts)
    Ib = sys.image(u, lams, wts)
    torch.cuda.synchronize()
    assert torch.equal(I1, I2)
    assert torch.equal(I, Ib)
    assert rel(to_np(I), to_np(I1)) <= 1e-6
    assert float(I.min()) >= 0.0 and float(I.sum()) > 0.0
    pick = [100, 125, 150]
    I3 = sys.image(u, lams[pick], [0.2, 0.5, 0.3])
    torch.cuda.synchronize()
    exp = _oracle_image(wl.field().astype(np.complex128), wl.d, wl.f, lams[pick], [0.2, 0.5, 0.3], oracle.ASM)
    assert rel(to_np(I3), exp) <= 4e-5


@pytest.mark.parametrize("method", [oracle.ASM, "auto"])
def test_4f_at_padding_that_is_not_a_power_of_two(method):
    """The 4f image on 48 x 40 fields padded to 96 x 80 (the paper's own
    2x padding without rounding up; mixed-radix lines), AS and the automatic
    AS/DI choice, against the oracle's composition on the same grid."""
    FourF = _fourf()
    name = "asm" if method == oracle.ASM else "auto"
    announce(f"4f padded 96 x 80 {name}")
    rng = np.random.default_rng(993)
    ny, nx, d = 48, 40, 10e-6
    wl = workloads.Polychromatic4fWorkload(count=7, fwhm=80e-9)
    lams, wts = wl.wavelengths(), wl.weights()
    f = 0.75 * max(oracle.critical_distance(ny, nx, d, d, lam) for lam in lams)
    u = crandn(rng, 2, ny, nx, dtype=np.complex64)
    I = FourF(f, d, d, method=name, padded=(96, 80)).image(to_gpu(u, torch), lams, wts)
    torch.cuda.synchronize()
    exp = _oracle_image(u, d, f, lams, wts, method, padded=(96, 80))
    assert rel(to_np(I), exp) <= 4e-5


@pytest.mark.parametrize("padded", [None, (96, 80)])
def test_cached_di_tables_give_the_same_image(padded):
    """With the DI tables kept by the system (built once by
    to_transfer_table), images equal the per-call-table images bitwise; on
    the 96 x 80 grid the per-call tables are built transposed for the
    any-length sequence and the kept ones are transposed per job."""
    FourF = _fourf()
    announce(f"4f cached DI tables {padded}")
    rng = np.random.default_rng(992)
    ny, nx, d = 48, 40, 10e-6
    wl = workloads.Polychromatic4fWorkload(count=7, fwhm=40e-9)
    lams, wts = wl.wavelengths(), wl.weights()
    f = 2.0 * max(oracle.critical_distance(ny, nx, d, d, lam) for lam in lams)
    u = to_gpu(crandn(rng, 2, ny, nx, dtype=np.complex64), torch)
    a = FourF(f, d, d, method="auto", padded=padded).image(u, lams, wts)
    cached = FourF(f, d, d, method="auto", cache_tables=True, padded=padded)
    b = cached.image(u, lams, wts)
    c = cached.image(u, lams, wts)
    torch.cuda.synchronize()
    assert len(cached._tables) == 2 * len(lams)
    assert torch.equal(a, b) and torch.equal(b, c)
