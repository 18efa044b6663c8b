"""The evaluation workloads at their full sizes, in the launch configuration
the benchmark times, checked where the FP64 oracle can reach them.

* Diffractive network (64 x 1024^2 complex64 fields, 5 phase masks, ASM
  10 cm, 2x padding, MSE loss, backward to the masks): the library's
  training step.  Field 0 through all five layers against the oracle; the
  fused loss against its definition on the returned output; the mask
  gradients of the complex128 step against central finite differences of
  its own loss along the gradient direction, and the complex64 gradients
  against the complex128 ones.
* Polarized multi-wavelength focusing (8 wavelengths x 3 components x
  2048^2, QWP -> LP -> lens f = 20 cm, Fresnel z = 20 cm, weighted-intensity
  loss, gradient to f), all jobs in one call.  The Gaussian input, the lens
  phase and the Fresnel transfer function are all separable in (y, x), so
  every output pixel is J[c][0] H(0,0) a(y) a(x), with a(.) a 1-D zero-padded
  propagation formed from the oracle's FFT and transfer function: sampled
  rows against that, the loss against its separable form, dL/df against
  central differences of the separable loss, and the closed forms (the QWP +
  LP pair passes half the power; the focal spot radius is lambda f/(pi w0)).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests._util import announce, rel, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _tp():
    import paper_2411_18591_amd as tp
    return tp


@pytest.mark.timeout(900)
def test_diffractive_network_full_size():
    tp = _tp()
    from paper_2411_18591_amd.diffnet import DiffractiveNet
    wl = workloads.DiffractiveNetWorkload()
    announce(f"diffractive network {wl.batch} x {wl.n}^2, {wl.layers} layers: inputs")
    u0 = wl.fields()
    masks = wl.masks()
    T = wl.target()
    opt = tp.Optics(dy=wl.d, dx=wl.d, wavelength=wl.wavelength, z=wl.z, pad=wl.pad)

    announce("diffractive network: complex64 step")
    net = DiffractiveNet(to_gpu(u0, torch), to_gpu(masks, torch), to_gpu(T, torch), opt)
    net.step()
    torch.cuda.synchronize()
    loss64 = float(net.loss.item())
    g64 = net.gmask.double().cpu().numpy()
    out0_64 = to_np(net.u[-1][0])
    uL = to_np(net.u[-1])
    I = uL.real.astype(np.float64) ** 2 + uL.imag.astype(np.float64) ** 2
    loss_def = float(np.mean((I - T.astype(np.float64)) ** 2))
    del uL, I, net
    assert abs(loss64 - loss_def) <= 1e-5 * loss_def

    announce("diffractive network: complex128 step and finite differences")
    net = DiffractiveNet(to_gpu(u0.astype(np.complex128), torch), to_gpu(masks.astype(np.float64), torch),
                         to_gpu(T.astype(np.float64), torch), opt)
    net.step()
    torch.cuda.synchronize()
    g128 = net.gmask.clone()
    out0_128 = to_np(net.u[-1][0])
    delta = g128 / g128.abs().max()
    deriv = float((g128 * delta).sum())
    eps = 1e-4
    net.masks += eps * delta
    lp = float(net.forward().item())
    net.masks -= 2 * eps * delta
    lm = float(net.forward().item())
    net.masks += eps * delta
    torch.cuda.synchronize()
    fd = (lp - lm) / (2 * eps)
    assert abs(fd - deriv) <= 1e-5 * abs(deriv), (fd, deriv)
    assert rel(g64, g128.cpu().numpy()) <= 1e-3
    del net

    announce("diffractive network: oracle on field 0 through 5 layers")
    us = oracle.stack_forward(u0[:1].astype(np.complex128), [m.astype(np.float64) for m in masks],
                              wl.d, wl.d, wl.wavelength, wl.z, oracle.ASM, wl.pad)
    e128, e64 = rel(out0_128, us[-1][0]), rel(out0_64, us[-1][0])
    announce(f"diffractive network: field 0 after 5 layers, error c128 {e128:.2e}, c64 {e64:.2e}")
    assert e128 <= 1e-12, e128
    assert e64 <= 2e-5, e64


def _prop1d(v, h):
    """crop(IDFT(h DFT(zero_pad(v)))) on the oracle's FFT: the 1-D factor of
    a separable propagation (the window's offset in the padded axis does not
    matter: the operation is a circular convolution)."""
    p = h.size
    x = np.zeros(p, dtype=np.complex128)
    x[: v.size] = v
    return oracle.fft(oracle.fft(x, -1) * h, +1)[: v.size] / p


def _separable_axis(n, d, lam, z, f, w0, pad):
    """a(.) and H(0,0) for one wavelength (square grid: a is the same along
    y and x)."""
    col = oracle.transfer(pad * n, 8, d, d, lam, z, oracle.FRESNEL)[:, 0]
    h00 = col[0]
    g = workloads.gaussian_amplitude(n, 1, d, d, w0)[:, 0]
    lens = oracle.lens(n, 1, d, d, lam, f)[:, 0]
    return _prop1d(g * lens, col / h00), h00


@pytest.mark.timeout(600)
@pytest.mark.parametrize("z_over_f", [1.0, 0.75])
def test_polarized_focusing_full_size(z_over_f):
    """z = f is the workload itself.  There dL/df vanishes: a real, even
    input gives a real focal-plane field u and a real first-order change
    du/df up to one common phase, so d|u|^2/df = 2 Re(conj(u) du/df) = 0; the
    gradient is then checked against zero on the loss's own scale.  The
    z = 0.75 f variant (same shapes, out of focus) has a finite dL/df for the
    finite-difference check."""
    tp = _tp()
    wl = workloads.PolarizedWorkload()
    wl.z = wl.f * z_over_f
    n, d, K = wl.n, wl.d, len(wl.wavelengths)
    announce(f"polarized focusing {K} wavelengths x 3 x {n}^2, z = {wl.z}, one call")
    J = tp.jones3(tp.waveplate(wl.qwp_angle, math.pi / 2), tp.linear_polarizer(wl.lp_angle))
    Jo = oracle.embed_jones(oracle.linear_polarizer(wl.lp_angle) @ oracle.waveplate(wl.qwp_angle, math.pi / 2))
    assert np.abs(np.array(J) - Jo).max() < 1e-15
    sJ = float(np.sum(np.abs(Jo[:, 0]) ** 2))
    assert abs(sJ - 0.5) < 1e-12  # circular light through a polarizer: half the power

    W = wl.weight()
    Eg = to_gpu(wl.field(), torch)
    Wg = to_gpu(W, torch)
    outs = torch.empty_like(Eg)
    grads = torch.empty_like(Eg)
    losses = torch.zeros(K, dtype=torch.float64, device="cuda")
    gfs = torch.zeros(K, dtype=torch.float64, device="cuda")
    opts = [tp.Optics(dy=d, dx=d, wavelength=float(lam), z=wl.z, method="fresnel", pad=wl.pad)
            for lam in wl.wavelengths]
    els = [dict(jones=J, lens_f=wl.f, epi=tp._capi.TO_EPI_WEIGHTED, epi_ref=Wg, epi_scale=d * d,
                epi_grad=grads[k], epi_loss=losses[k]) for k in range(K)]
    tp.propagate_jobs(list(Eg), opts, outs=list(outs), elements=els, ncomp=3)
    tp.propagate_backward_jobs(list(grads), opts, saved_ins=list(Eg), grad_ins=[None] * K,
                               grad_fs=list(gfs), elements=[dict(jones=J, lens_f=wl.f)] * K, ncomp=3)
    torch.cuda.synchronize()

    announce("polarized focusing: separable oracle checks")
    rng = np.random.default_rng(3100)
    rows = np.concatenate([[n // 2], rng.choice(n, 31, replace=False)])
    Wd = W.astype(np.float64)
    y = (np.arange(n) - n // 2) * d
    for k, lam in enumerate(wl.wavelengths):
        lam = float(lam)
        a, h00 = _separable_axis(n, d, lam, wl.z, wl.f, wl.w0, wl.pad)
        got = to_np(outs[k][:, torch.from_numpy(rows).cuda(), :])
        exp = np.stack([Jo[c, 0] * h00 * a[rows, None] * a[None, :] for c in range(3)])
        assert rel(got, exp) <= 2e-5, (k, rel(got, exp))
        a2 = np.abs(a) ** 2
        loss_exp = d * d * sJ * float(a2 @ Wd @ a2)
        assert abs(float(losses[k].item()) - loss_exp) <= 1e-4 * loss_exp, k

        # dL/df by central differences of the separable loss
        hf = 1e-5 * wl.f

        def loss_at(f):
            b, _ = _separable_axis(n, d, lam, wl.z, f, wl.w0, wl.pad)
            b2 = np.abs(b) ** 2
            return d * d * sJ * float(b2 @ Wd @ b2)
        fd = (loss_at(wl.f + hf) - loss_at(wl.f - hf)) / (2 * hf)
        gf = float(gfs[k].item())
        if z_over_f == 1.0:
            assert abs(fd) <= 1e-6 * loss_exp / wl.f
            assert abs(gf) <= 1e-4 * loss_exp / wl.f, (k, gf)
        else:
            assert abs(gf - fd) <= 1e-3 * abs(fd), (k, gf, fd)

        # closed forms: half the input power reaches the output; focal spot
        # radius lambda f / (pi w0) (collimated beam, Rayleigh range >> f)
        I = (outs[k].abs() ** 2).sum(0).double()
        p_out = float(I.sum()) * d * d
        g = workloads.gaussian_amplitude(n, n, d, d, wl.w0)
        p_in = float(np.sum(g * g)) * d * d
        assert abs(p_out - 0.5 * p_in) <= 1e-4 * p_in, k
        if z_over_f != 1.0:
            continue
        yy = torch.from_numpy(y).cuda()
        r2 = (yy[:, None] ** 2 + yy[None, :] ** 2)
        w_out = math.sqrt(2.0 * float((I * r2).sum() / I.sum()))
        w_exp = lam * wl.f / (math.pi * wl.w0)
        assert abs(w_out / w_exp - 1.0) <= 1e-2, (k, w_out, w_exp)
