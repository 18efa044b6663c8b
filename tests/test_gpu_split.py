"""Split transforms (complex64): the column pass and the fused row
boundaries of a chain factor each transform as one radix-R pass across the
whole transform and sub-transforms held inside one wavefront, and the fused
boundaries modulate, store and differentiate at the pixels in split order.

Checks, at padded lengths where the split applies to the rows (1024 with 8
points per thread, 2048 and 4096 with 16; 8192 forward only) and to the
columns (1024 ... 8192):
* a chain of phase layers with an MSE epilogue, forward and backward in one
  call each, against one call per layer (whose row passes take the
  unsplit transforms: two FP32 factorisations of the same propagation, each
  within ~4e-7 of the FP64 result per layer, so relative L2 <= 2e-6 for the
  fields and <= 2e-5 for the mask gradients) and against the FP64 oracle's
  stack (fields <= 2e-5, mask gradients <= 2e-4), including a ragged grid
  (nx < half the padded width: the pixel-range checks in split order);
* the largest padded grid (8192^2) as a two-layer chain against the layer
  by layer calls;
* a complex64 chain of lenses with per-layer optics: output field and
  focal-length gradients against the oracle (the lens phase derivative is
  evaluated at the split-order pixels)."""
import numpy as np
import pytest

import oracle
from tests._util import announce, crandn, rel, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SAME_FIELD, SAME_GRAD = 2e-6, 2e-5
ORACLE_FIELD, ORACLE_GRAD = 2e-5, 2e-4


def _tp():
    import paper_2411_18591_amd as tp
    return tp


def _chain(tp, u0, phis, T, opt, fused):
    """Forward chain with MSE epilogue and backward chain to the masks."""
    L = phis.shape[0]
    Pg, Tg = to_gpu(phis, torch), to_gpu(T, torch)
    u = [to_gpu(u0, torch)] + [torch.empty_like(to_gpu(u0, torch)) for _ in range(L)]
    g = [torch.empty_like(u[0]) for _ in range(2)]
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    gm = torch.zeros_like(Pg)
    els = [{"phase": Pg[l]} for l in range(L)]
    els[-1].update(epi=tp._capi.TO_EPI_MSE, epi_ref=Tg, epi_scale=1.0 / u0.size, epi_grad=g[0], epi_loss=loss)
    layers = list(range(L - 1, -1, -1))
    gout = [g[k % 2] for k in range(L)]
    gin = [g[(k + 1) % 2] for k in range(L)]
    if fused:
        tp.propagate_jobs(u[:L], [opt] * L, outs=u[1:], elements=els)
        tp.propagate_backward_jobs(gout, [opt] * L, saved_ins=[u[l] for l in layers], grad_ins=gin,
                                   grad_phases=[gm[l] for l in layers],
                                   elements=[{"phase": Pg[l]} for l in layers])
    else:
        for l in range(L):
            tp.propagate_jobs([u[l]], [opt], outs=[u[l + 1]], elements=[els[l]])
        for k, l in enumerate(layers):
            tp.propagate_backward_jobs([gout[k]], [opt], saved_ins=[u[l]], grad_ins=[gin[k]],
                                       grad_phases=[gm[l]], elements=[{"phase": Pg[l]}])
    torch.cuda.synchronize()
    return [to_np(t) for t in u], float(loss.item()), to_np(gm), to_np(g[L % 2])


def _inputs(rng, B, ny, nx, L):
    u0 = crandn(rng, B, ny, nx, dtype=np.complex64)
    phis = (rng.random((L, ny, nx)) * 2 * np.pi).astype(np.float32)
    T = rng.random((ny, nx)).astype(np.float32)
    return u0, phis, T


@pytest.mark.parametrize("shape", [(2, 512, 512, 3), (1, 1000, 1000, 2), (1, 2048, 2048, 2)])
def test_split_chain_matches_layers_and_oracle(shape):
    tp = _tp()
    B, ny, nx, L = shape
    announce(f"split chain {B}x{ny}x{nx} L={L} complex64")
    rng = np.random.default_rng(8100 + ny)
    d, lam, z = 8e-6, 0.7e-6, 0.03
    u0, phis, T = _inputs(rng, B, ny, nx, L)
    opt = tp.Optics(dy=d, dx=d, wavelength=lam, z=z, pad=2)
    uf, lf, gf, gif = _chain(tp, u0, phis, T, opt, True)
    us, ls, gs, gis = _chain(tp, u0, phis, T, opt, False)
    announce(f"split chain: fused vs per layer: fields {max(rel(uf[l], us[l]) for l in range(1, L + 1)):.2e}, "
             f"mask gradients {rel(gf, gs):.2e}, input gradient {rel(gif, gis):.2e}")
    for l in range(1, L + 1):
        assert rel(uf[l], us[l]) <= SAME_FIELD, (l, rel(uf[l], us[l]))
    assert abs(lf - ls) <= SAME_GRAD * abs(ls)
    assert rel(gf, gs) <= SAME_GRAD, rel(gf, gs)
    assert rel(gif, gis) <= SAME_FIELD, rel(gif, gis)

    pad = opt.padded_shape(ny, nx)
    ref = [u0.astype(np.complex128)]
    for l in range(L):
        ref.append(oracle.propagate(oracle.modulate(ref[-1], oracle.phase_mask(phis[l])), d, d, lam, z,
                                    oracle.ASM, padded=pad))
    loss, g = oracle.mse_intensity(ref[-1], T)
    grads = [None] * L
    for l in range(L - 1, -1, -1):
        m = oracle.phase_mask(phis[l])
        gmod = oracle.propagate(g, d, d, lam, z, oracle.ASM, adjoint=True, padded=pad)
        grads[l] = oracle.grad_phase(gmod, oracle.modulate(ref[l], m))
        g = oracle.modulate(gmod, m, conj=True)
    for l in range(1, L + 1):
        e = rel(uf[l], ref[l])
        announce(f"split chain layer {l}: field error vs oracle {e:.2e}")
        assert e <= ORACLE_FIELD, (l, e)
    assert abs(lf - loss) <= 4 * ORACLE_FIELD * loss
    announce(f"split chain: mask gradients vs oracle {max(rel(gf[l], grads[l]) for l in range(L)):.2e}, "
             f"input gradient {rel(gif, g):.2e}")
    for l in range(L):
        assert rel(gf[l], grads[l]) <= ORACLE_GRAD, (l, rel(gf[l], grads[l]))
    assert rel(gif, g) <= ORACLE_FIELD, rel(gif, g)


def test_split_chain_largest_grid():
    """4096^2 padded to 8192^2: the forward boundary and the 8192-point
    column pass take the split transforms, the backward boundary does not."""
    tp = _tp()
    announce("split chain 1x4096x4096 L=2 complex64")
    rng = np.random.default_rng(8190)
    u0, phis, T = _inputs(rng, 1, 4096, 4096, 2)
    opt = tp.Optics(dy=4e-6, dx=4e-6, wavelength=0.6e-6, z=0.05, pad=2)
    uf, lf, gf, gif = _chain(tp, u0, phis, T, opt, True)
    us, ls, gs, gis = _chain(tp, u0, phis, T, opt, False)
    announce(f"split chain 8192: fused vs per layer: fields {max(rel(uf[l], us[l]) for l in (1, 2)):.2e}, "
             f"mask gradients {rel(gf, gs):.2e}, input gradient {rel(gif, gis):.2e}")
    for l in (1, 2):
        assert rel(uf[l], us[l]) <= SAME_FIELD, (l, rel(uf[l], us[l]))
    assert abs(lf - ls) <= SAME_GRAD * abs(ls)
    assert rel(gf, gs) <= SAME_GRAD
    assert rel(gif, gis) <= SAME_FIELD


def test_split_chain_lens_grad_f():
    tp = _tp()
    announce("split chain with lenses, per-layer optics, complex64")
    rng = np.random.default_rng(8200)
    B, n, L = 2, 512, 3
    u0 = crandn(rng, B, n, n, dtype=np.complex64)
    opts = [tp.Optics(dy=6e-6, dx=6e-6, wavelength=lam, z=z, pad=2)
            for lam, z in ((500e-9, 0.01), (600e-9, 0.02), (550e-9, 0.015))]
    fs = [0.05, -0.08, 0.1]
    gout_np = crandn(rng, B, n, n, dtype=np.complex64)
    gout = to_gpu(gout_np, torch)
    u = [to_gpu(u0, torch)] + [torch.empty_like(to_gpu(u0, torch)) for _ in range(L)]
    gb = [gout.clone(), torch.empty_like(gout)]
    gfs = [torch.zeros((), dtype=torch.float64, device="cuda") for _ in range(L)]
    layers = list(range(L - 1, -1, -1))
    tp.propagate_jobs(u[:L], opts, outs=u[1:], elements=[{"lens_f": f} for f in fs])
    tp.propagate_backward_jobs([gb[k % 2] for k in range(L)], [opts[l] for l in layers],
                               saved_ins=[u[l] for l in layers], grad_ins=[gb[(k + 1) % 2] for k in range(L)],
                               grad_fs=[gfs[l] for l in layers], elements=[{"lens_f": fs[l]} for l in layers])
    torch.cuda.synchronize()
    v = u0.astype(np.complex128)
    us = [v]
    for l in range(L):
        o = opts[l]
        v = oracle.propagate(oracle.modulate(v, oracle.lens(n, n, o.dy, o.dx, o.wavelength, fs[l])), o.dy, o.dx,
                             o.wavelength, o.z, oracle.ASM, 2)
        us.append(v)
    for l in range(1, L + 1):
        assert rel(to_np(u[l]), us[l]) <= ORACLE_FIELD, l
    g = gout_np.astype(np.complex128)
    for l in range(L - 1, -1, -1):
        o = opts[l]
        M = oracle.lens(n, n, o.dy, o.dx, o.wavelength, fs[l])
        gm = oracle.propagate(g, o.dy, o.dx, o.wavelength, o.z, oracle.ASM, 2, adjoint=True)
        gf = oracle.grad_lens_f(gm, oracle.modulate(us[l], M), n, n, o.dy, o.dx, o.wavelength, fs[l])
        got = float(gfs[l].item())
        announce(f"split lens chain layer {l}: dL/df {got:.6e} vs oracle {gf:.6e}")
        assert abs(got - gf) <= ORACLE_GRAD * abs(gf), (l, got, gf)
        g = oracle.modulate(gm, M, conj=True)
    assert rel(to_np(gb[L % 2]), g) <= ORACLE_FIELD
