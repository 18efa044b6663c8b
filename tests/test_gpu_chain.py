"""Chains of propagations in one call (each layer's input is the previous
layer's output: the paper's diffractive-network example, section
"Gradient-based optimization").  The library runs them chunk by chunk with
fused layer boundaries; the result must equal running the layers one call at
a time, and the FP64 oracle's stack.

Bars: complex64 relative L2 <= 2e-5 against the oracle (fields), <= 2e-4
(mask gradients); fused against one-by-one <= 1e-6 (complex64) / 1e-13
(complex128): for complex128 the same arithmetic in the same order, up to
the compiler's choice of fused multiply-adds in the fused kernels; for
complex64 the fused boundaries take the split transforms, another FP32
factorisation of the same propagation (larger grids: test_gpu_split.py)."""
import numpy as np
import pytest

import oracle
from tests._util import announce, crandn, rel, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ORACLE_TOL = {np.complex64: 2e-5, np.complex128: 1e-12}
GRAD_TOL = {np.complex64: 2e-4, np.complex128: 1e-11}
SAME_TOL = {np.complex64: 1e-6, np.complex128: 1e-13}


def _tp():
    import paper_2411_18591_amd as tp
    return tp


def _stack(rng, B, ny, nx, L, dtype):
    rdt = np.float32 if dtype == np.complex64 else np.float64
    u0 = crandn(rng, B, ny, nx, dtype=dtype)
    phis = (rng.random((L, ny, nx)) * 2 * np.pi).astype(rdt)
    T = rng.random((ny, nx)).astype(rdt)
    return u0, phis, T


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("shape", [(3, 64, 64, 4), (5, 100, 72, 3), (2, 48, 200, 5)])
def test_forward_backward_chain_matches_layers_and_oracle(shape, dtype):
    """A chain of L phase layers with an MSE epilogue: one call forward, one
    call backward (layers L-1 .. 0, gradient buffers alternating) against
    one call per layer and against the oracle's stack."""
    tp = _tp()
    B, ny, nx, L = shape
    announce(f"chain {B}x{ny}x{nx} L={L} {dtype.__name__}")
    rng = np.random.default_rng(700 + ny + L)
    d, lam, z = 8e-6, 0.7e-6, 0.02
    u0, phis, T = _stack(rng, B, ny, nx, L, dtype)
    opt = tp.Optics(dy=d, dx=d, wavelength=lam, z=z, pad=2)
    Pg, Tg = to_gpu(phis, torch), to_gpu(T, torch)
    scale = 1.0 / u0.size

    def run(fused):
        u = [to_gpu(u0, torch)] + [torch.empty_like(to_gpu(u0, torch)) for _ in range(L)]
        g = [torch.empty_like(u[0]) for _ in range(2)]
        loss = torch.zeros((), dtype=torch.float64, device="cuda")
        gm = torch.zeros_like(Pg)
        els = [{"phase": Pg[l]} for l in range(L)]
        els[-1].update(epi=tp._capi.TO_EPI_MSE, epi_ref=Tg, epi_scale=scale, epi_grad=g[0], epi_loss=loss)
        layers = list(range(L - 1, -1, -1))
        gout = [g[k % 2] for k in range(L)]
        gin = [g[(k + 1) % 2] if l > 0 else None for k, l in enumerate(layers)]
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

    uf, lf, gf, gif = run(True)
    us, ls, gs, gis = run(False)
    for a, b in zip(uf, us):
        assert rel(a, b) <= SAME_TOL[dtype]
    assert abs(lf - ls) <= 10 * SAME_TOL[dtype] * abs(ls)
    assert rel(gf, gs) <= 10 * SAME_TOL[dtype]

    # the oracle's stack on the library's padded grid (2x, rounded up to a
    # power of two)
    pad = opt.padded_shape(ny, nx)
    ref = [u0.astype(np.complex128)]
    for l in range(L):
        ref.append(oracle.propagate(oracle.modulate(ref[-1], oracle.phase_mask(phis[l])), d, d, lam, z,
                                    oracle.ASM, padded=pad))
    loss, g = oracle.mse_intensity(ref[-1], T)
    grads = [None] * L
    for l in range(L - 1, -1, -1):
        m = oracle.phase_mask(phis[l])
        gm = oracle.propagate(g, d, d, lam, z, oracle.ASM, adjoint=True, padded=pad)
        grads[l] = oracle.grad_phase(gm, oracle.modulate(ref[l], m))
        g = oracle.modulate(gm, m, conj=True)
    for l in range(1, L + 1):
        e = rel(uf[l], ref[l])
        announce(f"chain layer {l}: field error vs oracle {e:.2e}")
        assert e <= ORACLE_TOL[dtype], (l, e)
    assert abs(lf - loss) <= 4 * ORACLE_TOL[dtype] * loss
    for l in range(L):
        assert rel(gf[l], grads[l]) <= GRAD_TOL[dtype], l


def test_chain_with_lens_and_grad_f():
    """Layers with a lens (focal-length gradients per layer) and varying
    distance and wavelength along the chain."""
    tp = _tp()
    announce("chain with lenses, per-layer optics")
    rng = np.random.default_rng(720)
    B, n, L = 2, 64, 3
    u0 = crandn(rng, B, n, n, dtype=np.complex128)
    opts = [tp.Optics(dy=6e-6, dx=6e-6, wavelength=lam, z=z, pad=2)
            for lam, z in ((500e-9, 0.01), (600e-9, 0.02), (550e-9, 0.015))]
    fs = [0.05, -0.08, 0.1]
    gout = to_gpu(crandn(rng, B, n, n, dtype=np.complex128), torch)

    def run(fused):
        u = [to_gpu(u0, torch)] + [torch.empty_like(to_gpu(u0, torch)) for _ in range(L)]
        gb = [gout.clone(), torch.empty_like(gout)]
        gfs = [torch.zeros((), dtype=torch.float64, device="cuda") for _ in range(L)]
        layers = list(range(L - 1, -1, -1))
        if fused:
            tp.propagate_jobs(u[:L], opts, outs=u[1:], elements=[{"lens_f": f} for f in fs])
            tp.propagate_backward_jobs([gb[k % 2] for k in range(L)], [opts[l] for l in layers],
                                       saved_ins=[u[l] for l in layers],
                                       grad_ins=[gb[(k + 1) % 2] for k in range(L)],
                                       grad_fs=[gfs[l] for l in layers], elements=[{"lens_f": fs[l]} for l in layers])
        else:
            for l in range(L):
                tp.propagate(u[l], opts[l], out=u[l + 1], lens_f=fs[l])
            for k, l in enumerate(layers):
                tp.propagate_backward(gb[k % 2], opts[l], saved_in=u[l], grad_in=gb[(k + 1) % 2], grad_f=gfs[l],
                                      lens_f=fs[l])
        torch.cuda.synchronize()
        return to_np(u[L]), [float(t.item()) for t in gfs], to_np(gb[L % 2])

    a = run(True)
    b = run(False)
    assert rel(a[0], b[0]) <= 1e-13
    assert rel(a[2], b[2]) <= 1e-13
    for x, y in zip(a[1], b[1]):
        assert abs(x - y) <= 1e-12 * abs(y)
    # oracle
    v = u0.astype(np.complex128)
    us = [v]
    for l in range(L):
        o = opts[l]
        v = oracle.propagate(oracle.modulate(v, oracle.lens(n, n, o.dy, o.dx, o.wavelength, fs[l])), o.dy, o.dx,
                             o.wavelength, o.z, oracle.ASM, 2)
        us.append(v)
    assert rel(a[0], us[L]) <= 1e-12
    g = to_np(gout).astype(np.complex128)
    for l in range(L - 1, -1, -1):
        o = opts[l]
        M = oracle.lens(n, n, o.dy, o.dx, o.wavelength, fs[l])
        gm = oracle.propagate(g, o.dy, o.dx, o.wavelength, o.z, oracle.ASM, 2, adjoint=True)
        gf = oracle.grad_lens_f(gm, oracle.modulate(us[l], M), n, n, o.dy, o.dx, o.wavelength, fs[l])
        assert abs(a[1][l] - gf) <= 1e-10 * abs(gf), l
        g = oracle.modulate(gm, M, conj=True)
    assert rel(a[2], g) <= 1e-12


def test_misaligned_aliasing_is_not_fused():
    """A second layer that writes over the first layer's input shifted by one
    field must see the one-by-one order (the library declines to fuse it)."""
    tp = _tp()
    announce("chain with misaligned aliasing")
    rng = np.random.default_rng(721)
    B, n = 4, 32
    Z = to_gpu(crandn(rng, B + 1, n, n, dtype=np.complex64), torch)
    Z2 = Z.clone()
    opt = tp.Optics(dy=5e-6, dx=5e-6, wavelength=600e-9, z=0.01, pad=2)
    Y = torch.empty((B, n, n), dtype=torch.complex64, device="cuda")
    Y2 = torch.empty_like(Y)
    tp.propagate_jobs([Z[:B], Y], [opt, opt], outs=[Y, Z[1:]])
    tp.propagate(Z2[:B], opt, out=Y2)
    tp.propagate(Y2, opt, out=Z2[1:])
    torch.cuda.synchronize()
    assert torch.equal(Z, Z2) and torch.equal(Y, Y2)


def test_long_chain_splits():
    """More layers than one fused chain holds (16): split into chains, same
    result as one layer per call."""
    tp = _tp()
    announce("chain of 19 layers")
    rng = np.random.default_rng(722)
    B, n, L = 2, 16, 19
    u0 = to_gpu(crandn(rng, B, n, n, dtype=np.complex128), torch)
    phis = to_gpu(rng.random((L, n, n)) * 6, torch)
    opt = tp.Optics(dy=5e-6, dx=5e-6, wavelength=600e-9, z=0.001, pad=2)
    u = [u0] + [torch.empty_like(u0) for _ in range(L)]
    tp.propagate_jobs(u[:L], [opt] * L, outs=u[1:], elements=[{"phase": phis[l]} for l in range(L)])
    v = u0
    for l in range(L):
        v = tp.propagate(v, opt, phase=phis[l])
    torch.cuda.synchronize()
    assert rel(to_np(u[L]), to_np(v)) <= 1e-13


def test_training_step_graph_capture():
    """The diffractive-network training step (one chained call forward, one
    backward) captured in a HIP graph: three replays with new inputs, each
    equal to an eager step."""
    tp = _tp()
    from paper_2411_18591_amd.diffnet import DiffractiveNet
    announce("training step in a HIP graph")
    rng = np.random.default_rng(730)
    B, n, L = 4, 64, 3
    opt = tp.Optics(dy=8e-6, dx=8e-6, wavelength=700e-9, z=0.02, pad=2)
    net = DiffractiveNet(torch.zeros((B, n, n), dtype=torch.complex64, device="cuda"),
                         to_gpu((rng.random((L, n, n)) * 6).astype(np.float32), torch),
                         to_gpu(rng.random((n, n)).astype(np.float32), torch), opt)

    def fill(seed):
        r = np.random.default_rng(seed)
        net.u[0].copy_(to_gpu(crandn(r, B, n, n, dtype=np.complex64), torch))

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fill(1)
        net.step()  # sizes the workspaces outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        net.step()
    torch.cuda.synchronize()
    for rep in range(3):
        fill(200 + rep)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [net.loss.clone(), net.gmask.clone(), net.u[L].clone()]
        net.step()
        torch.cuda.synchronize()
        assert torch.equal(got[0], net.loss) and torch.equal(got[1], net.gmask) and torch.equal(got[2], net.u[L]), rep


def test_transient_links_give_the_same_gradients():
    """Backward chain whose intermediate gradient buffers are marked
    transient (only the next layer reads them): the fused boundaries may skip
    storing them; the mask gradients and the first layer's input gradient
    are bitwise those of the same call without the flag."""
    tp = _tp()
    announce("transient backward links")
    rng = np.random.default_rng(760)
    B, n, L = 3, 64, 4
    u0, phis, T = _stack(rng, B, n, n, L, np.complex64)
    opt = tp.Optics(dy=8e-6, dx=8e-6, wavelength=0.7e-6, z=0.02, pad=2)
    Pg = to_gpu(phis, torch)
    u = [to_gpu(u0, torch)] + [torch.empty_like(to_gpu(u0, torch)) for _ in range(L)]
    tp.propagate_jobs(u[:L], [opt] * L, outs=u[1:], elements=[{"phase": Pg[l]} for l in range(L)])
    gL = to_gpu(crandn(rng, B, n, n, dtype=np.complex64), torch)
    layers = list(range(L - 1, -1, -1))

    def run(transient):
        g = [gL.clone(), torch.empty_like(gL)]
        gm = torch.zeros_like(Pg)
        gout = [g[k % 2] for k in range(L)]
        gin = [g[(k + 1) % 2] for k in range(L)]
        gin[-1] = torch.empty_like(gL)  # the first layer's input gradient, kept
        tp.propagate_backward_jobs(gout, [opt] * L, saved_ins=[u[l] for l in layers], grad_ins=gin,
                                   grad_phases=[gm[l] for l in layers],
                                   elements=[{"phase": Pg[l]} for l in layers],
                                   transient=[transient and k < L - 1 for k in range(L)])
        torch.cuda.synchronize()
        return gm.clone(), gin[-1].clone()

    gm_a, gi_a = run(False)
    gm_b, gi_b = run(True)
    assert torch.equal(gm_a, gm_b)
    assert torch.equal(gi_a, gi_b)
