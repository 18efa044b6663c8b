"""The unfused plain form (the comparison baseline) against the oracle and
against the fused path: same results to rounding (complex64 <= 2e-5 relative
L2, complex128 <= 1e-12)."""
import numpy as np
import pytest

import oracle
from tests._util import announce, crandn, rel, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {np.complex64: 2e-5, np.complex128: 1e-12}


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("shape", [(32, 32, 64, 64), (100, 60, 256, 128), (64, 64, 64, 64)])
def test_plain_forward_backward(shape, dtype):
    import paper_2411_18591_amd as tp
    ny, nx, py, px = shape
    announce(f"plain form {shape} {dtype.__name__}")
    rng = np.random.default_rng(31)
    rdt = np.float32 if dtype == np.complex64 else np.float64
    u = crandn(rng, 3, ny, nx, dtype=dtype)
    g = crandn(rng, 3, ny, nx, dtype=dtype)
    phi = (rng.random((ny, nx)) * 6).astype(rdt)
    T = rng.random((ny, nx)).astype(rdt)
    d, lam, z = (6e-6, 7e-6), 0.6e-6, 0.02
    opt = tp.Optics(dy=d[0], dx=d[1], wavelength=lam, z=z, padded=(py, px))
    ug, gg, pg, Tg = (to_gpu(a, torch) for a in (u, g, phi, T))
    out_p = tp.propagate(ug, opt, phase=pg, plain=True)
    out_f = tp.propagate(ug, opt, phase=pg)
    o2, go_p, lo_p = tp.propagate_loss(ug, opt, kind="mse", ref=Tg, scale=1.0 / u.size, phase=pg, plain=True)
    o3, go_f, lo_f = tp.propagate_loss(ug, opt, kind="mse", ref=Tg, scale=1.0 / u.size, phase=pg)
    gp_p = torch.zeros_like(pg)
    gp_f = torch.zeros_like(pg)
    gi_p = tp.propagate_backward(gg, opt, saved_in=ug, grad_phase=gp_p, phase=pg, plain=True)
    gi_f = tp.propagate_backward(gg, opt, saved_in=ug, grad_phase=gp_f, phase=pg)
    torch.cuda.synchronize()
    M = oracle.phase_mask(phi)
    exp_out = oracle.propagate(oracle.modulate(u, M), d[0], d[1], lam, z, padded=(py, px))
    g_mod = oracle.propagate(g, d[0], d[1], lam, z, padded=(py, px), adjoint=True)
    exp_gin = oracle.modulate(g_mod, M, conj=True)
    exp_gp = oracle.grad_phase(g_mod, oracle.modulate(u, M))
    loss, exp_go = oracle.mse_intensity(exp_out, T)
    tol = TOL[dtype]
    assert rel(to_np(out_p), exp_out) <= tol
    assert rel(to_np(out_p), to_np(out_f)) <= tol
    assert rel(to_np(go_p), exp_go) <= 4 * tol
    assert abs(float(lo_p.item()) - loss) <= 4 * tol * loss
    assert rel(to_np(gi_p), exp_gin) <= tol
    assert rel(to_np(gp_p), exp_gp) <= (1e-4 if dtype == np.complex64 else 1e-11)
    assert rel(to_np(gp_p), to_np(gp_f)) <= (1e-4 if dtype == np.complex64 else 1e-11)
