"""The entry point that allocates nothing (to_propagate_noalloc) against
to_propagate on the same jobs, called through the C-ABI: two calls in a
row, the second with a smaller input, so the static area's leftovers from
the first call must not leak into the second.  The first call spans three
chunks of the static area (1024^2 complex64 fields padded to 2048^2, three
fields per chunk) and carries the MSE loss epilogue; the second is a ragged
grid with a lens and the Fresnel transfer function.  A complex128 pair
follows.  Bars: complex64 fields and gradients relative L2 <= 2e-5 against
the fused entry point (both are FP32 FFTs of the same operator), complex128
<= 1e-12; losses to the same relative bars."""
import numpy as np
import pytest
import torch

import paper_2411_18591_amd as tp
from paper_2411_18591_amd import _capi

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = a.detach().cpu().numpy(), b.detach().cpu().numpy()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def field(rng, shape, dtype):
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return torch.from_numpy(u.astype(np.complex64 if dtype == torch.complex64 else np.complex128)).cuda()


def run_both(u, opt, dtype, **kw):
    """One job through to_propagate and through to_propagate_noalloc."""
    outs = []
    for noalloc in (False, True):
        out = torch.full_like(u, float("nan"))
        extra = {}
        if kw.get("epi") == _capi.TO_EPI_MSE:
            extra = dict(epi_grad=torch.full_like(u, float("nan")),
                         epi_loss=torch.zeros((), dtype=torch.float64, device=u.device))
        job = tp.make_job(u, opt, out=out, **kw, **extra)
        s = torch.cuda.current_stream().cuda_stream
        if noalloc:
            _capi.propagate_noalloc([job], tp._dtype_code(u), s)
        else:
            _capi.propagate([job], tp._dtype_code(u), s)
        torch.cuda.synchronize()
        outs.append((out, extra))
    return outs


@pytest.mark.parametrize("dtype,bar", [(torch.complex64, 2e-5), (torch.complex128, 1e-12)])
def test_noalloc_matches_to_propagate_twice(dtype, bar):
    rng = np.random.default_rng(7)
    rdt = torch.float32 if dtype == torch.complex64 else torch.float64
    # call 1: several chunks of the static area, phase mask, MSE loss
    n1, b1 = (1024, 7) if dtype == torch.complex64 else (512, 10)
    print(f"[noalloc] call 1: {b1} x {n1}^2 {dtype}", flush=True)
    u1 = field(rng, (b1, n1, n1), dtype)
    phi = torch.from_numpy(rng.random((n1, n1)) * 2 * np.pi).to(rdt).cuda()
    target = torch.from_numpy(rng.random((n1, n1))).to(rdt).cuda()
    opt1 = tp.Optics(dy=8e-6, dx=8e-6, wavelength=0.7e-6, z=0.1, pad=2)
    (o_ref, e_ref), (o_na, e_na) = run_both(u1, opt1, dtype, phase=phi, epi=_capi.TO_EPI_MSE, epi_ref=target,
                                            epi_scale=1.0 / u1.numel())
    assert torch.isfinite(o_na).all()
    assert rel(o_na, o_ref) <= bar
    assert rel(e_na["epi_grad"], e_ref["epi_grad"]) <= bar
    assert abs(float(e_na["epi_loss"]) - float(e_ref["epi_loss"])) <= bar * abs(float(e_ref["epi_loss"]))
    # call 2: smaller, ragged, lens + Fresnel
    print("[noalloc] call 2: 2 x 200 x 160", flush=True)
    u2 = field(rng, (2, 200, 160), dtype)
    opt2 = tp.Optics(dy=5e-6, dx=6e-6, wavelength=0.6e-6, z=0.03, pad=2, method="fresnel")
    (o_ref, _), (o_na, _) = run_both(u2, opt2, dtype, lens_f=0.05)
    assert torch.isfinite(o_na).all()
    assert rel(o_na, o_ref) <= bar
