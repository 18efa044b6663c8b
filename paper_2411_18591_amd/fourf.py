"""Polychromatic imaging through a 4f system (section "Polychromatic fields"
on the 4f system of the paper's first example): lenses of focal length f at
z = f and z = 3f, the image at z = 4f.  Per wavelength lambda the field goes
through

    v = P_f( L_f P_2f( L_f P_f(u) ) ),   L_f the thin lens of Eq. (field_modulation),

and the detected image is the incoherent sum of Eq. (I_poly),
I = sum_lambda w_lambda |v_lambda|^2 (weights on the intensity).

All wavelengths go to the library in one call: each wavelength is a chain
of three jobs (fused layer boundaries), and the last job of each chain adds
its weighted intensity to the shared image in the intensity epilogue, in
call order (so the sum is deterministic).  With ``method="auto"`` (the
paper's default) each distance takes the AS or DI method by the critical
distance; DI tables are built once per call and (wavelength, distance)."""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import Optics, _capi, _dtype_code, _real_dtype, _stream, make_job


class FourF:
    def __init__(self, f: float, dy: float, dx: float, *, pad: int = 2, method: str = "auto",
                 y0: float = 0.0, x0: float = 0.0, padded=None):
        self.f = float(f)
        self.dy, self.dx = float(dy), float(dx)
        self.pad = pad
        self.method = method
        self.y0, self.x0 = float(y0), float(x0)
        self.padded = padded

    def _opt(self, wavelength: float, z: float) -> Optics:
        return Optics(dy=self.dy, dx=self.dx, wavelength=float(wavelength), z=z, method=self.method,
                      pad=self.pad, y0=self.y0, x0=self.x0, padded=self.padded)

    def image(self, u: torch.Tensor, wavelengths: Sequence[float], weights: Sequence[float], *,
              out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Weighted incoherent image of fields ``u`` ([B, ny, nx] or [ny, nx],
        complex) at z = 4f: returns (or accumulates into ``out``) the real
        intensity of the shape of u."""
        if len(wavelengths) != len(weights):
            raise ValueError("one weight per wavelength")
        if out is None:
            out = torch.zeros(u.shape, dtype=_real_dtype(u), device=u.device)
        t1 = torch.empty_like(u)
        t2 = torch.empty_like(u)
        jobs = []
        for lam, w in zip(wavelengths, weights):
            jobs.append(make_job(u, self._opt(lam, self.f), out=t1))
            jobs.append(make_job(t1, self._opt(lam, 2 * self.f), out=t2, lens_f=self.f))
            jobs.append(make_job(t2, self._opt(lam, self.f), lens_f=self.f, epi=_capi.TO_EPI_INTENSITY,
                                 epi_out=out, epi_scale=float(w)))
        if jobs:
            _capi.propagate(jobs, _dtype_code(u), _stream(u))
        return out
