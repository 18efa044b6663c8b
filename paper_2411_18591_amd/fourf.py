"""Polychromatic imaging through a 4f system (section "Polychromatic fields"
on the 4f system of the paper's first example): lenses of focal length f at
z = f and z = 3f, the image at z = 4f.  Per wavelength lambda the field goes
through

    v = P_f( L_f P_2f( L_f P_f(u) ) ),   L_f the thin lens of Eq. (field_modulation),

and the detected image is the incoherent sum of Eq. (I_poly),
I = sum_lambda w_lambda |v_lambda|^2 (weights on the intensity).

All wavelengths go to the library in one call: each wavelength is a chain
of three jobs (fused layer boundaries), and the last job of each chain adds
its weighted intensity to the shared image in the intensity epilogue.  The
chains use ``sets`` sets of intermediate buffers in turn, so the library can
run that many chains at once on its lanes (accumulating into private copies
of the image that it adds up in lane order: deterministic for a given call);
``sets=1`` gives the plain call-order sum.  With ``method="auto"`` (the
paper's default) each distance takes the AS or DI method by the critical
distance; DI tables are built within each call, once per (wavelength,
distance), or, with ``cache_tables=True``, once for the life of the object
(py x px complex per table: 32 MiB each at 2048^2 complex64, so 16 GiB for
the 502 tables of a 251-wavelength 4f image)."""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import Optics, _capi, _dtype_code, _real_dtype, _stream, make_job, resolve_method, transfer_table


class FourF:
    def __init__(self, f: float, dy: float, dx: float, *, pad: int = 2, method: str = "auto",
                 y0: float = 0.0, x0: float = 0.0, padded=None, cache_tables: bool = False):
        self.f = float(f)
        self.dy, self.dx = float(dy), float(dx)
        self.pad = pad
        self.method = method
        self.y0, self.x0 = float(y0), float(x0)
        self.padded = padded
        self.cache_tables = cache_tables
        self._tables = {}

    def _table(self, u: torch.Tensor, opt: Optics):
        """The cached DI table of this distance and wavelength (None when the
        method is not DI or caching is off)."""
        if not self.cache_tables:
            return None
        ny, nx = u.shape[-2], u.shape[-1]
        if resolve_method(opt, ny, nx) != "di":
            return None
        key = (opt.wavelength, opt.z, ny, nx, u.dtype, u.device)
        if key not in self._tables:
            self._tables[key] = transfer_table(opt, ny, nx, dtype=u.dtype, device=u.device)
        return self._tables[key]

    def _opt(self, wavelength: float, z: float) -> Optics:
        return Optics(dy=self.dy, dx=self.dx, wavelength=float(wavelength), z=z, method=self.method,
                      pad=self.pad, y0=self.y0, x0=self.x0, padded=self.padded)

    def image(self, u: torch.Tensor, wavelengths: Sequence[float], weights: Sequence[float], *,
              out: Optional[torch.Tensor] = None, sets: int = 4) -> torch.Tensor:
        """Weighted incoherent image of fields ``u`` ([B, ny, nx] or [ny, nx],
        complex) at z = 4f: returns (or accumulates into ``out``) the real
        intensity of the shape of u."""
        if len(wavelengths) != len(weights):
            raise ValueError("one weight per wavelength")
        if out is None:
            out = torch.zeros(u.shape, dtype=_real_dtype(u), device=u.device)
        sets = max(1, min(int(sets), len(wavelengths)))
        tmp = [(torch.empty_like(u), torch.empty_like(u)) for _ in range(sets)]
        jobs = []
        for k, (lam, w) in enumerate(zip(wavelengths, weights)):
            t1, t2 = tmp[k % sets]
            of, o2 = self._opt(lam, self.f), self._opt(lam, 2 * self.f)
            hf, h2 = self._table(u, of), self._table(u, o2)
            jobs.append(make_job(u, of, out=t1, tf_table=hf))
            jobs.append(make_job(t1, o2, out=t2, lens_f=self.f, tf_table=h2))
            jobs.append(make_job(t2, of, lens_f=self.f, epi=_capi.TO_EPI_INTENSITY, epi_out=out,
                                 epi_scale=float(w), tf_table=hf))
        if jobs:
            _capi.propagate(jobs, _dtype_code(u), _stream(u))
        return out
