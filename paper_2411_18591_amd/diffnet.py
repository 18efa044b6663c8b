"""Training step of a diffractive network: phase masks separated by free
space, as in the paper's training example (section "Gradient-based
optimization"), generalised to L layers and a batch of fields:

    u_l = P_z(exp(i phi_l) u_{l-1}),  l = 1..L,
    loss = scale * sum (|u_L|^2 - T)^2   (MSE, T shared by the batch),

and the backward pass to every mask.  The forward pass keeps each layer's
input (needed by the mask gradients: recomputation of the modulated field,
no stored spectra); the loss and dL/du_L are fused into the last
propagation; the backward pass runs the adjoint propagations back to the
first mask, two gradient buffers alternating.

Every propagation goes through the library's fused kernels (or, with
``plain=True``, through its unfused plain form).  When the optics resolve to
direct integration (method "di", or "auto" beyond the critical distance),
the DI transfer table is built once here and carried by every job, since
the geometry does not change between steps."""
from __future__ import annotations

import torch

from . import Optics, _capi, propagate_backward_jobs, propagate_jobs, resolve_method, transfer_table


class DiffractiveNet:
    def __init__(self, u0: torch.Tensor, masks: torch.Tensor, target: torch.Tensor, opt: Optics,
                 scale: float | None = None):
        if u0.dim() != 3 or masks.dim() != 3 or masks.shape[1:] != u0.shape[1:]:
            raise ValueError("u0 is [B, N, N'] and masks [L, N, N']")
        self.opt = opt
        self.L = masks.shape[0]
        self.masks = masks
        self.target = target
        self.scale = 1.0 / u0.numel() if scale is None else float(scale)
        self.u = [u0] + [torch.empty_like(u0) for _ in range(self.L)]
        self.gmask = torch.zeros_like(masks)
        self.gbuf = [torch.empty_like(u0) for _ in range(2)]
        self.loss = torch.zeros((), dtype=torch.float64, device=u0.device)
        ny, nx = u0.shape[1:]
        self.tf_table = None
        if resolve_method(opt, ny, nx) == "di":
            self.tf_table = transfer_table(opt, ny, nx, dtype=u0.dtype, device=u0.device)

    def _element(self, l: int) -> dict:
        el = {"phase": self.masks[l]}
        if self.tf_table is not None:
            el["tf_table"] = self.tf_table
        return el

    def forward(self, plain: bool = False) -> torch.Tensor:
        """u_1 .. u_L and the loss (device float64 scalar); dL/du_L in gbuf[0].
        All layers go to the library in one call: it recognises the chain
        (each layer reads the previous one's output) and runs it chunk by
        chunk with fused layer boundaries."""
        self.loss.zero_()
        L = self.L
        elements = [self._element(l) for l in range(L)]
        elements[-1].update(epi=_capi.TO_EPI_MSE, epi_ref=self.target, epi_scale=self.scale,
                            epi_grad=self.gbuf[0], epi_loss=self.loss)
        propagate_jobs(self.u[:L], [self.opt] * L, outs=self.u[1:], elements=elements, plain=plain)
        return self.loss

    def backward(self, plain: bool = False) -> torch.Tensor:
        """dL/dphi_l for every mask into gmask (overwritten), in one call
        (layers L-1 .. 0, the gradient buffers alternating; their contents
        afterwards are unspecified: they only link the layers)."""
        self.gmask.zero_()
        L = self.L
        layers = list(range(L - 1, -1, -1))
        gout = [self.gbuf[k % 2] for k in range(L)]
        gin = [self.gbuf[(k + 1) % 2] if l > 0 else None for k, l in enumerate(layers)]
        # the intermediate gradients only link consecutive layers of the chain
        propagate_backward_jobs(gout, [self.opt] * L, saved_ins=[self.u[l] for l in layers], grad_ins=gin,
                                grad_phases=[self.gmask[l] for l in layers],
                                elements=[self._element(l) for l in layers], plain=plain,
                                transient=[g is not None for g in gin])
        return self.gmask

    def step(self, plain: bool = False):
        self.forward(plain)
        self.backward(plain)
