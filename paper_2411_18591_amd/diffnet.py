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
``plain=True``, through its unfused plain form)."""
from __future__ import annotations

import torch

from . import Optics, propagate, propagate_backward, propagate_loss


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

    def forward(self, plain: bool = False) -> torch.Tensor:
        """u_1 .. u_L and the loss (device float64 scalar); dL/du_L in gbuf[0]."""
        self.loss.zero_()
        for l in range(self.L - 1):
            propagate(self.u[l], self.opt, out=self.u[l + 1], phase=self.masks[l], plain=plain)
        propagate_loss(self.u[self.L - 1], self.opt, kind="mse", ref=self.target, scale=self.scale,
                       out=self.u[self.L], grad=self.gbuf[0], loss=self.loss, phase=self.masks[self.L - 1],
                       plain=plain)
        return self.loss

    def backward(self, plain: bool = False) -> torch.Tensor:
        """dL/dphi_l for every mask into gmask (overwritten)."""
        self.gmask.zero_()
        cur = 0
        for l in range(self.L - 1, -1, -1):
            nxt = 1 - cur
            propagate_backward(self.gbuf[cur], self.opt, saved_in=self.u[l], grad_phase=self.gmask[l],
                               phase=self.masks[l], want_grad_in=l > 0, grad_in=self.gbuf[nxt], plain=plain)
            cur = nxt
        return self.gmask

    def step(self, plain: bool = False):
        self.forward(plain)
        self.backward(plain)
