"""Autograd form: the library's forward solve and hand-written adjoint behind
``torch.autograd.Function``.

``forward`` runs ``fwi_forward`` (one launch per time step over every simulation of the
batch, checkpoints or imaging operands kept in the workspace) and returns the predicted
data.  ``backward`` receives dL/dd and runs ``fwi_adjoint`` with that residual, which
returns J^T (dL/dd) summed over each sample's simulations -- the adjoint-state gradient
stated after Eq. 5 of the paper, for any differentiable loss built on the data.
"""
from __future__ import annotations

import torch

from . import fwi


class _FwiData(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, batch, time, ws):
        nt_rec = time.nt // time.rec_every
        d = torch.empty(batch.data_size(nt_rec), dtype=torch.float32, device=v.device)
        vd = v.detach().contiguous()
        fwi.fwi_forward(batch, time, vd, d, ws)
        ctx.save_for_backward(vd)
        ctx.batch, ctx.time, ctx.ws = batch, time, ws
        return d

    @staticmethod
    def backward(ctx, grad_d):
        (v,) = ctx.saved_tensors
        grad = torch.empty_like(v)
        fwi.fwi_adjoint(ctx.batch, ctx.time, v, grad_d.contiguous().float(), None, grad, None, ctx.ws)
        return grad, None, None, None


class FwiOperator:
    """d = F(v) for a fixed batch geometry and time axis, differentiable in v.

    ``ckpt_every`` (time axis) selects the schedule: 0 keeps every imaging operand, K >= 1
    keeps checkpoints every K steps and recomputes each segment in the backward pass.
    The workspace is allocated once and reused; one forward must be followed by its
    backward before the next forward (the workspace holds that forward's state).
    """

    def __init__(self, batch: fwi.Batch, time, device="cuda"):
        self.batch, self.time = batch, time
        fwi.fwi_check(batch, time)
        self.ws = fwi.alloc_workspace(batch, time, device)

    def __call__(self, v: torch.Tensor) -> torch.Tensor:
        return _FwiData.apply(v, self.batch, self.time, self.ws)

    def split(self, d: torch.Tensor):
        """Per-simulation views [nt_rec][nrec] of a flat data tensor."""
        nt_rec = self.time.nt // self.time.rec_every
        off = self.batch.data_off(nt_rec)
        return [d[off[s]:off[s + 1]].view(nt_rec, int(self.batch.nrec[s])) for s in range(self.batch.nsim)]
