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
    def forward(ctx, v, op):
        nt_rec = op.time.nt // op.time.rec_every
        d = torch.empty(op.batch.data_size(nt_rec), dtype=torch.float32, device=v.device)
        vd = v.detach().contiguous()
        fwi.fwi_forward(op.batch, op.time, vd, d, op.ws)
        op._calls += 1
        op._holds = op._calls  # the workspace now holds the state of this forward
        ctx.save_for_backward(vd)
        ctx.op, ctx.token = op, op._calls
        return d

    @staticmethod
    def backward(ctx, grad_d):
        (v,) = ctx.saved_tensors
        op = ctx.op
        if op._holds != ctx.token:
            # a later forward on the same operator replaced this one's checkpoints (or
            # imaging operands): recompute them from the saved model first
            nt_rec = op.time.nt // op.time.rec_every
            scratch = torch.empty(op.batch.data_size(nt_rec), dtype=torch.float32, device=v.device)
            fwi.fwi_forward(op.batch, op.time, v, scratch, op.ws)
            op._holds = ctx.token
            op.replays += 1
        grad = torch.empty_like(v)
        fwi.fwi_adjoint(op.batch, op.time, v, grad_d.contiguous().float(), None, grad, None, op.ws)
        return grad, None


class FwiOperator:
    """d = F(v) for a fixed batch geometry and time axis, differentiable in v.

    ``ckpt_every`` (time axis) selects the schedule: 0 keeps every imaging operand, K >= 1
    keeps checkpoints every K steps and recomputes each segment in the backward pass.
    The workspace is allocated once and reused.  It holds the state of the most recent
    forward; a backward through an earlier output (two forwards in one loss, a probe
    taken before backward, gradcheck) first re-runs that output's forward from its saved
    model (counted in ``replays``), so every backward sees its own forward's state.
    """

    def __init__(self, batch: fwi.Batch, time, device="cuda"):
        self.batch, self.time = batch, time
        fwi.fwi_check(batch, time)
        self.ws = fwi.alloc_workspace(batch, time, device)
        self._calls = 0      # forwards run so far
        self._holds = 0      # which of them the workspace holds
        self.replays = 0     # forwards re-run by a backward

    def __call__(self, v: torch.Tensor) -> torch.Tensor:
        return _FwiData.apply(v, self)

    def split(self, d: torch.Tensor):
        """Per-simulation views [nt_rec][nrec] of a flat data tensor."""
        nt_rec = self.time.nt // self.time.rec_every
        off = self.batch.data_off(nt_rec)
        return [d[off[s]:off[s + 1]].view(nt_rec, int(self.batch.nrec[s])) for s in range(self.batch.nsim)]
