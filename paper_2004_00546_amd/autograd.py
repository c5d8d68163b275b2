"""torch.autograd.Function over the C ABI.

``ParaexpLoss.apply(a, problem)`` returns J(a) for one instance; its backward
returns dJ/da.  Forward: ``pxp_assemble`` (controls -> forcing pattern or
initial state), ``paraexp_direct`` (for Burgers the serial march that keeps
its checkpoints in a workspace of this forward's own, saved for its
backward, paper section 3.5),
``pxp_cost`` (J and lambda_T).  Backward: ``paraexp_adjoint`` from lambda_T
(Krylov pieces, or the Magnus chain for Burgers) and
``pxp_reduce_gradient`` (eqs. paramupdate, initupdate); the incoming
gradient gJ scales the result.  Every step runs in libparaexp.so; torch only
holds the device buffers.  Terminal cost only: an integral-cost problem is
refused by ``pxp_cost`` (its cost needs the trajectory, which the one-call
gradient forms), and the forward raises.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib, api


class Problem:
    """Device-resident description of one instance and its workspace."""

    def __init__(self, inst: dict, device="cuda:0", **prob_kw):
        self.inst = inst
        self.device = torch.device(device)
        self.p = api.make_problem(inst, **prob_kw)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.basis = torch.tensor(np.asarray(inst["basis"], dtype=np.float64), **f64)
        n = self.basis.shape[1]
        self.q0 = torch.tensor(np.asarray(inst.get("q0", np.zeros(n)), dtype=np.float64), **f64)
        self.u_tgt = torch.tensor(np.asarray(inst["u_tgt"], dtype=np.float64), **f64)
        self.forcing = inst["control"] == "forcing"
        self.nbytes = max(_lib.pxp_workspace_size([self.p]), 256)
        self.ws = self.new_workspace()
        self.n = n
        # the Burgers direct march leaves its checkpoints in the workspace
        # for the adjoint: each forward then gets a workspace of its own,
        # saved with the autograd context, so a second forward before the
        # first backward cannot overwrite the trajectory that backward reads
        self.ckpt_in_ws = inst["op"] == "burgers1d"

    def new_workspace(self):
        ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        _lib.pxp_workspace_init(ws)
        return ws


class ParaexpLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a: torch.Tensor, prob: Problem):
        a = a.detach().to(prob.device, torch.float64).contiguous()
        f64 = dict(dtype=torch.float64, device=prob.device)
        field = torch.empty(prob.n, **f64)
        if prob.forcing:
            _lib.pxp_assemble([prob.p], a, prob.basis, None, field)
            q0, F = prob.q0, field
        else:
            _lib.pxp_assemble([prob.p], a, prob.basis, prob.q0, field)
            q0, F = field, None
        qT = torch.empty(prob.n, **f64)
        ws = prob.new_workspace() if prob.ckpt_in_ws else prob.ws
        _lib.paraexp_direct([prob.p], q0, F, qT, ws)
        J = torch.empty(1, **f64)
        lamT = torch.empty(prob.n, **f64)
        _lib.pxp_cost([prob.p], qT, prob.u_tgt, a, J, lamT)
        code, _ = _lib.pxp_device_status(ws)
        if code != _lib.PXP_OK:
            raise _lib.PxpError(code, "paraexp_direct (device status)")
        ctx.prob = prob
        ctx.ws = ws
        ctx.save_for_backward(a, lamT)
        return J[0]

    @staticmethod
    def backward(ctx, gJ):
        a, lamT = ctx.saved_tensors
        prob = ctx.prob
        f64 = dict(dtype=torch.float64, device=prob.device)
        v = torch.empty(prob.n, **f64)
        ws = ctx.ws
        if prob.forcing:
            _lib.paraexp_adjoint([prob.p], lamT, None, v, ws)
        else:
            _lib.paraexp_adjoint([prob.p], lamT, v, None, ws)
        code, _ = _lib.pxp_device_status(ws)
        if code != _lib.PXP_OK:
            raise _lib.PxpError(code, "paraexp_adjoint (device status)")
        grad = torch.empty_like(a)
        _lib.pxp_reduce_gradient([prob.p], prob.basis, v, a, grad)
        return gJ * grad, None


def paraexp_loss(a: torch.Tensor, prob: Problem) -> torch.Tensor:
    return ParaexpLoss.apply(a, prob)
