"""torch.autograd.Function wrappers of the library's operators.

* ``response(s, problem, masked=True)``: x = M R s (sec. 2, eq. ddecomp; spin-2 rotation of
  appendix C), whose backward is the hand-written adjoint kernel (forward FFT, inverse
  rotation, mask): ds = 2 R^T M dx on the free modes.
* ``chi2(s, theta, problem)``: chi^2(s; theta) of eq. eq_chi for one field [c][n][n/2+1] or a
  batch [B][c][n][n/2+1]; its backward gives d chi^2 / ds = 4 g (eq. eq_cost, per stored
  coefficient) and d chi^2 / d theta_b = -2 E_b (the prior term's derivative; E_b of eq. el
  evaluated with the prior at theta), both computed by the library (wf_chi2_grad and
  wf_chi2_dtheta, which also contracts with the upstream gradient).

Gradients follow PyTorch's complex convention (d/dRe + i d/dIm for a real loss), which is
the library's.  theta is a CPU float64 tensor (the C-ABI takes band amplitudes on the host).
"""
from __future__ import annotations

import numpy as np
import torch

from . import WF_ADJ_GRAD, WF_MASK, wf_adjoint, wf_chi2_dtheta, wf_chi2_grad, wf_forward

__all__ = ["ResponseOp", "Chi2Op", "response", "chi2"]


class ResponseOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, problem, masked):
        ctx.problem = problem
        ctx.masked = bool(masked)
        return wf_forward(problem, s.contiguous(), flags=WF_MASK if masked else 0)

    @staticmethod
    def backward(ctx, gx):
        flags = WF_ADJ_GRAD | (WF_MASK if ctx.masked else 0)
        gs = wf_adjoint(ctx.problem, gx.contiguous().to(ctx.problem.rdtype), flags=flags)
        return gs, None, None


class Chi2Op(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, theta, problem):
        th = theta.detach().to("cpu", torch.float64).numpy()
        p = problem.with_theta(th)
        s = s.contiguous()
        chi, g = wf_chi2_grad(p, s)
        ctx.p = p
        ctx.theta_device = theta.device
        ctx.save_for_backward(s, g)
        return torch.as_tensor(np.asarray(chi, np.float64), device=s.device)

    @staticmethod
    def backward(ctx, gout):
        s, g = ctx.saved_tensors
        batched = s.dim() == 4
        go = gout.to(torch.float64)
        gs = None
        if ctx.needs_input_grad[0]:
            w = go.reshape((-1, 1, 1, 1) if batched else ()).to(g.real.dtype)
            gs = g * w
        gth = None
        if ctx.needs_input_grad[1]:
            gow = go.detach().cpu().numpy().reshape(-1)
            gth = torch.as_tensor(wf_chi2_dtheta(ctx.p, s, gow), dtype=torch.float64, device=ctx.theta_device)
        return gs, gth, None


def response(s, problem, masked: bool = True):
    return ResponseOp.apply(s, problem, masked)


def chi2(s, theta, problem):
    return Chi2Op.apply(s, theta, problem)
