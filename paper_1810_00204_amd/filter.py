"""Differentiable belief filter on the GPU: the negative log-likelihood of
logged runs under the Bayes filter, with its hand-written adjoint
(qv_filter_nll_grad) behind a torch.autograd.Function, so that the slip
logits and the sensor flip logits can be fitted to logs."""
from __future__ import annotations

import numpy as np

from . import binding as B


class FilterProblem:
    """Device copies of the map, the runs and the start belief."""

    def __init__(self, prob, acts, obs, b0=None, device="cuda", ckpt_every=10):
        import torch
        self.m = B.DeviceModel(prob, device)
        self.acts = torch.as_tensor(np.ascontiguousarray(acts, np.int32)).to(device)
        self.obs = torch.as_tensor(np.ascontiguousarray(obs, np.int32)).to(device)
        self.ntraj, self.T = self.acts.shape
        b0 = prob.b0 if b0 is None else b0
        b0 = np.ascontiguousarray(b0, np.float32)
        self.b0_per_traj = 1 if b0.ndim == 2 else 0
        self.b0 = torch.as_tensor(b0).to(device)
        self.ckpt_every = int(ckpt_every)
        nb = B.qv_filter_workspace_bytes(self.m, self.ntraj, self.T, self.ckpt_every)
        if nb == 0:
            raise B.QvError(B.QV_ERR_UNSUPPORTED, "qv_filter_workspace_bytes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        self.device = device

    def run(self, theta, phi, grad=True, check=True, stream=None):
        """Returns (nll per run [ntraj], d sum(nll)/d theta [A, 9] or None,
        d sum(nll)/d phi [4] or None)."""
        import torch
        theta = theta.detach().to(self.device, torch.float32).contiguous()
        phi = phi.detach().to(self.device, torch.float32).contiguous()
        nll = torch.empty(self.ntraj, dtype=torch.float32, device=self.device)
        gs = torch.empty_like(theta) if grad else None
        gf = torch.empty_like(phi) if grad else None
        st = B.qv_filter_nll_grad(self.m, theta, phi, self.ntraj, self.T, self.b0,
                                  self.b0_per_traj, self.acts, self.obs, self.ckpt_every, nll,
                                  gs, gf, 1 if check else 0, self.ws, stream)
        B.check(st, "qv_filter_nll_grad")
        return nll, gs, gf


class FilterNLL:
    """``FilterNLL.apply(theta, phi, problem)`` -> total NLL (a scalar tensor);
    its backward returns the adjoint gradients computed in the same call."""

    _fn = None

    @classmethod
    def apply(cls, theta, phi, problem):
        if cls._fn is None:
            cls._fn = _make_function()
        return cls._fn.apply(theta, phi, problem)


def _make_function():
    import torch

    class _FilterNLL(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, phi, problem):
            nll, gs, gf = problem.run(theta, phi, grad=True)
            # gradients on the parameters' own device and dtype
            ctx.save_for_backward(gs.to(theta.device, theta.dtype), gf.to(phi.device, phi.dtype))
            return nll.sum().to(theta.device, theta.dtype)

        @staticmethod
        def backward(ctx, grad_out):
            gs, gf = ctx.saved_tensors
            return grad_out * gs, grad_out * gf, None

    return _FilterNLL
