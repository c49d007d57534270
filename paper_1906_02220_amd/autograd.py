"""torch.autograd bindings of the library's hand-written CTMRG gradient.

``purification_objective(A, B, gamma, chi, sweeps, op, w_log_kappa,
w_expect)`` returns, as a 0-d tensor, w_log_kappa ln(kappa) + w_expect <op>
after `sweeps` sweeps (ctm_grad_purification); calling ``backward()`` on
anything computed from it propagates the library's dL/dA and dL/dB, scaled by
the incoming gradient.  ``tensor_objective`` is the same for a site tensor
(ctm_grad_tensor).  The forward call computes the gradient as well (one
library call does both).  Tensors in GPU memory go to the library as device
pointers (ctm_grad_purification_dev, ctm_grad_tensor_dev) and their
gradients come back in GPU memory; other tensors are exchanged as host FP64
arrays.  This module only marshals arguments.
"""
import numpy as np
import torch

from . import ctm


def _host(t):
    return t.detach().to("cpu", torch.float64).contiguous().numpy()


def _lib_input(t):
    """A GPU tensor goes to the library as is (device-pointer path), any
    other as a host FP64 array."""
    return t.detach() if t.is_cuda else _host(t)


def _as_grad(g, like):
    g = g if torch.is_tensor(g) else torch.from_numpy(g)
    return g.to(like.device, like.dtype)


class _PurificationObjective(torch.autograd.Function):
    @staticmethod
    def forward(fctx, A, B, context, gamma, chi, sweeps, op, w_log_kappa, w_expect,
                checkpoint_every, opts):
        lk, ex, gA, gB, info = ctm.grad_purification(
            context, _lib_input(A), _lib_input(B), gamma, chi, sweeps, op=op,
            w_log_kappa=w_log_kappa, w_expect=w_expect, checkpoint_every=checkpoint_every, **opts)
        fctx.save_for_backward(_as_grad(gA, A), _as_grad(gB, B))
        fctx.info = info
        return A.new_tensor(w_log_kappa * lk + w_expect * ex)

    @staticmethod
    def backward(fctx, grad_out):
        gA, gB = fctx.saved_tensors
        return (grad_out * gA, grad_out * gB) + (None,) * 9


class _TensorObjective(torch.autograd.Function):
    @staticmethod
    def forward(fctx, a, context, chi, sweeps, a_imp, w_log_kappa, w_expect, checkpoint_every,
                opts):
        lk, ex, ga, info = ctm.grad_tensor(
            context, _lib_input(a), chi, sweeps, a_imp=a_imp, w_log_kappa=w_log_kappa,
            w_expect=w_expect, checkpoint_every=checkpoint_every, **opts)
        fctx.save_for_backward(_as_grad(ga, a))
        fctx.info = info
        return a.new_tensor(w_log_kappa * lk + w_expect * ex)

    @staticmethod
    def backward(fctx, grad_out):
        (ga,) = fctx.saved_tensors
        return (grad_out * ga,) + (None,) * 8


def purification_objective(context, A, B, gamma, chi, sweeps, op=None, w_log_kappa=1.0,
                           w_expect=0.0, checkpoint_every=0, **opts):
    """Differentiable w_log_kappa ln(kappa) + w_expect <op> of the purification
    (A, B) (torch tensors of shape (2, 2, Dx, Dy, Dz))."""
    opn = None if op is None else np.ascontiguousarray(
        op.detach().cpu().numpy() if torch.is_tensor(op) else op, dtype=np.float64)
    return _PurificationObjective.apply(A, B, context, gamma, chi, sweeps, opn, float(w_log_kappa),
                                        float(w_expect), int(checkpoint_every), opts)


def tensor_objective(context, a, chi, sweeps, a_imp=None, w_log_kappa=1.0, w_expect=0.0,
                     checkpoint_every=0, **opts):
    """Differentiable w_log_kappa ln(kappa) + w_expect <E, a_imp> / <E, a> of a
    site tensor a (torch tensor of shape (d, d, d, d)); a_imp is held fixed."""
    ai = None if a_imp is None else np.ascontiguousarray(
        a_imp.detach().cpu().numpy() if torch.is_tensor(a_imp) else a_imp, dtype=np.float64)
    return _TensorObjective.apply(a, context, chi, sweeps, ai, float(w_log_kappa),
                                  float(w_expect), int(checkpoint_every), opts)
