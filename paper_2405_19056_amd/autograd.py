"""torch.autograd integration of the library's forward, L1 loss and backward.

    y = GlassNetFunction.apply(net, gbuf, layers, scene, w)
    loss = L1Function.apply(net, y, target)
    loss.backward()          # w.grad <- the library's hand-written backward

Argument marshalling only: the forward, the loss and its gradient and the
backward all run in libglassnet's kernels (Sec. 3.5: the four networks are
trained jointly, end to end; the L1 term of the loss).  Gradients with
respect to the buffers are not produced (they are rasterizer outputs).
"""
from __future__ import annotations

import torch

from .glassnet import GlassNet


class GlassNetFunction(torch.autograd.Function):
    """y = GlassNet(w) on the handle `net`.  w is saved for the backward and
    uploaded again there, so the gradient is taken at the weights of this
    forward even if the handle's weights changed in between (torch's version
    counter also rejects an in-place edit of w before the backward)."""

    @staticmethod
    def forward(ctx, net: GlassNet, gbuf, layers, scene, w):
        net.set_weights(w.detach())
        out = net.forward(gbuf, layers, scene)
        ctx.net = net
        ctx.save_for_backward(gbuf, layers, scene, w)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        gbuf, layers, scene, w = ctx.saved_tensors
        ctx.net.set_weights(w.detach())
        gw = ctx.net.backward(gbuf, layers, scene, grad_out.contiguous())
        return None, None, None, None, gw


class L1Function(torch.autograd.Function):
    """mean |y - t| and its subgradient, both from the library's loss kernel;
    the upstream gradient scales the subgradient on the device."""

    @staticmethod
    def forward(ctx, net: GlassNet, y, target):
        y, target = y.detach().contiguous(), target.contiguous()
        loss = net.l1_loss(y, target)
        ctx.net = net
        ctx.save_for_backward(y, target)
        return loss

    @staticmethod
    def backward(ctx, g):
        y, target = ctx.saved_tensors
        grad = torch.empty_like(y)
        scratch = torch.empty((), dtype=torch.float32, device=y.device)
        ctx.net.l1_loss(y, target, loss=scratch, grad_out=grad,
                        grad_scale=g.detach().to(torch.float32).contiguous())
        return None, grad, None


def train_step(net: GlassNet, gbuf, layers, scene, target, w, grad_w=None, stream=None):
    """One step without autograd: forward with weights w, L1 loss, backward.

    Returns (loss tensor, grad_w tensor); everything stays on the device.
    """
    net.set_weights(w, stream=stream)
    y = net.forward(gbuf, layers, scene, stream=stream)
    dy = torch.empty_like(y)
    loss = net.l1_loss(y, target, grad_out=dy, stream=stream)
    gw = net.backward(gbuf, layers, scene, dy, grad_w=grad_w, stream=stream)
    return loss, gw


def train_step_adam(net: GlassNet, gbuf, layers, scene, target, state, step, lr=1e-4,
                    weight_decay=1e-4, grad_w=None, dssim=True, stream=None):
    """One training step of Sec. 3.5 / 4 on the handle's own weights: forward,
    the L1 + DSSIM loss (dssim=False: L1 alone), backward, and an Adam step
    (weight decay as an L2 term) applied on the device.  `state` is
    net.adam_state(); `step` counts from 1.  Returns (losses, grad_w): losses
    is a device tensor [L1, DSSIM]."""
    y = net.forward(gbuf, layers, scene, stream=stream)
    dy = torch.empty_like(y)
    losses = torch.zeros(2, dtype=torch.float32, device=y.device)
    net.l1_loss(y, target, loss=losses[0], grad_out=dy, stream=stream)
    if dssim:
        net.dssim_loss(y, target, loss=losses[1], grad_out=dy, accumulate=True, stream=stream)
    gw = net.backward(gbuf, layers, scene, dy, grad_w=grad_w, stream=stream)
    net.adam_step(gw, state, step, lr=lr, weight_decay=weight_decay, stream=stream)
    return losses, gw


def train_step_sr(net: GlassNet, sr_w, state, lowres, gbuf_hi, target, step, lr=1e-4,
                  weight_decay=0.0, grad_w=None, dssim=True, stream=None):
    """One training step of the x2 super-sampling network on its own (Sec. 4.1
    trains it apart from GlassNet) with the loss of Sec. 3.5: forward, L1 +
    DSSIM (dssim=False: L1 alone), its weight gradient and an Adam step on the
    caller's weight vector sr_w.  `state` is a zeroed device tensor of
    2 x sr_w.numel() floats; `step` counts from 1.  Returns (losses, grad_w):
    losses is a device tensor [L1, DSSIM]."""
    y = net.sr_forward(sr_w, lowres, gbuf_hi, stream=stream)
    dy = torch.empty_like(y)
    losses = torch.zeros(2, dtype=torch.float32, device=y.device)
    net.l1_loss(y, target, loss=losses[0], grad_out=dy, stream=stream)
    if dssim:
        net.dssim_loss(y, target, loss=losses[1], grad_out=dy, accumulate=True, stream=stream)
    gw = net.sr_backward(sr_w, lowres, gbuf_hi, dy, grad_w=grad_w, stream=stream)
    net.adam_update(sr_w, gw, state, step, lr=lr, weight_decay=weight_decay, stream=stream)
    return losses, gw

