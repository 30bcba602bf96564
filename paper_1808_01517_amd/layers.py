"""torch.autograd Functions and nn.Modules over the library's kernels.

The modules mirror the paper's layer API (Sec. 2.2 and 2.3 parameter
lists): Signal2SH(sh_order, gradients, lb_lambda), SH2Signal(sh_order,
gradients) and LocalSphericalConvolution(shells_in, shells_out,
sampled_gradients, sh_order_in, sh_order_out, kernel_sizes,
angular_distance, lb_lambda) with its kernel at `lsc.sconv.weight`
[O, C, 1, n+1] and `lsc.sconv.bias` [O].  Tensors are either the paper's
5-D layout subjects x (#shells * #dirs or #channels * K) x H x W x D, or
voxel-major [V, ...]; 5-D inputs are permuted to voxel-major for the
library and back.  Forward and backward both run in the library's HIP
kernels; PyTorch only holds the memory.
"""
from __future__ import annotations

import numpy as np
import torch
from torch import nn

from . import (DEFAULT_FORM, LSCPlan, SHPlan, lsc_bwd, lsc_fwd, sh2signal_bwd, sh2signal_fwd, signal2sh_bwd,
               signal2sh_fwd)


def _to_voxels(t: torch.Tensor, channels: int):
    """[B, ch, H, W, D] -> ([B*H*W*D, ch], restore-info); 2-D tensors pass through."""
    if t.dim() == 5:
        B, ch, H, W, D = t.shape
        if ch != channels:
            raise ValueError(f"expected {channels} channels, got {ch}")
        return t.permute(0, 2, 3, 4, 1).reshape(-1, ch).contiguous(), (B, H, W, D)
    return t.reshape(t.shape[0], -1).contiguous(), None


def _from_voxels(v: torch.Tensor, info):
    if info is None:
        return v
    B, H, W, D = info
    return v.reshape(B, H, W, D, -1).permute(0, 4, 1, 2, 3).contiguous()


class _Signal2SHFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan, precision):
        ctx.plan, ctx.precision = plan, precision
        return signal2sh_fwd(plan, x, precision=precision)

    @staticmethod
    def backward(ctx, dc):
        return signal2sh_bwd(ctx.plan, dc.contiguous(), precision=ctx.precision), None, None


class _SH2SignalFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, plan, precision):
        ctx.plan, ctx.precision = plan, precision
        return sh2signal_fwd(plan, c, precision=precision)

    @staticmethod
    def backward(ctx, dx):
        return sh2signal_bwd(ctx.plan, dx.contiguous(), precision=ctx.precision), None, None


class _LSCFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, W, b, plan, relu, precision, form):
        out = lsc_fwd(plan, a, W, b, relu=relu, precision=precision, form=form)
        ctx.plan, ctx.relu, ctx.precision, ctx.form = plan, relu, precision, form
        ctx.has_bias = b is not None
        ctx.save_for_backward(a, W, out if relu else None)
        return out

    @staticmethod
    def backward(ctx, g):
        a, W, out = ctx.saved_tensors
        need_a, need_W, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        da, dW, db = lsc_bwd(ctx.plan, a, W, g.contiguous(), a_out=out, relu=ctx.relu, need_input_grad=need_a,
                             need_weight_grad=need_W, need_bias_grad=need_b and ctx.has_bias,
                             precision=ctx.precision, form=ctx.form)
        if dW is not None:
            dW = dW.view_as(W)
        return da, dW, db, None, None, None, None


def _table(gradients, bvals):
    g = np.asarray(gradients, dtype=np.float64).reshape(-1, 3)
    if bvals is None:  # a single shell: every direction is diffusion weighted
        bvals = np.full(g.shape[0], 1000.0)
    return g, np.asarray(bvals, dtype=np.float64).reshape(-1)


class Signal2SH(nn.Module):
    """Signal -> SH coefficients (Sec. 2.2).  Input must be b0-normalised."""

    def __init__(self, sh_order: int, gradients, bvals=None, lb_lambda: float = 0.006, precision="fp32"):
        super().__init__()
        g, b = _table(gradients, bvals)
        self.plan = SHPlan(g, b, sh_order, lb_lambda)
        self.precision = precision

    def forward(self, x):
        v, info = _to_voxels(x, self.plan.n_dw)
        c = _Signal2SHFn.apply(v, self.plan, self.precision)
        return _from_voxels(c.reshape(c.shape[0], -1), info) if info else c


class SH2Signal(nn.Module):
    """SH coefficients -> signal on the given (resampled) directions (Sec. 2.2)."""

    def __init__(self, sh_order: int, gradients, bvals=None, precision="fp32"):
        super().__init__()
        g, b = _table(gradients, bvals)
        # evaluation needs the basis only: any table works, also one with
        # fewer directions than coefficients (the plan then has no fit)
        self.plan = SHPlan(g, b, sh_order, 0.0)
        self.precision = precision

    def forward(self, c):
        p = self.plan
        v, info = _to_voxels(c, p.n_shells * p.K)
        x = _SH2SignalFn.apply(v.reshape(-1, p.n_shells, p.K), p, self.precision)
        return _from_voxels(x, info) if info else x


class LocalSphericalConvolution(nn.Module):
    """Local spherical convolution with cyclic kernels (Sec. 2.3, 2.3.1).

    Weight `sconv.weight` [shells_out, shells_in, 1, T] and bias
    `sconv.bias` [shells_out], T = 1 + sum(kernel_sizes)."""

    def __init__(self, shells_in: int, shells_out: int, sampled_gradients, sh_order_in: int, sh_order_out: int,
                 kernel_sizes, angular_distance: float = np.pi / 5, lb_lambda: float = 0.006, relu: bool = False,
                 precision="fp32", form=DEFAULT_FORM):
        super().__init__()
        self.plan = LSCPlan(sampled_gradients, sh_order_in, sh_order_out, kernel_sizes, angular_distance, lb_lambda)
        self.C, self.O = int(shells_in), int(shells_out)
        T = self.plan.T
        self.sconv = nn.Module()
        bound = 1.0 / np.sqrt(self.C * T)
        self.sconv.weight = nn.Parameter(torch.empty(self.O, self.C, 1, T).uniform_(-bound, bound))
        self.sconv.bias = nn.Parameter(torch.empty(self.O).uniform_(-bound, bound))
        self.relu = relu
        self.precision = precision
        self.form = form

    def forward(self, a):
        p = self.plan
        v, info = _to_voxels(a, self.C * p.K_in)
        W = self.sconv.weight
        b = self.sconv.bias
        out = _LSCFn.apply(v.reshape(-1, self.C, p.K_in), W.reshape(self.O, self.C, -1), b, p, self.relu,
                           self.precision, self.form)
        return _from_voxels(out.reshape(out.shape[0], -1), info) if info else out
