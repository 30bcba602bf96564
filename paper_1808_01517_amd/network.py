"""Signal2SH -> LSC ... LSC -> SH2Signal networks driven by the library.

`LSCNetwork` owns its plans, float32 master weights, Adam moments and every
activation / gradient buffer, and runs forward, q-space MSE, backward and
the Adam update as library kernels on the current stream.

Recomputation: the output of a layer k listed in `recompute` (any layer but
the last) is not kept for the backward pass.  All such outputs of one shape
share a single buffer, which later layers overwrite; the backward pass
recomputes the output from the stored layer input right before the next
layer's adjoint consumes it.  The kernels are deterministic, so gradients
are bitwise identical to the run that keeps every activation.

When the output table allows it, the loss step runs as one fused pass
(SH2Signal, MSE and the SH2Signal adjoint).  With `bf16_activations` in the
BF16 folded form, hidden activations and their gradients are stored in
bfloat16, which leaves every value the contractions see unchanged.  With
`relu_bits` each hidden ReLU's backward mask is read from
one bit per element that the forward writes beside the activation; the
results are bitwise those of the activation mask.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import (DEFAULT_FORM, LSCPlan, SHPlan, Workspace, adam_step, lib, lsc_bwd, lsc_fwd, lsc_workspace_bytes,
               mse_fwd_bwd, relu_bits_like, sh2signal_bwd, sh2signal_fwd, sh2signal_mse_fwd_bwd,
               sh2signal_mse_supported, signal2sh_bwd, signal2sh_fwd)


@dataclass
class LayerSpec:
    C: int
    O: int
    sh_order_in: int
    sh_order_out: int
    relu: bool


class LSCNetwork:
    def __init__(self, plan_in: SHPlan, plan_out: SHPlan, sampled_gradients, specs, kernel_sizes, angular_distance,
                 lb_lambda=0.006, weights=None, precision="fp32", form=DEFAULT_FORM, recompute=(), device="cuda:0",
                 max_batch=8192, bf16_activations=False, relu_bits=False):
        self.plan_in, self.plan_out = plan_in, plan_out
        self.specs = list(specs)
        self.precision, self.form = precision, form
        # hidden activations (and their gradients) stored in bfloat16: BF16
        # folded form, rows of a multiple of 8 entries; the contractions round
        # them to bfloat16 on load anyway
        self.bf16_activations = bool(bf16_activations) and precision == "bf16" and form == "folded"
        # a hidden ReLU's backward mask as one bit per element, written by the
        # forward beside the activation (folded form); off by default: at
        # batches of a few thousand voxels the activations stay in cache and
        # the extra epilogue work outweighs the saved reads
        self.relu_bits = bool(relu_bits) and form == "folded"
        self.recompute = set(int(k) for k in recompute)
        if any(k < 0 or k >= len(specs) - 1 for k in self.recompute):
            raise ValueError("only layers before the last can be recomputed")
        if any(k + 1 in self.recompute for k in self.recompute):
            raise ValueError("two consecutive layers cannot both be recomputed (their outputs would share a buffer)")
        self.dev = torch.device(device)
        self.plans = [LSCPlan(sampled_gradients, s.sh_order_in, s.sh_order_out, kernel_sizes, angular_distance,
                              lb_lambda) for s in self.specs]
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.W, self.b = [], []
        for k, (s, p) in enumerate(zip(self.specs, self.plans)):
            if weights is not None:
                Wk, bk = weights[k]
                self.W.append(torch.as_tensor(np.asarray(Wk, dtype=np.float32)).to(self.dev).contiguous())
                self.b.append(torch.as_tensor(np.asarray(bk, dtype=np.float32)).to(self.dev).contiguous())
            else:
                bound = 1.0 / np.sqrt(s.C * p.T)
                self.W.append(torch.empty((s.O, s.C, p.T), **f32).uniform_(-bound, bound))
                self.b.append(torch.empty((s.O,), **f32).uniform_(-bound, bound))
        self.dW = [torch.zeros_like(w) for w in self.W]
        self.db = [torch.zeros_like(b) for b in self.b]
        self.m = [torch.zeros_like(w) for w in self.W] + [torch.zeros_like(b) for b in self.b]
        self.v = [torch.zeros_like(w) for w in self.W] + [torch.zeros_like(b) for b in self.b]
        self.t = 0
        ws = max(lsc_workspace_bytes(p, s.C, s.O, max_batch, precision, form) for s, p in zip(self.specs, self.plans))
        self.ws = Workspace(ws, self.dev)
        self._alloc(max_batch)

    # ---------------------------------------------------------- buffers
    def _alloc(self, V):
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.cap = V
        S, K = self.plan_in.n_shells, self.plan_in.K
        self.acts = [torch.empty((V, S, K), **f32)]
        shared = {}
        n = len(self.specs)
        for k, (s, p) in enumerate(zip(self.specs, self.plans)):
            shape = (V, s.O, p.K_out)
            half = self.bf16_activations and k < n - 1 and (s.O * p.K_out) % 8 == 0
            dt = torch.bfloat16 if half else torch.float32
            if k in self.recompute:
                if (shape, dt) not in shared:
                    shared[(shape, dt)] = torch.empty(shape, dtype=dt, device=self.dev)
                self.acts.append(shared[(shape, dt)])
            else:
                self.acts.append(torch.empty(shape, dtype=dt, device=self.dev))
        self.grads = [torch.empty(a.shape, dtype=a.dtype, device=self.dev) for a in self.acts]
        # bits[k] describes acts[k]; shared exactly as the activations are
        self.bits = [None] * (n + 1)
        shared_bits = {}
        for k, (s, p) in enumerate(zip(self.specs, self.plans)):
            if self.relu_bits and s.relu and k < n - 1 and (s.O * p.K_out) % 16 == 0:
                a = self.acts[k + 1]
                key = id(a)
                if key not in shared_bits:
                    shared_bits[key] = relu_bits_like(a)
                self.bits[k + 1] = shared_bits[key]
        self.xhat = torch.empty((V, self.plan_out.n_dw), **f32)
        self.dxhat = torch.empty_like(self.xhat)
        self.loss = torch.empty((), **f32)
        self.mse_ws = torch.empty(lib().dlm_mse_workspace_bytes(V * self.plan_out.n_dw), dtype=torch.uint8,
                                  device=self.dev)
        # the fused loss head (SH2Signal, MSE and its adjoint in one pass)
        # when the output table allows it; dxhat is then not materialised
        self.fused_head = sh2signal_mse_supported(self.plan_out)
        if self.fused_head:
            self.head_ws = torch.empty(lib().dlm_sh2signal_mse_workspace_bytes(self.plan_out.handle, V),
                                       dtype=torch.uint8, device=self.dev)

    def parameters(self):
        return self.W + self.b

    def state_dict(self):
        return {"W": [w.detach().cpu() for w in self.W], "b": [b.detach().cpu() for b in self.b],
                "m": [x.detach().cpu() for x in self.m], "v": [x.detach().cpu() for x in self.v], "t": self.t}

    def load_state_dict(self, sd):
        for dst, src in zip(self.W + self.b + self.m + self.v, sd["W"] + sd["b"] + sd["m"] + sd["v"]):
            dst.copy_(src.to(self.dev))
        self.t = int(sd["t"])

    # ------------------------------------------------------------ passes
    def _layer_fwd(self, k, V):
        s, p = self.specs[k], self.plans[k]
        bits = self.bits[k + 1]
        lsc_fwd(p, self.acts[k][:V], self.W[k], self.b[k], relu=s.relu, out=self.acts[k + 1][:V],
                precision=self.precision, workspace=self.ws, form=self.form,
                relu_bits=None if bits is None else bits[:V])

    def _forward_sh(self, x: torch.Tensor) -> int:
        V = x.shape[0]
        if V > self.cap:
            self._alloc(V)
        signal2sh_fwd(self.plan_in, x, out=self.acts[0][:V], precision=self.precision)
        for k in range(len(self.specs)):
            self._layer_fwd(k, V)
        return V

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        V = self._forward_sh(x)
        sh2signal_fwd(self.plan_out, self.acts[-1][:V], out=self.xhat[:V], precision=self.precision)
        return self.xhat[:V]

    def backward(self, V: int, need_input_grad=False):
        """Gradients of the last loss w.r.t. every weight (and the input when
        asked), from the q-space gradient in `dxhat`."""
        sh2signal_bwd(self.plan_out, self.dxhat[:V], out=self.grads[-1][:V], precision=self.precision)
        return self._backward_layers(V, need_input_grad)

    def _backward_layers(self, V: int, need_input_grad: bool):
        n = len(self.specs)
        for k in range(n - 1, -1, -1):
            s, p = self.specs[k], self.plans[k]
            if (k - 1) in self.recompute:
                self._layer_fwd(k - 1, V)  # this layer's input was not kept: recompute it
            # A ReLU between layers k-1 and k is applied by layer k's adjoint as it
            # writes the input gradient (the mask is read once); only a ReLU on the
            # last layer's output would be masked by its own adjoint.
            relu_in = k > 0 and self.specs[k - 1].relu
            relu_out = s.relu and k == n - 1
            lsc_bwd(p, self.acts[k][:V], self.W[k], self.grads[k + 1][:V],
                    a_out=self.acts[k + 1][:V] if relu_out else None, relu=relu_out, relu_in=relu_in,
                    need_input_grad=(k > 0 or need_input_grad), precision=self.precision, workspace=self.ws,
                    outs=(self.grads[k][:V], self.dW[k], self.db[k]), form=self.form,
                    relu_bits=self.bits[k][:V] if relu_in and self.bits[k] is not None else None)
        if need_input_grad:
            return signal2sh_bwd(self.plan_in, self.grads[0][:V], precision=self.precision)
        return None

    def loss_and_grads(self, x: torch.Tensor, target: torch.Tensor, need_input_grad=False):
        """Forward, q-space MSE against `target` and backward; the prediction
        is left in `xhat`."""
        if not self.fused_head:
            V = x.shape[0]
            self.forward(x)
            mse_fwd_bwd(self.xhat[:V], target, outs=(self.loss, self.dxhat[:V], self.mse_ws))
            return self.loss, self.backward(V, need_input_grad)
        V = self._forward_sh(x)
        sh2signal_mse_fwd_bwd(self.plan_out, self.acts[-1][:V], target, precision=self.precision,
                              outs=(self.loss, self.grads[-1][:V], self.head_ws), xhat_out=self.xhat[:V])
        return self.loss, self._backward_layers(V, need_input_grad)

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        for p, g, m, v in zip(self.W + self.b, self.dW + self.db, self.m, self.v):
            adam_step(p, g, m, v, self.t, lr, beta1, beta2, eps)

    def train_step(self, x, target, lr=1e-3):
        loss, _ = self.loss_and_grads(x, target)
        self.adam(lr)
        return loss
