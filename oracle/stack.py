"""Layer stacks, q-space MSE loss and whole forward + backward passes (FP64).

Test infrastructure only (see the package docstring).

A stack is Signal2SH -> LSC -> ReLU -> ... -> LSC -> SH2Signal, the way the
LSC example of Sec. 2.3 chains s2sh, lsc and sh2s; the SH output of every
LSC except the last goes through a ReLU.  The loss is computed back in
q-space (Sec. 1 motivates going back to the spherical surface space for the
loss): mean squared error over all voxels and directions.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lsc, sh


def mse(pred: np.ndarray, target: np.ndarray) -> tuple[float, np.ndarray]:
    """loss = mean((pred - target)^2); dloss/dpred = 2 (pred - target) / numel."""
    diff = pred - target
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


def relative_mse(pred: np.ndarray, target: np.ndarray, eps: float) -> tuple[float, np.ndarray]:
    """A relative q-space loss (Sec. 1: relative losses become usable once the
    prediction is back in q-space): each error is measured against the
    target's magnitude, loss = mean(((pred - target) / (|target| + eps))^2);
    dloss/dpred = 2 (pred - target) / ((|target| + eps)^2 numel)."""
    w = 1.0 / (np.abs(target) + eps)
    r = (pred - target) * w
    return float(np.mean(r * r)), 2.0 * r * w / r.size


@dataclass
class Layer:
    plan: lsc.LSCPlan
    W: np.ndarray
    b: np.ndarray
    relu: bool


class Stack:
    """Signal2SH(plan_in) -> LSC layers -> SH2Signal(plan_out)."""

    def __init__(self, plan_in: sh.SHPlan, layers: list, plan_out: sh.SHPlan):
        self.plan_in = plan_in
        self.layers = layers
        self.plan_out = plan_out

    def forward(self, x: np.ndarray):
        """Returns (xhat, cache) where cache holds every layer input and pre-activation."""
        c = sh.signal2sh(self.plan_in, x)
        acts, zs = [c], []
        a = c
        for L in self.layers:
            a, z = lsc.lsc_forward(L.plan, a, L.W, L.b, L.relu)
            acts.append(a)
            zs.append(z)
        xhat = sh.sh2signal(self.plan_out, a)
        return xhat, (acts, zs)

    def backward(self, cache, dxhat: np.ndarray):
        """Returns (dx, [dW], [db]) for upstream gradient dxhat."""
        acts, zs = cache
        g = sh.sh2signal_adjoint(self.plan_out, dxhat)
        dWs, dbs = [None] * len(self.layers), [None] * len(self.layers)
        for k in range(len(self.layers) - 1, -1, -1):
            L = self.layers[k]
            g, dWs[k], dbs[k] = lsc.lsc_backward(L.plan, acts[k], L.W, zs[k], g, L.relu)
        dx = sh.signal2sh_adjoint(self.plan_in, g)
        return dx, dWs, dbs

    def loss_and_grads(self, x: np.ndarray, target: np.ndarray):
        xhat, cache = self.forward(x)
        loss, dxhat = mse(xhat, target)
        dx, dWs, dbs = self.backward(cache, dxhat)
        return loss, xhat, dx, dWs, dbs
