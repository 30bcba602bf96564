"""Local spherical convolution (LSC) in FP64, step by step as Sec. 2.3 states it.

Test infrastructure only (see the package docstring).

Steps, in the paper's order (Sec. 2.3 and its Fig. 4 workflow):
1. Kernel: a centre point plus n_r points on ring r at angular distance
   rho_r from the centre (cyclic kernel, Fig. 3), stored as a vector of
   T = 1 + sum n_r weights per (output, input) channel pair.
2. Resampling: for each of the m sampled directions g_i the kernel points
   around g_i are evaluated from the input SH coefficients (SH
   interpolation), giving an m x T neighbourhood matrix per channel.
3. Row dot: each row is multiplied point-wise with the kernel vector and
   summed (a cross-correlation, no flip), summed over input channels
   (multi-b-value extension, Sec. 2.3.1), plus the output channel's bias.
4. Refit: the m values of each output channel are fitted back to SH of
   order sh_order_out with the Laplace-Beltrami regularised fit (the
   layer's lb_lambda / sh_order_out / sampled_gradients parameters).

Readings where the paper is silent (all recorded in the design notes):
rings r = 1..R sit at rho_r = r * alpha / R with alpha = angular_distance
(the outer ring) and kernel_sizes = [n_1..n_R]; the local frame at g is
e_theta = (cos t cos p, cos t sin p, -sin t), e_phi = (-sin p, cos p, 0);
ring point b sits at azimuth psi_b = 2 pi b / n_r from e_theta toward
e_phi, the same origin on every ring; tap order is centre, ring 1, ring 2...
"""
from __future__ import annotations

import numpy as np

from . import sh


def local_frame(g: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Unit g and the tangent vectors e_theta, e_phi at g (rows)."""
    g = np.asarray(g, dtype=np.float64)
    g = g / np.linalg.norm(g, axis=1, keepdims=True)
    theta, phi = sh.cart_to_sphere(g)
    e_t = np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi), -np.sin(theta)], axis=1)
    e_p = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], axis=1)
    return g, e_t, e_p


def ring_radii(kernel_sizes, angular_distance: float) -> np.ndarray:
    R = len(kernel_sizes)
    return np.array([(r + 1) * angular_distance / R for r in range(R)], dtype=np.float64)


def kernel_points(sampled_gradients: np.ndarray, kernel_sizes, angular_distance: float) -> np.ndarray:
    """Cyclic-kernel points around every sampled direction, shape (m, T, 3)."""
    g, e_t, e_p = local_frame(sampled_gradients)
    rho = ring_radii(kernel_sizes, angular_distance)
    pts = [g[:, None, :]]
    for r, n_r in enumerate(kernel_sizes):
        psi = 2.0 * np.pi * np.arange(n_r) / n_r
        tang = np.cos(psi)[None, :, None] * e_t[:, None, :] + np.sin(psi)[None, :, None] * e_p[:, None, :]
        pts.append(np.cos(rho[r]) * g[:, None, :] + np.sin(rho[r]) * tang)
    return np.concatenate(pts, axis=1)


class LSCPlan:
    """Tables of one LSC layer geometry.

    B_nb : (m*T, K_in)  SH basis at every kernel point (resampling)
    P_m  : (K_out, m)   regularised fit on the sampled directions (refit)"""

    def __init__(self, sampled_gradients, sh_order_in, sh_order_out, kernel_sizes, angular_distance,
                 lb_lambda=0.006):
        self.g = np.asarray(sampled_gradients, dtype=np.float64)
        self.m = self.g.shape[0]
        self.kernel_sizes = tuple(int(k) for k in kernel_sizes)
        self.T = 1 + sum(self.kernel_sizes)
        self.sh_order_in = sh_order_in
        self.sh_order_out = sh_order_out
        self.K_in = sh.n_coeffs(sh_order_in)
        self.K_out = sh.n_coeffs(sh_order_out)
        self.alpha = float(angular_distance)
        self.lb_lambda = lb_lambda
        self.points = kernel_points(self.g, self.kernel_sizes, self.alpha)
        self.B_nb = sh.basis_at(sh_order_in, self.points.reshape(-1, 3))
        self.B_m = sh.basis_at(sh_order_out, self.g)
        self.P_m = sh.fit_matrix(self.B_m, sh_order_out, lb_lambda)


def resample(plan: LSCPlan, a: np.ndarray) -> np.ndarray:
    """Neighbourhood matrices X[v, c, i, t] = sum_j B_nb[(i,t), j] a[v, c, j]."""
    V, C, _ = a.shape
    return (a @ plan.B_nb.T).reshape(V, C, plan.m, plan.T)


def kernel_dot(X: np.ndarray, W: np.ndarray, bias) -> np.ndarray:
    """y[v, o, i] = bias[o] + sum_c sum_t W[o, c, t] X[v, c, i, t]."""
    y = np.einsum("oct,vcit->voi", W, X)
    if bias is not None:
        y = y + np.asarray(bias)[None, :, None]
    return y


def refit(plan: LSCPlan, y: np.ndarray) -> np.ndarray:
    """a_out[v, o, :] = P_m y[v, o, :]."""
    return y @ plan.P_m.T


def lsc_forward(plan: LSCPlan, a: np.ndarray, W: np.ndarray, bias=None, relu: bool = False):
    """Full layer.  Returns (a_out, z) with z the pre-activation SH output."""
    X = resample(plan, a)
    y = kernel_dot(X, W, bias)
    z = refit(plan, y)
    return (np.maximum(z, 0.0) if relu else z), z


def lsc_backward(plan: LSCPlan, a: np.ndarray, W: np.ndarray, z, da_out: np.ndarray, relu: bool = False):
    """Adjoint of lsc_forward.  Returns (da_in, dW, dbias).

    ReLU'(z) = [z > 0]; dy = P_m^T da; dW[o,c,t] = sum_{v,i} dy X;
    db[o] = sum_{v,i} dy; dX = sum_o W dy; da = B_nb^T dX."""
    g = da_out * (z > 0.0) if relu else da_out
    dy = g @ plan.P_m                                    # (V, O, m)
    X = resample(plan, a)
    dW = np.einsum("voi,vcit->oct", dy, X)
    db = dy.sum(axis=(0, 2))
    dX = np.einsum("oct,voi->vcit", W, dy)
    V, C = a.shape[:2]
    da = dX.reshape(V, C, plan.m * plan.T) @ plan.B_nb
    return da, dW, db
