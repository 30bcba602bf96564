"""Real even-order spherical harmonics, Signal2SH and SH2Signal in FP64.

Test infrastructure only (see the package docstring).

Conventions (the paper names the basis by citation only, Sec. 1 / Sec. 2.2):
* Only even orders l = 0, 2, ..., L (antipodally symmetric diffusion signal);
  K = (L+1)(L+2)/2 coefficients, index j = l(l+1)/2 + m, m = -l..l.
* m < 0: sqrt(2) N_l^|m| P_l^|m|(cos t) cos(|m| p);  m = 0: N_l^0 P_l(cos t);
  m > 0: sqrt(2) N_l^m P_l^m(cos t) sin(m p);
  N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), P_l^m with the Condon-Shortley
  phase (-1)^m.
"""
from __future__ import annotations

import math

import numpy as np


def n_coeffs(sh_order: int) -> int:
    """K = (L+1)(L+2)/2 for even L."""
    if sh_order < 0 or sh_order % 2:
        raise ValueError("sh_order must be even and >= 0")
    return (sh_order + 1) * (sh_order + 2) // 2


def degree_order(sh_order: int) -> tuple[np.ndarray, np.ndarray]:
    """(l_j, m_j) for j = 0..K-1 in the index order l(l+1)/2 + m."""
    ls, ms = [], []
    for l in range(0, sh_order + 1, 2):
        for m in range(-l, l + 1):
            ls.append(l)
            ms.append(m)
    return np.array(ls), np.array(ms)


def cart_to_sphere(g: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Unit-normalise the rows of g; return polar angle theta and azimuth phi."""
    g = np.asarray(g, dtype=np.float64)
    g = g / np.linalg.norm(g, axis=1, keepdims=True)
    theta = np.arccos(np.clip(g[:, 2], -1.0, 1.0))
    phi = np.arctan2(g[:, 1], g[:, 0])
    return theta, phi


def assoc_legendre(lmax: int, x: np.ndarray) -> dict:
    """P_l^m(x) for 0 <= m <= l <= lmax, Condon-Shortley phase included,
    by the textbook upward recurrences:
      P_m^m = (-1)^m (2m-1)!! (1-x^2)^(m/2)
      P_{m+1}^m = x (2m+1) P_m^m
      (l-m) P_l^m = (2l-1) x P_{l-1}^m - (l+m-1) P_{l-2}^m"""
    x = np.asarray(x, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = {}
    pmm = np.ones_like(x)
    for m in range(0, lmax + 1):
        if m > 0:
            pmm = -(2 * m - 1) * s * pmm
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = x * (2 * m + 1) * pmm
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * x * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def sh_norm(l: int, m: int) -> float:
    """N_l^m = sqrt((2l+1)/(4 pi) * (l-m)!/(l+m)!) with exact integer factorials."""
    return math.sqrt((2 * l + 1) / (4.0 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def real_sh_basis(sh_order: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """B[i, j] = Y_j(theta_i, phi_i), shape (n, K)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    P = assoc_legendre(sh_order, np.cos(theta))
    ls, ms = degree_order(sh_order)
    B = np.empty((theta.shape[0], ls.shape[0]))
    for j, (l, m) in enumerate(zip(ls, ms)):
        am = abs(int(m))
        base = sh_norm(int(l), am) * P[(int(l), am)]
        if m < 0:
            B[:, j] = math.sqrt(2.0) * base * np.cos(am * phi)
        elif m == 0:
            B[:, j] = base
        else:
            B[:, j] = math.sqrt(2.0) * base * np.sin(am * phi)
    return B


def basis_at(sh_order: int, g: np.ndarray) -> np.ndarray:
    theta, phi = cart_to_sphere(g)
    return real_sh_basis(sh_order, theta, phi)


def lb_penalty(sh_order: int) -> np.ndarray:
    """Diagonal of the Laplace-Beltrami penalty, l^2 (l+1)^2 per coefficient."""
    ls, _ = degree_order(sh_order)
    return (ls * (ls + 1)).astype(np.float64) ** 2


def fit_matrix(B: np.ndarray, sh_order: int, lb_lambda: float) -> np.ndarray:
    """P = (B^T B + lambda L)^{-1} B^T, the regularised least-squares fit
    (Signal2SH's lb_lambda parameter, Sec. 2.2), shape (K, n)."""
    L = np.diag(lb_penalty(sh_order))
    return np.linalg.solve(B.T @ B + lb_lambda * L, B.T)


def has_fit(B: np.ndarray, sh_order: int, lb_lambda: float) -> bool:
    """Whether the regularised normal matrix B^T B + lambda L has full rank
    K, i.e. the least-squares fit of Signal2SH exists.  SH2Signal needs only
    the basis (evaluation on any N resampled directions, Sec. 2.2), so a
    table with fewer directions than coefficients at lambda = 0 is fine for
    it."""
    A = B.T @ B + lb_lambda * np.diag(lb_penalty(sh_order))
    return int(np.linalg.matrix_rank(A)) == A.shape[0]


def group_shells(bvals: np.ndarray, b0_max: float = 50.0, rel_tol: float = 0.05):
    """Drop b0 volumes (b < b0_max) and group the rest into shells.

    A volume joins the first shell whose centre is within rel_tol of its b;
    shells are ordered by increasing centre b; within a shell volumes keep
    their table order.  Returns (list of index arrays, list of shell b)."""
    bvals = np.asarray(bvals, dtype=np.float64)
    centres: list[float] = []
    members: list[list[int]] = []
    for i, b in enumerate(bvals):
        if b < b0_max:
            continue
        for k, c in enumerate(centres):
            if abs(b - c) <= rel_tol * c:
                members[k].append(i)
                centres[k] = float(np.mean(bvals[members[k]]))
                break
        else:
            centres.append(float(b))
            members.append([i])
    order = np.argsort(centres, kind="stable")
    return [np.array(members[k], dtype=np.int64) for k in order], [centres[k] for k in order]


class SHPlan:
    """Per-shell basis and fit matrices of one gradient table."""

    def __init__(self, bvecs, bvals, sh_order, lb_lambda=0.006, b0_max=50.0, rel_tol=0.05):
        self.sh_order = sh_order
        self.K = n_coeffs(sh_order)
        self.lb_lambda = lb_lambda
        self.shell_idx, self.shell_b = group_shells(bvals, b0_max, rel_tol)
        bvecs = np.asarray(bvecs, dtype=np.float64)
        self.B = [basis_at(sh_order, bvecs[idx]) for idx in self.shell_idx]
        # P_s exists only where the fit does; without it the plan evaluates
        # only (sh2signal and its adjoint) and signal2sh raises
        self.has_fit = all(has_fit(B, sh_order, lb_lambda) for B in self.B)
        self.P = [fit_matrix(B, sh_order, lb_lambda) for B in self.B] if self.has_fit else None
        self.dirs = [idx.shape[0] for idx in self.shell_idx]

    @property
    def n_shells(self) -> int:
        return len(self.B)


def signal2sh(plan: SHPlan, x: np.ndarray) -> np.ndarray:
    """c[v, s, :] = P_s x[v, s-block] for b0-normalised signal x of shape
    (V, sum N_s) in shell-major order; returns (V, S, K)."""
    if plan.P is None:
        raise np.linalg.LinAlgError("the plan's regularised normal matrix is singular: no fit")
    V = x.shape[0]
    out = np.empty((V, plan.n_shells, plan.K))
    off = 0
    for s, P in enumerate(plan.P):
        n = P.shape[1]
        out[:, s, :] = x[:, off:off + n] @ P.T
        off += n
    return out


def sh2signal(plan: SHPlan, c: np.ndarray) -> np.ndarray:
    """x[v, s-block] = B_s c[v, s, :]; c of shape (V, S, K) -> (V, sum N_s)."""
    return np.concatenate([c[:, s, :] @ B.T for s, B in enumerate(plan.B)], axis=1)


def signal2sh_adjoint(plan: SHPlan, dc: np.ndarray) -> np.ndarray:
    """dx = P_s^T dc per shell (gradient of Signal2SH w.r.t. its input)."""
    if plan.P is None:
        raise np.linalg.LinAlgError("the plan's regularised normal matrix is singular: no fit")
    return np.concatenate([dc[:, s, :] @ P for s, P in enumerate(plan.P)], axis=1)


def sh2signal_adjoint(plan: SHPlan, dx: np.ndarray) -> np.ndarray:
    """dc = B_s^T dx per shell (gradient of SH2Signal w.r.t. its input)."""
    V = dx.shape[0]
    out = np.empty((V, plan.n_shells, plan.K))
    off = 0
    for s, B in enumerate(plan.B):
        n = B.shape[0]
        out[:, s, :] = dx[:, off:off + n] @ B
        off += n
    return out


def normalize_b0(raw: np.ndarray, bvals: np.ndarray, plan: SHPlan, b0_max: float = 50.0) -> np.ndarray:
    """The normalisation Signal2SH requires of its input (Sec. 2.2): every
    diffusion-weighted volume divided by the voxel's mean over the b=0
    volumes, returned in the plan's shell-major order.  raw: (V, n_total) in
    acquisition order."""
    b0 = np.asarray(bvals) < b0_max
    mean_b0 = raw[:, b0].mean(axis=1, keepdims=True)
    order = np.concatenate(plan.shell_idx)
    return raw[:, order] / mean_b0
