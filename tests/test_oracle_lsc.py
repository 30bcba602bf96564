"""Pins of the FP64 oracle's local spherical convolution (Sec. 2.3).

Isotropic kernels have a frame-free closed form (Funk-Hecke); the centre
tap, the bias and a permutation of the sampled directions have exact
consequences; and small cases are recomputed by nested loops from points
built by explicit rotation matrices and scipy's harmonics.
"""
import math
import os

import numpy as np
import pytest
import scipy.special as sps

from datagen import fibonacci_hemisphere, perturb_directions, rng_for
from oracle import lsc, sh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, name)) if ln.strip() and not ln.startswith("#")]
    return {int(l): float(h) for l, h in rows}


def _P(l, x):
    return np.polynomial.legendre.legval(x, [0] * l + [1])


def _isotropic_W(w0, wr, kernel_sizes):
    """Kernel vector(s) with w0 at the centre and wr[r] at every point of ring r."""
    w0 = np.asarray(w0, dtype=float)
    taps = [w0[..., None]]
    for r, n in enumerate(kernel_sizes):
        taps.append(np.repeat(np.asarray(wr[r], dtype=float)[..., None], n, axis=-1))
    return np.concatenate(taps, axis=-1)


def _dirs(n, seed=0, perturb=2.0):
    return perturb_directions(fibonacci_hemisphere(n), perturb, rng_for(77, 1, seed))


def test_geometry_points_on_rings():
    g = _dirs(30)
    ks, alpha = (6, 8), np.deg2rad(30)
    pts = lsc.kernel_points(g, ks, alpha)
    assert pts.shape == (30, 15, 3)
    assert np.abs(np.linalg.norm(pts, axis=2) - 1).max() < 1e-15
    gn = g / np.linalg.norm(g, axis=1, keepdims=True)
    assert np.abs(pts[:, 0] - gn).max() < 1e-15
    ang = np.arccos(np.clip(np.einsum("itk,ik->it", pts, gn), -1, 1))
    assert np.abs(ang[:, 1:7] - np.deg2rad(15)).max() < 1e-7   # arccos near 1 loses digits
    assert np.abs(ang[:, 7:] - np.deg2rad(30)).max() < 1e-7
    cosang = np.einsum("itk,ik->it", pts, gn)
    assert np.abs(cosang[:, 1:7] - math.cos(np.deg2rad(15))).max() < 1e-14
    # equispaced azimuths: consecutive tangent components differ by 2 pi / n
    _, et, ep = lsc.local_frame(g)
    for sl, n in ((slice(1, 7), 6), (slice(7, 15), 8)):
        q = pts[:, sl]
        psi = np.arctan2(np.einsum("itk,ik->it", q, ep), np.einsum("itk,ik->it", q, et))
        d = np.mod(np.diff(psi, axis=1), 2 * np.pi)
        assert np.abs(d - 2 * np.pi / n).max() < 1e-12
        assert np.abs(psi[:, 0]).max() < 1e-12
    F = np.stack([gn, et, ep], axis=2)
    assert np.abs(np.einsum("ika,ikb->iab", F, F) - np.eye(3)).max() < 1e-15


def test_funk_hecke_paper_moving_average():
    # Sec. 2.3 example: n = 5, alpha = pi/5, all weights 1/6, bias 0, order 4.
    gold = _golden("funk_hecke_moving_average.txt")
    alpha = np.pi / 5
    for l in (0, 2, 4):
        assert abs(gold[l] - (1 / 6 + 5 / 6 * _P(l, math.cos(alpha)))) < 1e-15
    plan = lsc.LSCPlan(_dirs(30), 4, 4, [5], alpha, lb_lambda=0.0)
    W = np.full((1, 1, 6), 1.0 / 6.0)
    a = np.random.default_rng(0).standard_normal((6, 1, 15))
    out, _ = lsc.lsc_forward(plan, a, W, np.zeros(1))
    ls, _ = sh.degree_order(4)
    h = np.array([gold[int(l)] for l in ls])
    assert np.abs(out - a * h).max() < 1e-12


def test_funk_hecke_c1_uniform_kernel():
    gold = _golden("funk_hecke_c1_uniform.txt")
    r1, r2 = np.deg2rad(15), np.deg2rad(30)
    for l in (0, 2, 4):
        assert abs(gold[l] - (1 + 6 * _P(l, math.cos(r1)) + 6 * _P(l, math.cos(r2))) / 13) < 1e-15
    plan = lsc.LSCPlan(_dirs(30, 1), 4, 4, [6, 6], np.deg2rad(30), lb_lambda=0.0)
    W = np.full((1, 1, 13), 1.0 / 13.0)
    a = np.random.default_rng(1).standard_normal((4, 1, 15))
    out, _ = lsc.lsc_forward(plan, a, W, None)
    ls, _ = sh.degree_order(4)
    assert np.abs(out - a * np.array([gold[int(l)] for l in ls])).max() < 1e-12


def test_funk_hecke_multichannel_order8():
    # isotropic kernel per (o, c) pair, 9 points per ring so that order 8 has no
    # azimuthal aliasing: a_out[o, lm] = sum_c h_{o,c,l} a_c[lm].
    ks, alpha = (9, 9), np.deg2rad(30)
    C, O = 3, 4
    rng = np.random.default_rng(2)
    w0, w1, w2 = rng.standard_normal((O, C)), rng.standard_normal((O, C)), rng.standard_normal((O, C))
    W = _isotropic_W(w0, [w1, w2], ks)
    plan = lsc.LSCPlan(fibonacci_hemisphere(90), 8, 8, ks, alpha, lb_lambda=0.0)
    a = rng.standard_normal((5, C, 45))
    out, _ = lsc.lsc_forward(plan, a, W, None)
    ls, _ = sh.degree_order(8)
    rho = lsc.ring_radii(ks, alpha)
    H = w0[..., None] + 9 * w1[..., None] * _P_all(ls, rho[0]) + 9 * w2[..., None] * _P_all(ls, rho[1])
    expect = np.einsum("ocj,vcj->voj", H, a)
    assert np.abs(out - expect).max() < 1e-11


def _P_all(ls, rho):
    return np.array([_P(int(l), math.cos(rho)) for l in ls])[None, None, :]


def test_center_only_kernel_is_channel_mixing():
    C, O = 3, 5
    rng = np.random.default_rng(3)
    W = np.zeros((O, C, 17))
    W[:, :, 0] = rng.standard_normal((O, C))
    plan = lsc.LSCPlan(_dirs(90, 2), 8, 8, [8, 8], np.deg2rad(30), lb_lambda=0.0)
    a = rng.standard_normal((4, C, 45))
    out, _ = lsc.lsc_forward(plan, a, W, None)
    assert np.abs(out - np.einsum("oc,vcj->voj", W[:, :, 0], a)).max() < 1e-11


@pytest.mark.parametrize("lam", [0.0, 0.006])
def test_bias_only_touches_l0(lam):
    C, O = 2, 3
    rng = np.random.default_rng(4)
    plan = lsc.LSCPlan(_dirs(90, 3), 8, 8, [8, 8], np.deg2rad(30), lb_lambda=lam)
    a = rng.standard_normal((4, C, 45))
    W = rng.standard_normal((O, C, 17))
    b = rng.standard_normal(O)
    with_b, _ = lsc.lsc_forward(plan, a, W, b)
    without, _ = lsc.lsc_forward(plan, a, W, None)
    d = with_b - without
    assert np.abs(d[:, :, 0] - b[None, :] * math.sqrt(4 * math.pi)).max() < 1e-11
    assert np.abs(d[:, :, 1:]).max() < 1e-11


def test_permuting_sampled_directions():
    rng = np.random.default_rng(5)
    g = _dirs(90, 4)
    perm = rng.permutation(90)
    ks, alpha = (8, 8), np.deg2rad(30)
    p1 = lsc.LSCPlan(g, 8, 8, ks, alpha, 0.006)
    p2 = lsc.LSCPlan(g[perm], 8, 8, ks, alpha, 0.006)
    a = rng.standard_normal((3, 3, 45))
    W = rng.standard_normal((4, 3, 17))
    b = rng.standard_normal(4)
    y1 = lsc.kernel_dot(lsc.resample(p1, a), W, b)
    y2 = lsc.kernel_dot(lsc.resample(p2, a), W, b)
    assert np.abs(y2 - y1[:, :, perm]).max() < 1e-12
    o1, _ = lsc.lsc_forward(p1, a, W, b)
    o2, _ = lsc.lsc_forward(p2, a, W, b)
    assert np.abs(o1 - o2).max() < 1e-11


def _rot_points(g, ks, alpha):
    """Kernel points by rotating north-pole rings: R = Rz(phi) Ry(theta) maps
    e_z -> g, e_x -> e_theta, e_y -> e_phi."""
    out = []
    R_ = len(ks)
    for gi in g:
        gi = gi / np.linalg.norm(gi)
        th, ph = math.acos(gi[2]), math.atan2(gi[1], gi[0])
        Ry = np.array([[math.cos(th), 0, math.sin(th)], [0, 1, 0], [-math.sin(th), 0, math.cos(th)]])
        Rz = np.array([[math.cos(ph), -math.sin(ph), 0], [math.sin(ph), math.cos(ph), 0], [0, 0, 1]])
        R = Rz @ Ry
        row = [R @ np.array([0.0, 0.0, 1.0])]
        for r, n in enumerate(ks):
            rho = (r + 1) * alpha / R_
            for b in range(n):
                psi = 2 * math.pi * b / n
                row.append(R @ np.array([math.sin(rho) * math.cos(psi), math.sin(rho) * math.sin(psi), math.cos(rho)]))
        out.append(row)
    return out


def _real_Y(L, p):
    th = math.acos(max(-1.0, min(1.0, p[2])))
    ph = math.atan2(p[1], p[0])
    vals = []
    for l in range(0, L + 1, 2):
        for m in range(-l, l + 1):
            Y = complex(sps.sph_harm_y(l, abs(m), th, ph))
            vals.append(math.sqrt(2) * Y.real if m < 0 else (Y.real if m == 0 else math.sqrt(2) * Y.imag))
    return vals


def _solve(A, rhs):
    n = len(A)
    M = [A[r][:] + [rhs[r]] for r in range(n)]
    for col in range(n):
        piv = max(range(col, n), key=lambda r: abs(M[r][col]))
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col:
                f = M[r][col] / M[col][col]
                M[r] = [M[r][k] - f * M[col][k] for k in range(n + 1)]
    return [M[r][n] / M[r][r] for r in range(n)]


@pytest.mark.parametrize("ks", [(4,), (3, 3)])
def test_brute_force_loops_small(ks):
    L, m, lam = 2, 8, 0.05
    alpha = 0.5
    g = _dirs(m, 5, perturb=5.0)
    C, O = 2, 3
    rng = np.random.default_rng(6)
    a = rng.standard_normal((2, C, 6))
    T = 1 + sum(ks)
    W = rng.standard_normal((O, C, T))
    b = rng.standard_normal(O)
    pts = _rot_points(g, ks, alpha)
    Ypts = [[_real_Y(L, p) for p in row] for row in pts]
    Bm = [_real_Y(L, gi / np.linalg.norm(gi)) for gi in g]
    pen = [0] + [36] * 5
    A = [[sum(Bm[i][r] * Bm[i][c] for i in range(m)) + (lam * pen[r] if r == c else 0.0) for c in range(6)]
         for r in range(6)]
    plan = lsc.LSCPlan(g, L, L, ks, alpha, lam)
    got, _ = lsc.lsc_forward(plan, a, W, b)
    for v in range(2):
        for o in range(O):
            y = []
            for i in range(m):
                s = b[o]
                for c in range(C):
                    for t in range(T):
                        s += W[o, c, t] * sum(Ypts[i][t][j] * a[v, c, j] for j in range(6))
                y.append(s)
            coef = _solve(A, [sum(Bm[i][r] * y[i] for i in range(m)) for r in range(6)])
            assert np.abs(np.array(coef) - got[v, o]).max() < 1e-11


def test_lsc_adjoints_dot_product():
    rng = np.random.default_rng(7)
    plan = lsc.LSCPlan(_dirs(30, 6), 4, 6, [6, 6], np.deg2rad(30), 0.006)
    V, C, O = 3, 2, 3
    a = rng.standard_normal((V, C, 15))
    W = rng.standard_normal((O, C, 13))
    b = rng.standard_normal(O)
    w = rng.standard_normal((V, O, 28))
    out0, z0 = lsc.lsc_forward(plan, a, W, None)
    da, dW, db = lsc.lsc_backward(plan, a, W, z0, w)
    # linear in a (bias 0)
    assert abs(np.sum(out0 * w) - np.sum(a * da)) < 1e-11 * abs(np.sum(out0 * w))
    # linear in W at fixed a
    assert abs(np.sum(out0 * w) - np.sum(W * dW)) < 1e-11 * abs(np.sum(out0 * w))
    # bias
    outb, _ = lsc.lsc_forward(plan, a, np.zeros_like(W), b)
    assert abs(np.sum(outb * w) - np.sum(b * db)) < 1e-11 * abs(np.sum(outb * w))
