"""Pins of the FP64 oracle's SH basis, Signal2SH and SH2Signal.

Each test ties the oracle to something other than itself: quadrature,
the addition theorem, textbook closed forms, scipy's complex harmonics,
the Laplace-Beltrami eigen-relation, exact recovery, brute-force loops.
"""
import math

import numpy as np
import pytest
import scipy.special as sps

from datagen import fibonacci_hemisphere, perturb_directions, rng_for
from oracle import sh


def _quadrature(n_theta=32, n_phi=64):
    x, w = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    T, P = np.meshgrid(np.arccos(x), phi, indexing="ij")
    W = np.outer(w, np.full(n_phi, 2 * np.pi / n_phi))
    return T.ravel(), P.ravel(), W.ravel()


@pytest.mark.parametrize("L", [0, 2, 4, 8, 12, 16])
def test_orthonormal_under_quadrature(L):
    # Gauss-Legendre(32) in cos(theta) x 64 uniform phi is exact for these products.
    t, p, w = _quadrature()
    B = sh.real_sh_basis(L, t, p)
    G = (B * w[:, None]).T @ B
    assert np.abs(G - np.eye(B.shape[1])).max() < 1e-13


def test_coefficient_count_and_order():
    assert [sh.n_coeffs(L) for L in (0, 2, 4, 6, 8)] == [1, 6, 15, 28, 45]
    ls, ms = sh.degree_order(4)
    assert list(ls[:6]) == [0, 2, 2, 2, 2, 2] and list(ms[:6]) == [0, -2, -1, 0, 1, 2]
    with pytest.raises(ValueError):
        sh.n_coeffs(3)


def test_textbook_values():
    # Y_00 and every l = 2 function written out by hand.
    rng = np.random.default_rng(0)
    t = rng.uniform(0, np.pi, 50)
    p = rng.uniform(-np.pi, np.pi, 50)
    B = sh.real_sh_basis(2, t, p)
    st, ct = np.sin(t), np.cos(t)
    expect = np.stack([
        np.full_like(t, 0.28209479177387814),
        math.sqrt(15 / (16 * math.pi)) * st ** 2 * np.cos(2 * p),
        -math.sqrt(15 / (4 * math.pi)) * ct * st * np.cos(p),
        math.sqrt(5 / (16 * math.pi)) * (3 * ct ** 2 - 1),
        -math.sqrt(15 / (4 * math.pi)) * ct * st * np.sin(p),
        math.sqrt(15 / (16 * math.pi)) * st ** 2 * np.sin(2 * p),
    ], axis=1)
    assert np.abs(B - expect).max() < 1e-14


@pytest.mark.parametrize("L", [4, 8, 12])
def test_matches_scipy_complex_harmonics(L):
    # real-from-complex map: m<0 -> sqrt2 Re Y_l^|m|, m=0 -> Y_l^0, m>0 -> sqrt2 Im Y_l^m
    rng = np.random.default_rng(1)
    t = rng.uniform(0, np.pi, 40)
    p = rng.uniform(-np.pi, np.pi, 40)
    B = sh.real_sh_basis(L, t, p)
    ls, ms = sh.degree_order(L)
    for j, (l, m) in enumerate(zip(ls, ms)):
        Y = sps.sph_harm_y(int(l), abs(int(m)), t, p)
        ref = math.sqrt(2) * Y.real if m < 0 else (Y.real if m == 0 else math.sqrt(2) * Y.imag)
        assert np.abs(B[:, j] - ref).max() < 1e-12, (l, m)


@pytest.mark.parametrize("L", [4, 8])
def test_addition_theorem(L):
    # sum_m Y_lm(u) Y_lm(v) = (2l+1)/(4 pi) P_l(u.v): convention free.
    rng = np.random.default_rng(2)
    u = rng.standard_normal((20, 3)); u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = rng.standard_normal((20, 3)); v /= np.linalg.norm(v, axis=1, keepdims=True)
    Bu, Bv = sh.basis_at(L, u), sh.basis_at(L, v)
    ls, _ = sh.degree_order(L)
    cos = np.sum(u * v, axis=1)
    for l in range(0, L + 1, 2):
        sel = ls == l
        lhs = np.sum(Bu[:, sel] * Bv[:, sel], axis=1)
        rhs = (2 * l + 1) / (4 * np.pi) * np.polynomial.legendre.legval(cos, [0] * l + [1])
        assert np.abs(lhs - rhs).max() < 1e-13


def test_lb_penalty_is_laplace_beltrami_squared():
    # Delta_S Y_lm = -l(l+1) Y_lm, checked by finite differences in (theta, phi);
    # the penalty must be its square, l^2 (l+1)^2.
    L = 6
    rng = np.random.default_rng(3)
    t = rng.uniform(0.4, 2.7, 10)
    p = rng.uniform(-3, 3, 10)
    h = 1e-4
    f = lambda tt, pp: sh.real_sh_basis(L, tt, pp)
    d2t = (f(t + h, p) - 2 * f(t, p) + f(t - h, p)) / h ** 2
    d1t = (f(t + h, p) - f(t - h, p)) / (2 * h)
    d2p = (f(t, p + h) - 2 * f(t, p) + f(t, p - h)) / h ** 2
    lap = d2t + (np.cos(t) / np.sin(t))[:, None] * d1t + d2p / (np.sin(t) ** 2)[:, None]
    ratio = -lap / f(t, p)
    ls, _ = sh.degree_order(L)
    ok = np.abs(f(t, p)) > 1e-3
    assert np.abs((ratio - ls * (ls + 1))[ok]).max() < 1e-3
    assert np.array_equal(sh.lb_penalty(4), np.array([0.0] + [36.0] * 5 + [400.0] * 9))


def _table(n, seed=0):
    return perturb_directions(fibonacci_hemisphere(n), 2.0, rng_for(99, 1, seed))


@pytest.mark.parametrize("L,N", [(4, 30), (8, 90), (2, 6)])
def test_exact_recovery_lambda0(L, N):
    g = _table(N)
    B = sh.basis_at(L, g)
    P = sh.fit_matrix(B, L, 0.0)
    c = np.random.default_rng(4).standard_normal((7, B.shape[1]))
    assert np.abs((B @ c.T).T @ P.T - c).max() < 1e-11
    # agrees with plain least squares at lambda = 0
    x = np.random.default_rng(5).standard_normal(N)
    ref = np.linalg.lstsq(B, x, rcond=None)[0]
    assert np.abs(P @ x - ref).max() < 1e-11


def test_regularised_bias_closed_form():
    # P B c = c - lambda (B^T B + lambda L)^{-1} L c with L written out by hand.
    L_, N, lam = 4, 30, 0.006
    g = _table(N, 1)
    B = sh.basis_at(L_, g)
    Ld = np.diag([0.0] + [2.0 ** 2 * 3 ** 2] * 5 + [4.0 ** 2 * 5 ** 2] * 9)
    c = np.random.default_rng(6).standard_normal(B.shape[1])
    got = sh.fit_matrix(B, L_, lam) @ (B @ c)
    expect = c - lam * np.linalg.solve(B.T @ B + lam * Ld, Ld @ c)
    assert np.abs(got - expect).max() < 1e-12
    assert np.abs(got - c).max() > 1e-6  # the penalty does act


@pytest.mark.parametrize("lam", [0.0, 0.006, 0.06, 5.0])
def test_constant_signal_maps_to_scaled_e0(lam):
    g = _table(90, 2)
    P = sh.fit_matrix(sh.basis_at(8, g), 8, lam)
    c = P @ np.ones(90)
    e0 = np.zeros(45); e0[0] = math.sqrt(4 * math.pi)
    assert np.abs(c - e0).max() < 1e-12


def test_brute_force_fit_small():
    # N = 6, L = 2: normal equations by loops and Gauss-Jordan elimination.
    g = _table(6, 3)
    lam = 0.3
    th = np.arccos(g[:, 2]); ph = np.arctan2(g[:, 1], g[:, 0])
    Y = [[sps.sph_harm_y(l, abs(m), th[i], ph[i]) for (l, m) in
          [(0, 0), (2, -2), (2, -1), (2, 0), (2, 1), (2, 2)]] for i in range(6)]
    ms = [0, -2, -1, 0, 1, 2]
    B = [[(math.sqrt(2) * Y[i][j].real if ms[j] < 0 else (Y[i][j].real if ms[j] == 0 else math.sqrt(2) * Y[i][j].imag))
          for j in range(6)] for i in range(6)]
    pen = [0, 36, 36, 36, 36, 36]
    x = [0.9, 0.5, 0.2, 0.7, 0.4, 0.1]
    A = [[sum(B[i][r] * B[i][c] for i in range(6)) + (lam * pen[r] if r == c else 0.0) for c in range(6)] for r in range(6)]
    rhs = [sum(B[i][r] * x[i] for i in range(6)) for r in range(6)]
    M = [A[r][:] + [rhs[r]] for r in range(6)]
    for col in range(6):
        piv = max(range(col, 6), key=lambda r: abs(M[r][col]))
        M[col], M[piv] = M[piv], M[col]
        for r in range(6):
            if r != col:
                f = M[r][col] / M[col][col]
                M[r] = [M[r][k] - f * M[col][k] for k in range(7)]
    sol = [M[r][6] / M[r][r] for r in range(6)]
    plan = sh.SHPlan(g, np.full(6, 1000.0), 2, lam)
    got = sh.signal2sh(plan, np.array([x]))[0, 0]
    assert np.abs(got - np.array(sol)).max() < 1e-12


def test_sh2signal_of_signal2sh_is_identity_on_bandlimited():
    g = _table(90, 4)
    plan = sh.SHPlan(g, np.full(90, 2000.0), 8, 0.0)
    c = np.random.default_rng(7).standard_normal((5, 1, 45))
    x = sh.sh2signal(plan, c)
    assert np.abs(sh.sh2signal(plan, sh.signal2sh(plan, x)) - x).max() < 1e-11
    BP = plan.B[0] @ plan.P[0]
    assert np.abs(BP @ BP - BP).max() < 1e-11


def test_sh2signal_of_e0_is_constant():
    plan = sh.SHPlan(_table(30, 5), np.full(30, 1000.0), 4, 0.006)
    c = np.zeros((1, 1, 15)); c[0, 0, 0] = 1.0
    assert np.abs(sh.sh2signal(plan, c) - 1 / (2 * math.sqrt(math.pi))).max() < 1e-15


def test_shell_grouping():
    bvals = np.array([0, 5, 1000, 2990, 1010, 2000, 0, 3000, 1990, 30])
    idx, b = sh.group_shells(bvals)
    assert [list(i) for i in idx] == [[2, 4], [5, 8], [3, 7]]
    assert np.allclose(b, [1005, 1995, 2995])


def test_multishell_blocks_are_independent():
    # per-shell fits: changing shell 1's data leaves shell 0's coefficients alone
    rng = np.random.default_rng(8)
    g = np.concatenate([_table(30, 6), _table(30, 7)])
    plan = sh.SHPlan(g, np.r_[np.full(30, 1000.0), np.full(30, 2000.0)], 4, 0.006)
    x = rng.standard_normal((3, 60))
    c = sh.signal2sh(plan, x)
    x2 = x.copy(); x2[:, 30:] += 1.0
    c2 = sh.signal2sh(plan, x2)
    assert np.array_equal(c[:, 0], c2[:, 0])
    assert np.abs(c2[:, 1, 0] - c[:, 1, 0] - math.sqrt(4 * math.pi)).max() < 1e-12


@pytest.mark.parametrize("fn,adj,shape_in,shape_out", [
    (sh.signal2sh, sh.signal2sh_adjoint, (4, 60), (4, 2, 15)),
    (sh.sh2signal, sh.sh2signal_adjoint, (4, 2, 15), (4, 60)),
])
def test_transform_adjoints(fn, adj, shape_in, shape_out):
    g = np.concatenate([_table(30, 8), _table(30, 9)])
    plan = sh.SHPlan(g, np.r_[np.full(30, 1000.0), np.full(30, 2000.0)], 4, 0.006)
    rng = np.random.default_rng(9)
    u = rng.standard_normal(shape_in)
    w = rng.standard_normal(shape_out)
    lhs = np.sum(fn(plan, u) * w)
    rhs = np.sum(u * adj(plan, w))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_fit_exists_unless_normal_matrix_is_rank_deficient():
    # At lambda = 0 the normal matrix B^T B has rank min(N, K) for directions
    # in general position, so the fit needs N >= K.  For lambda > 0 the
    # penalty covers every l > 0 and only Y_00 (a nonzero constant, never in
    # the null space of B) is unpenalised: a fit exists for any N >= 1.
    g = _table(30, 10)
    assert not sh.has_fit(sh.basis_at(8, g), 8, 0.0)          # N = 30 < K = 45
    assert sh.has_fit(sh.basis_at(8, g), 8, 0.006)
    assert sh.has_fit(sh.basis_at(4, g), 4, 0.0)              # N = 30 >= K = 15
    assert sh.has_fit(sh.basis_at(8, g[:1]), 8, 0.006)        # one direction
    plan = sh.SHPlan(g, np.full(30, 1000.0), 8, 0.0)
    assert not plan.has_fit and plan.P is None
    with pytest.raises(np.linalg.LinAlgError):
        sh.signal2sh(plan, np.ones((1, 30)))
    with pytest.raises(np.linalg.LinAlgError):
        sh.signal2sh_adjoint(plan, np.ones((1, 1, 45)))


def test_evaluation_only_plan_evaluates_closed_forms():
    # SH2Signal onto 30 directions at order 8 (no fit): the l = 2, m = 0
    # coefficient alone gives the textbook sqrt(5/(16 pi)) (3 z^2 - 1), and
    # the l = 8 block filled with Y_8m(v) gives the addition theorem's
    # (2l+1)/(4 pi) P_8(g . v) at every direction g, independent of convention.
    g = _table(30, 11)
    plan = sh.SHPlan(g, np.full(30, 1000.0), 8, 0.0)
    gn = g / np.linalg.norm(g, axis=1, keepdims=True)
    ls, ms = sh.degree_order(8)
    c = np.zeros((1, 1, 45))
    c[0, 0, int(np.flatnonzero((ls == 2) & (ms == 0))[0])] = 1.0
    expect = math.sqrt(5 / (16 * math.pi)) * (3 * gn[:, 2] ** 2 - 1)
    assert np.abs(sh.sh2signal(plan, c)[0] - expect).max() < 1e-14
    v = np.array([[0.3, -0.5, 0.81]])
    v /= np.linalg.norm(v)
    c = np.zeros((1, 1, 45))
    c[0, 0, ls == 8] = sh.basis_at(8, v)[0, ls == 8]
    expect = 17 / (4 * math.pi) * sps.eval_legendre(8, gn @ v[0])
    assert np.abs(sh.sh2signal(plan, c)[0] - expect).max() < 1e-12
