"""Pins of the oracle's stacks: finite differences of the whole forward +
loss, superposition of the ReLU-free stack, and the input generator's
closed forms."""
import math

import numpy as np
import pytest

import datagen as dg
from oracle import lsc, sh, stack


def _small_stack(relu=True, lam=0.006, seed=0):
    acq = dg.make_acquisition(50 + seed, (1000.0, 2000.0), 30, 2.0, 2)
    plan = sh.SHPlan(acq.bvecs, acq.bvals, 4, lam)
    plan_out = sh.SHPlan(acq.bvecs, acq.bvals, 6, lam)
    g = dg.fibonacci_hemisphere(30)
    p1 = lsc.LSCPlan(g, 4, 4, (6, 6), np.deg2rad(30), lam)
    p2 = lsc.LSCPlan(g, 4, 6, (6, 6), np.deg2rad(30), lam)
    W1, b1 = dg.lsc_weights(50 + seed, 0, 2, 3, 13)
    W2, b2 = dg.lsc_weights(50 + seed, 1, 3, 2, 13)
    layers = [stack.Layer(p1, W1, b1, relu), stack.Layer(p2, W2, b2, False)]
    return stack.Stack(plan, layers, plan_out), acq


def test_stack_finite_differences():
    net, acq = _small_stack()
    # redraw the voxels until every ReLU input (first layer) is away from the kink
    for seed in range(50):
        batch = dg.stick_ball_batch(acq, 6, 2, 30.0, dg.rng_for(50, 2, seed))
        x, target = batch.x, batch.clean
        _, cache = net.forward(x)
        if np.abs(cache[1][0]).min() > 1e-4:
            break
    assert np.abs(cache[1][0]).min() > 1e-4
    loss, _, dx, dWs, dbs = net.loss_and_grads(x, target)
    h = 1e-6
    rng = np.random.default_rng(0)

    def fd(get, idx):
        arr = get()
        old = arr[idx]
        arr[idx] = old + h
        lp = net.loss_and_grads(x, target)[0]
        arr[idx] = old - h
        lm = net.loss_and_grads(x, target)[0]
        arr[idx] = old
        return (lp - lm) / (2 * h)

    for k in range(2):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in net.layers[k].W.shape)
            num = fd(lambda: net.layers[k].W, idx)
            assert abs(num - dWs[k][idx]) <= 1e-6 * max(1e-3, abs(num))
        for o in range(net.layers[k].b.shape[0]):
            num = fd(lambda: net.layers[k].b, (o,))
            assert abs(num - dbs[k][o]) <= 1e-6 * max(1e-3, abs(num))
    for _ in range(6):
        idx = (int(rng.integers(0, 6)), int(rng.integers(0, 60)))
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        num = (net.loss_and_grads(xp, target)[0] - net.loss_and_grads(xm, target)[0]) / (2 * h)
        assert abs(num - dx[idx]) <= 1e-6 * max(1e-3, abs(num))


def test_linear_stack_superposition():
    net, acq = _small_stack(relu=False, seed=1)
    for L in net.layers:
        L.b = np.zeros_like(L.b)
    rng = np.random.default_rng(1)
    x1, x2 = rng.standard_normal((3, 60)), rng.standard_normal((3, 60))
    f = lambda x: net.forward(x)[0]
    assert np.abs(f(2.0 * x1 - 3.0 * x2) - (2.0 * f(x1) - 3.0 * f(x2))).max() < 1e-12


def test_mse_definition():
    p = np.array([[1.0, 2.0], [3.0, 5.0]])
    t = np.array([[0.0, 2.0], [3.0, 1.0]])
    loss, g = stack.mse(p, t)
    assert loss == pytest.approx((1 + 16) / 4)
    assert np.allclose(g, 2 * (p - t) / 4)


# ----------------------------------------------------------------- generator

def test_fibonacci_hemisphere():
    g = dg.fibonacci_hemisphere(90)
    assert np.abs(np.linalg.norm(g, axis=1) - 1).max() < 1e-15
    assert (g[:, 2] > 0).all() and (g[:, 2] < 1).all()


def test_perturbation_is_bounded():
    g = dg.fibonacci_hemisphere(90)
    p = dg.perturb_directions(g, 2.0, dg.rng_for(0, 1, 0))
    ang = np.degrees(np.arccos(np.clip(np.sum(g * p, axis=1), -1, 1)))
    assert ang.max() <= 2.0 + 1e-9 and ang.max() > 1.0
    assert np.abs(np.linalg.norm(p, axis=1) - 1).max() < 1e-15


def test_single_stick_closed_form():
    u = np.array([[0.0, 0.0, 1.0]])
    dirs = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    b = np.array([1000.0, 1000.0])
    S = dg._stick_ball_clean(dirs, b, np.array([[0.0, 1.0]]), u[None], np.array([1]), dg.DIFFUSIVITY)
    assert S[0, 0] == pytest.approx(math.exp(-1000 * 1.7e-3))
    assert S[0, 1] == pytest.approx(1.0)


def test_rician_floor():
    rng = dg.rng_for(0, 9, 0)
    x = dg._rician(np.zeros(400000), 0.05, rng)
    assert x.mean() == pytest.approx(0.05 * math.sqrt(math.pi / 2), rel=5e-3)


def test_batch_shapes_and_determinism():
    acq = dg.make_acquisition(1, (1000.0, 2000.0, 3000.0), 90, 2.0, 18)
    assert acq.bvecs.shape == (288, 3) and (acq.bvals == 0).sum() == 18
    b1 = dg.stick_ball_batch(acq, 64, 3, 20.0, dg.rng_for(1, 2, 0))
    b2 = dg.stick_ball_batch(acq, 64, 3, 20.0, dg.rng_for(1, 2, 0))
    assert b1.x.shape == (64, 270) and np.array_equal(b1.x, b2.x)
    fr = b1.params[0]
    assert np.allclose(fr.sum(1), 1.0) and (fr >= 0).all()


def test_farthest_point_subset():
    g = dg.fibonacci_hemisphere(90)
    idx = dg.farthest_point_subset(g, 15)
    assert idx.shape == (15,) and len(set(idx.tolist())) == 15 and 0 in idx


def test_relative_mse_definition_and_special_cases():
    p = np.array([[1.0, 2.0], [3.0, 5.0]])
    t = np.array([[2.0, -2.0], [3.0, 4.0]])
    loss, g = stack.relative_mse(p, t, 0.0)
    assert loss == pytest.approx(((1 - 2) ** 2 / 4 + (2 + 2) ** 2 / 4 + 0 + 1 / 16) / 4)
    # constant target c: relative MSE is MSE / c^2 (eps = 0)
    rng = np.random.default_rng(3)
    pr = rng.standard_normal((5, 7))
    c = 1.7
    lr, gr = stack.relative_mse(pr, np.full_like(pr, c), 0.0)
    lm, gm = stack.mse(pr, np.full_like(pr, c))
    assert lr == pytest.approx(lm / c ** 2) and np.allclose(gr, gm / c ** 2)
    # finite differences
    tt = rng.uniform(0.2, 1.0, (4, 6))
    eps = 1e-3
    _, gg = stack.relative_mse(pr[:4, :6], tt, eps)
    h = 1e-6
    for ix in [(0, 0), (2, 3), (3, 5)]:
        a = pr[:4, :6].copy(); a[ix] += h
        b = pr[:4, :6].copy(); b[ix] -= h
        fd = (stack.relative_mse(a, tt, eps)[0] - stack.relative_mse(b, tt, eps)[0]) / (2 * h)
        assert abs(fd - gg[ix]) < 1e-7 * max(1.0, abs(fd))


def test_b0_normalisation_definition():
    acq = dg.make_acquisition(7, (1000.0, 2000.0), 30, 2.0, 4)
    plan = sh.SHPlan(acq.bvecs, acq.bvals, 4, 0.006)
    rng = np.random.default_rng(4)
    raw = rng.uniform(0.5, 2.0, (3, acq.bvals.size))
    x = sh.normalize_b0(raw, acq.bvals, plan)
    assert x.shape == (3, 60)
    # hand check for voxel 0, first DW volume of shell 0 (acquisition index 4)
    assert x[0, 0] == pytest.approx(raw[0, 4] / raw[0, :4].mean())
    # scaling a voxel's raw data leaves the normalised signal unchanged
    assert np.allclose(sh.normalize_b0(raw * 3.0, acq.bvals, plan), x)
    # generator consistency: the datagen batches are normalised the same way
    b = dg.stick_ball_batch(acq, 5, 2, 30.0, dg.rng_for(7, 2, 0))
    raw_dw = b.x * b.raw_b0.mean(axis=1, keepdims=True)
    rawfull = np.concatenate([b.raw_b0, raw_dw], axis=1)
    assert np.allclose(sh.normalize_b0(rawfull, acq.bvals, plan), b.x)
