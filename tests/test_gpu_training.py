"""GPU tests of the training-side forms: autograd modules, per-batch table
distortion, the four-layer network's gradients against the FP64 oracle and
FP64 finite differences, recomputation, checkpoint/resume, and the learned
predictor against the plain SH fit."""
import numpy as np
import pytest
import torch

import datagen as dg
import paper_1808_01517_amd as dl
from paper_1808_01517_amd import apps
from paper_1808_01517_amd.layers import LocalSphericalConvolution, SH2Signal, Signal2SH
from oracle import lsc as olsc
from oracle import sh as osh
from oracle import stack as ostack

from parity_util import check, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def test_modules_autograd_match_oracle():
    # the paper's single-shell example geometry: order 4, kernel [5], alpha = pi/5
    g = dg.perturb_directions(dg.fibonacci_hemisphere(30), 2.0, dg.rng_for(21, 1, 0))
    s2sh = Signal2SH(4, g, lb_lambda=0.006)
    lsc = LocalSphericalConvolution(1, 1, g, 4, 4, [5], np.pi / 5, 0.006).to(DEV)
    sh2s = SH2Signal(4, g)
    ma = torch.full((1, 1, 1, 6), 1.0 / 6.0)
    lsc.sconv.weight = torch.nn.Parameter(ma.to(DEV))
    lsc.sconv.bias = torch.nn.Parameter(torch.zeros(1, device=DEV))
    rng = np.random.default_rng(0)
    x5 = rng.uniform(0.1, 1.0, size=(1, 30, 3, 4, 5))      # subjects x dirs x H x W x D
    xt = cu(x5).requires_grad_(True)
    out = sh2s(lsc(s2sh(xt)))
    assert out.shape == (1, 30, 3, 4, 5)
    # oracle on the voxel-major view
    xv = f32(x5).transpose(0, 2, 3, 4, 1).reshape(-1, 30)
    op = osh.SHPlan(g, np.full(30, 1000.0), 4, 0.006)
    lp = olsc.LSCPlan(g, 4, 4, [5], np.pi / 5, 0.006)
    net = ostack.Stack(op, [ostack.Layer(lp, np.full((1, 1, 6), 1 / 6), np.zeros(1), False)],
                       osh.SHPlan(g, np.full(30, 1000.0), 4, 0.0))
    ref, cache = net.forward(xv)
    got = out.detach().permute(0, 2, 3, 4, 1).reshape(-1, 30)
    check("out", got, ref, "fp32")
    up = rng.standard_normal(out.shape)
    out.backward(cu(up))
    upv = up.transpose(0, 2, 3, 4, 1).reshape(-1, 30)
    dx, dWs, dbs = net.backward(cache, upv)
    check("dx", xt.grad.permute(0, 2, 3, 4, 1).reshape(-1, 30), dx, "fp32")
    check("dW", lsc.sconv.weight.grad.reshape(1, 1, 6), dWs[0], "fp32", kind="sum")
    check("db", lsc.sconv.bias.grad, dbs[0], "fp32", kind="sum")


def test_update_gradients_matches_fresh_plan():
    w = dg.C4
    acq = dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
    x = cu(dg.stick_ball_batch(acq, 500, 3, 20.0, dg.rng_for(5, 2, 0)).x)
    c_old = dl.signal2sh_fwd(plan, x)
    dacq = dg.distort_acquisition(acq, 3.0, dg.rng_for(w.config, dg.STREAM_DISTORT, 7))
    plan.update_gradients(dacq.bvecs)
    c_new = dl.signal2sh_fwd(plan, x)
    ref = osh.signal2sh(osh.SHPlan(dacq.bvecs, dacq.bvals, 8, 0.006), x.double().cpu().numpy())
    check("c", c_new, ref, "fp32")
    assert rel(c_old, ref) > 1e-4   # the tables really changed


def _c4_oracle(net_gpu, dacq):
    w = dg.C4
    op = osh.SHPlan(dacq.bvecs, dacq.bvals, 8, w.lb_lambda)
    g = dg.lsc_sampled_gradients(w)
    layers = []
    for k, s in enumerate(net_gpu.specs):
        lp = olsc.LSCPlan(g, s.sh_order_in, s.sh_order_out, w.kernel_sizes, w.angular_distance, w.lb_lambda)
        layers.append(ostack.Layer(lp, net_gpu.W[k].double().cpu().numpy(), net_gpu.b[k].double().cpu().numpy(),
                                   s.relu))
    return ostack.Stack(op, layers, op)


@pytest.mark.parametrize("form", ["folded", "resample"])
def test_c4_gradients_vs_oracle_and_finite_differences(form):
    net, acq = apps.c4_network("fp32", form, recompute=(0, 2), batch=64)
    dacq, x, clean = apps.c4_batch(acq, 3, V=64)
    net.plan_in.update_gradients(dacq.bvecs)
    loss, dx = net.loss_and_grads(cu(x), cu(clean), need_input_grad=True)
    torch.cuda.synchronize()
    onet = _c4_oracle(net, dacq)
    xd, cd = f32(x), f32(clean)
    l_ref, _, dx_ref, dW_ref, db_ref = onet.loss_and_grads(xd, cd)
    assert abs(float(loss) - l_ref) / l_ref <= 1e-5
    check("dx", dx, dx_ref, "fp32")
    for k in range(4):
        check(f"dW{k}", net.dW[k], dW_ref[k], "fp32", kind="sum")
        check(f"db{k}", net.db[k], db_ref[k], "fp32", kind="sum")
    # FP64 central differences of the oracle's loss at sampled coordinates
    rng = np.random.default_rng(11)
    h = 1e-6
    for k in range(4):
        L = onet.layers[k]
        idx = [tuple(int(rng.integers(0, n)) for n in L.W.shape) for _ in range(4)]
        fd, an = [], []
        for ix in idx:
            old = L.W[ix]
            L.W[ix] = old + h
            lp = ostack.mse(onet.forward(xd)[0], cd)[0]
            L.W[ix] = old - h
            lm = ostack.mse(onet.forward(xd)[0], cd)[0]
            L.W[ix] = old
            fd.append((lp - lm) / (2 * h))
            an.append(float(net.dW[k].double().cpu().numpy()[ix]))
        assert rel(np.array(an), np.array(fd)) <= 1e-4, (k, an, fd)


def test_recompute_gives_identical_gradients():
    a, acq = apps.c4_network("fp32", "folded", recompute=(0, 2), batch=300)
    b, _ = apps.c4_network("fp32", "folded", recompute=(), batch=300)
    _, x, clean = apps.c4_batch(acq, 1, V=300)
    a.loss_and_grads(cu(x), cu(clean))
    b.loss_and_grads(cu(x), cu(clean))
    torch.cuda.synchronize()
    for k in range(4):
        assert torch.equal(a.dW[k], b.dW[k]) and torch.equal(a.db[k], b.db[k])


@pytest.mark.parametrize("prec,half", [("fp32", False), ("bf16", False), ("bf16", True)])
def test_relu_bits_give_identical_gradients(prec, half):
    """Hidden ReLU masks from the forward's bits (three hidden layers, two of
    them recomputed into one shared buffer) against masks from the stored
    activations: bitwise the same gradients and loss."""
    a, acq = apps.c4_network(prec, "folded", recompute=(0, 2), batch=300, bf16_activations=half, relu_bits=True)
    b, _ = apps.c4_network(prec, "folded", recompute=(0, 2), batch=300, bf16_activations=half, relu_bits=False)
    assert sum(x is not None for x in a.bits) == 3 and all(x is None for x in b.bits)
    _, x, clean = apps.c4_batch(acq, 2, V=300)
    a.loss_and_grads(cu(x), cu(clean))
    b.loss_and_grads(cu(x), cu(clean))
    torch.cuda.synchronize()
    assert torch.equal(a.loss, b.loss)
    for k in range(4):
        assert torch.equal(a.dW[k], b.dW[k]) and torch.equal(a.db[k], b.db[k])


def test_checkpoint_resume_is_exact(tmp_path):
    def run(n_steps, net):
        for i in range(n_steps):
            dacq, x, clean = apps.c4_batch(acq, 100 + net.t, V=256)
            net.plan_in.update_gradients(dacq.bvecs)
            net.train_step(cu(x), cu(clean), lr=1e-3)
        torch.cuda.synchronize()

    full, acq = apps.c4_network("fp32", "folded", batch=256)
    run(4, full)
    part, _ = apps.c4_network("fp32", "folded", batch=256)
    run(2, part)
    path = tmp_path / "ckpt.pt"
    torch.save(part.state_dict(), path)
    resumed, _ = apps.c4_network("fp32", "folded", batch=256)
    resumed.load_state_dict(torch.load(path, weights_only=True))
    run(2, resumed)
    for k in range(4):
        assert torch.equal(full.W[k], resumed.W[k]) and torch.equal(full.b[k], resumed.b[k])


@pytest.mark.parametrize("prec,half", [("fp32", False), ("bf16", False), ("bf16", True)])
def test_learned_network_gradients_vs_oracle(prec, half):
    # half: hidden activations (64 x 45 per voxel) and their gradients stored in bfloat16
    S = apps.learned_setup(precision=prec, batch=128, bf16_activations=half)
    net, acq, cols = S["net"], S["acq"], S["cols"]
    b = dg.stick_ball_batch(acq, 128, 3, 20.0, dg.rng_for(4, 2, 77))
    xs = f32(b.x[:, cols])
    tgt = f32(b.clean)
    net.loss_and_grads(cu(xs), cu(tgt))
    torch.cuda.synchronize()
    w = dg.C5
    g = dg.lsc_sampled_gradients(w)
    layers = [ostack.Layer(olsc.LSCPlan(g, s.sh_order_in, s.sh_order_out, w.kernel_sizes, w.angular_distance,
                                        w.lb_lambda), net.W[k].double().cpu().numpy(),
                           net.b[k].double().cpu().numpy(), s.relu) for k, s in enumerate(net.specs)]
    sub = S["sub"]
    onet = ostack.Stack(osh.SHPlan(sub.bvecs, sub.bvals, 4, w.lb_lambda), layers,
                        osh.SHPlan(acq.bvecs, acq.bvals, 8, w.lb_lambda))
    _, cache = onet.forward(xs)
    # ReLU pattern from the GPU's own activations (BF16 rounding can flip signs near 0)
    zs = [net.acts[k + 1][:128].double().cpu().numpy() if L.relu else z
          for k, (z, L) in enumerate(zip(cache[1], layers))]
    xhat = net.xhat[:128].double().cpu().numpy()
    _, dxh = ostack.mse(xhat, tgt)
    _, dWs, dbs = onet.backward((cache[0], zs), dxh)
    for k in range(3):
        check(f"dW{k}", net.dW[k], dWs[k], prec, kind="sum")
        check(f"db{k}", net.db[k], dbs[k], prec, kind="sum")


def test_learned_predictor_beats_plain_fit():
    """Trained on 131 072 voxels (a short run), scored on the 262 144
    held-out voxels of the learned-form workload."""
    res, S, net = apps.run_learned(train_voxels=1 << 17, eval_voxels=1 << 18, epochs=6, lr=2e-3, batch=4096)
    print(res)
    assert res["eval_voxels"] == 1 << 18
    assert res["nrmse_net_vs_clean"] < res["nrmse_fit_vs_clean"]
    # the plain fit computed by the library matches the oracle's fit on a sample
    w = dg.C5
    b = dg.stick_ball_batch(S["acq"], 200, 3, 20.0, dg.rng_for(w.config, 3, 999))
    xs = f32(b.x[:, S["cols"]])
    got = apps.plain_fit(S, cu(xs))
    sub, acq = S["sub"], S["acq"]
    ref = osh.sh2signal(osh.SHPlan(acq.bvecs, acq.bvals, 4, 0.0),
                        osh.signal2sh(osh.SHPlan(sub.bvecs, sub.bvals, 4, w.lb_lambda), xs))
    check("plain fit", got, ref, "fp32")
