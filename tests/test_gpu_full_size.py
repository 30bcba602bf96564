"""The three-shell stack at its full size (1 048 576 voxels of 3 x 90
directions, order 8, LSC 3 -> 32 -> 3) in the configuration the benchmark
times: folded LSC, fused loss head, workspace passes of 131 072 voxels; in
BF16 the 1440-wide activation and its gradient stored in bfloat16 and the
hidden ReLU's mask carried as bits.

The oracle cannot run a million voxels in a test, so the checks are
  * every per-voxel result (last LSC output, loss-head gradient, input
    gradient) on 48 sampled voxels (both ends, the workspace-pass seams,
    random ones) against the FP64 oracle run on just those voxels, with the
    loss scale 1/(V * 270) of the full batch, norm-wise and per voxel;
  * ReLU bits on the sampled rows against a host packing, and the backward
    with bits bitwise equal to the backward with the activation mask over
    the whole batch;
  * the weight gradient of the full batch against the sum of the gradients
    of its two halves (a property of the sum over voxels at any size).
"""
import numpy as np
import pytest
import torch

import bench
import datagen as dg
import paper_1808_01517_amd as dl
from oracle import lsc as olsc
from oracle import sh as osh
from oracle import stack as ostack

from parity_util import check, fmt

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CHUNK = 1 << 17


def pack_bits(a: np.ndarray) -> np.ndarray:
    pos = (a.reshape(a.shape[0], -1, 16) > 0).astype(np.uint16)
    return (pos << np.arange(16, dtype=np.uint16)).sum(axis=2, dtype=np.uint16)


@pytest.fixture(scope="module")
def data():
    w = dg.C2
    acq, x, clean = bench.make_data(w, w.voxels)
    return w, acq, x, clean


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_c2_full_size_sampled_parity(prec, data):
    w, acq, x_h, clean_h = data
    V = x_h.shape[0]
    assert V == 1 << 20
    plan = dl.SHPlan(acq.bvecs, acq.bvals, w.sh_order, w.lb_lambda)
    assert dl.sh2signal_mse_supported(plan)
    g = dg.lsc_sampled_gradients(w)
    ch = w.channels
    layers, olayers = [], []
    for k in range(len(ch) - 1):
        p = dl.LSCPlan(g, w.sh_order_lsc_in, w.sh_order_lsc_out, w.kernel_sizes, w.angular_distance, w.lb_lambda)
        op = olsc.LSCPlan(g, w.sh_order_lsc_in, w.sh_order_lsc_out, w.kernel_sizes, w.angular_distance, w.lb_lambda)
        Wk, bk = dg.lsc_weights(w.config, k, ch[k], ch[k + 1], p.T)
        Wk, bk = Wk.astype(np.float32), bk.astype(np.float32)
        relu = k < len(ch) - 2
        layers.append((p, torch.from_numpy(Wk).to(DEV), torch.from_numpy(bk).to(DEV), relu))
        olayers.append(ostack.Layer(op, Wk.astype(np.float64), bk.astype(np.float64), relu))
    half = prec == "bf16"
    x = torch.from_numpy(x_h).to(DEV)
    tgt = torch.from_numpy(clean_h).to(DEV)
    ws = dl.Workspace(max(dl.lsc_workspace_bytes(p, ch[k], ch[k + 1], CHUNK, prec, "folded")
                          for k, (p, _, _, _) in enumerate(layers)), torch.device(DEV))
    p1, W1, b1, _ = layers[0]
    p2, W2, b2, _ = layers[1]
    # forward, as the benchmark step runs it
    c0 = dl.signal2sh_fwd(plan, x, precision=prec)
    a1 = torch.empty((V, ch[1], p1.K_out), dtype=torch.bfloat16 if half else torch.float32, device=DEV)
    bits = dl.relu_bits_like(a1) if half else None
    dl.lsc_fwd(p1, c0, W1, b1, relu=True, out=a1, precision=prec, workspace=ws, form="folded", relu_bits=bits)
    a2 = dl.lsc_fwd(p2, a1, W2, b2, precision=prec, workspace=ws, form="folded")
    loss = torch.empty((), dtype=torch.float32, device=DEV)
    dc = torch.empty_like(a2)
    head_ws = torch.empty(dl.lib().dlm_sh2signal_mse_workspace_bytes(plan.handle, V), dtype=torch.uint8, device=DEV)
    dl.sh2signal_mse_fwd_bwd(plan, a2, tgt, precision=prec, outs=(loss, dc, head_ws))
    # backward
    g1, dW2, db2 = dl.lsc_bwd(p2, a1, W2, dc, relu_in=True, precision=prec, workspace=ws, form="folded",
                              relu_bits=bits)
    g0, dW1, db1 = dl.lsc_bwd(p1, c0, W1, g1, precision=prec, workspace=ws, form="folded")
    dx = dl.signal2sh_bwd(plan, g0, precision=prec)
    torch.cuda.synchronize()
    assert np.isfinite(float(loss))

    # the oracle on sampled voxels, with the full batch's loss scale
    rng = np.random.default_rng(2024)
    idx = np.unique(np.concatenate([[0, 1, CHUNK - 1, CHUNK, 2 * CHUNK - 1, V // 2, V - 2, V - 1],
                                    rng.integers(0, V, 40)]))
    xs = x_h[idx].astype(np.float64)
    ts = clean_h[idx].astype(np.float64)
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, w.sh_order, w.lb_lambda)
    net = ostack.Stack(oplan, olayers, oplan)
    xhat_ref, cache = net.forward(xs)
    dxh_ref = 2.0 * (xhat_ref - ts) / (V * x_h.shape[1])
    dc_ref = osh.sh2signal_adjoint(oplan, dxh_ref)
    dx_ref, _, _ = net.backward(cache, dxh_ref)
    sel = torch.from_numpy(idx).to(DEV)
    errs = {}
    check("a2", a2.index_select(0, sel), cache[0][-1], prec, errs)
    check("dc", dc.index_select(0, sel), dc_ref, prec, errs)
    check("dx", dx.index_select(0, sel), dx_ref, prec, errs)

    # the backward with the activation mask: bitwise the same
    if half:
        got = bits.index_select(0, sel).cpu().numpy().view(np.uint16)
        assert np.array_equal(got, pack_bits(a1.index_select(0, sel).float().cpu().numpy()))
        g1m, dW2m, db2m = dl.lsc_bwd(p2, a1, W2, dc, relu_in=True, precision=prec, workspace=ws, form="folded")
        torch.cuda.synchronize()
        assert torch.equal(g1m, g1) and torch.equal(dW2m, dW2) and torch.equal(db2m, db2)
        del g1m

    # the weight gradient is a sum over voxels: full batch = first half + second half
    h = V // 2
    _, dW2a, db2a = dl.lsc_bwd(p2, a1[:h], W2, dc[:h], need_input_grad=False, precision=prec, workspace=ws,
                               form="folded")
    _, dW2b, db2b = dl.lsc_bwd(p2, a1[h:], W2, dc[h:], need_input_grad=False, precision=prec, workspace=ws,
                               form="folded")
    check("dW2_split", dW2, dW2a.double() + dW2b.double(), prec, errs, kind="sum")
    check("db2_split", db2, db2a.double() + db2b.double(), prec, errs, kind="sum")
    print(f"[parity] full size {prec}, {len(idx)} sampled voxels (norm-wise/per-row): " + fmt(errs), flush=True)
