"""Workload drivers built on the library: the four-layer differentiation
workload and the learned subsampled-q-space predictor.

Differentiation workload: Signal2SH -> LSC 3->32->64->32->3 (ReLU after
the first three) -> SH2Signal on the three-shell, 90-direction, order-8
geometry; batches of 8192 voxels, each drawing a fresh seeded distortion
of up to 3 degrees of every gradient direction (the plan's float64 fit is
rebuilt per batch, Sec. 1 motivates exactly this per-scan variation); MSE in
q-space against the noise-free signal on the distorted table; outputs of
layers 1 and 3 recomputed in the backward pass.

Learned predictor: from 15 directions per shell (greedy farthest-point
subset of each shell's 90), Signal2SH at order 4 -> LSC 3->64 (order 4->8)
-> ReLU -> LSC 64->64 -> ReLU -> LSC 64->3 -> SH2Signal at order 8 onto
the full 3 x 90 table, trained with the library's MSE and Adam kernels in
the BF16 form with float32 master weights; judged by the normalised RMSE
against the noise-free full-table signal, next to the plain order-4
least-squares fit from the same 15 directions (Sec. 1 cites deep learning
from few directions as the motivating application).

    python -m paper_1808_01517_amd.apps learned [--train-voxels N] [--epochs E]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

import datagen as dg

from . import SHPlan, sh2signal_fwd, signal2sh_fwd
from .network import LayerSpec, LSCNetwork

# ----------------------------------------------------------------- helpers


def _gen(acq, V, w, stream, chunk=1 << 16, workers=16):
    """Noisy normalised signal, noise-free signal (float32) for V voxels."""
    n = acq.dw_bvecs.shape[0]
    x = np.empty((V, n), dtype=np.float32)
    clean = np.empty((V, n), dtype=np.float32)

    def one(ci):
        lo, hi = ci * chunk, min(V, (ci + 1) * chunk)
        b = dg.stick_ball_batch(acq, hi - lo, w.nf_max, w.snr, dg.rng_for(w.config, stream, ci), dtype=np.float32)
        x[lo:hi] = b.x
        clean[lo:hi] = b.clean

    with ThreadPoolExecutor(max_workers=min(workers, os.cpu_count() or 4)) as ex:
        list(ex.map(one, range((V + chunk - 1) // chunk)))
    return x, clean


def nrmse(pred: torch.Tensor, ref: torch.Tensor) -> float:
    """||pred - ref||_2 / ||ref||_2 over every voxel and direction (float64 sums)."""
    d = (pred.double() - ref.double()).pow(2).sum()
    return float(torch.sqrt(d / ref.double().pow(2).sum()))


# --------------------------------------------------- differentiation workload

def c4_network(precision="fp32", form="folded", recompute=(0, 2), device="cuda:0", weights=None, batch=8192,
               bf16_activations=False, relu_bits=False):
    w = dg.C4
    acq = dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
    plan = SHPlan(acq.bvecs, acq.bvals, w.sh_order, w.lb_lambda)
    ch = w.channels
    specs = [LayerSpec(ch[k], ch[k + 1], w.sh_order_lsc_in, w.sh_order_lsc_out, k < len(ch) - 2)
             for k in range(len(ch) - 1)]
    if weights is None:
        weights = [dg.lsc_weights(w.config, k, ch[k], ch[k + 1], 1 + sum(w.kernel_sizes)) for k in range(len(ch) - 1)]
    net = LSCNetwork(plan, plan, dg.lsc_sampled_gradients(w), specs, w.kernel_sizes, w.angular_distance,
                     w.lb_lambda, weights=weights, precision=precision, form=form, recompute=recompute,
                     device=device, max_batch=batch, bf16_activations=bf16_activations, relu_bits=relu_bits)
    return net, acq


def c4_batch(acq, index: int, V: int = 8192):
    """Batch `index`: a fresh distortion (<= 3 deg) of the nominal table and
    V voxels sampled on it.  Returns (distorted acquisition, x, clean)."""
    w = dg.C4
    dacq = dg.distort_acquisition(acq, 3.0, dg.rng_for(w.config, dg.STREAM_DISTORT, index))
    b = dg.stick_ball_batch(dacq, V, w.nf_max, w.snr, dg.rng_for(w.config, dg.STREAM_DATA, index), dtype=np.float32)
    return dacq, b.x, b.clean


# ------------------------------------------------------------ learned form

def learned_setup(train_voxels=None, eval_voxels=262144, precision="bf16", form="folded", device="cuda:0",
                  batch=8192, subset=15, bf16_activations=False, relu_bits=False):
    w = dg.C5
    acq = dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
    idx = [dg.farthest_point_subset(d, subset) for d in acq.shell_dirs]
    sub_dirs = [d[i] for d, i in zip(acq.shell_dirs, idx)]
    sub = dg.Acquisition(bvecs=np.concatenate([np.zeros((w.n_b0, 3))] + sub_dirs),
                         bvals=np.concatenate([np.zeros(w.n_b0)] + [np.full(subset, b) for b in w.shell_b]),
                         shell_b=list(w.shell_b), shell_dirs=sub_dirs, n_b0=w.n_b0)
    cols = np.concatenate([s * w.dirs_per_shell + i for s, i in enumerate(idx)])
    plan_in = SHPlan(sub.bvecs, sub.bvals, w.sh_order_lsc_in, w.lb_lambda)
    plan_out = SHPlan(acq.bvecs, acq.bvals, w.sh_order, w.lb_lambda)
    ch = w.channels
    specs = [LayerSpec(ch[0], ch[1], w.sh_order_lsc_in, w.sh_order_lsc_out, True)]
    specs += [LayerSpec(ch[k], ch[k + 1], w.sh_order_lsc_out, w.sh_order_lsc_out, k < len(ch) - 2)
              for k in range(1, len(ch) - 1)]
    weights = [dg.lsc_weights(w.config, k, ch[k], ch[k + 1], 1 + sum(w.kernel_sizes)) for k in range(len(ch) - 1)]
    net = LSCNetwork(plan_in, plan_out, dg.lsc_sampled_gradients(w), specs, w.kernel_sizes, w.angular_distance,
                     w.lb_lambda, weights=weights, precision=precision, form=form, device=device, max_batch=batch,
                     bf16_activations=bf16_activations, relu_bits=relu_bits)
    # the plain method: order-4 fit from the same subset, evaluated on the full table
    fit_in = SHPlan(sub.bvecs, sub.bvals, w.sh_order_lsc_in, w.lb_lambda)
    fit_in0 = SHPlan(sub.bvecs, sub.bvals, w.sh_order_lsc_in, 0.0)
    fit_out = SHPlan(acq.bvecs, acq.bvals, w.sh_order_lsc_in, 0.0)
    return dict(w=w, acq=acq, sub=sub, cols=cols, net=net, fit_in=fit_in, fit_in0=fit_in0, fit_out=fit_out)


def plain_fit(setup, x_sub: torch.Tensor, lam0=False) -> torch.Tensor:
    fin = setup["fit_in0"] if lam0 else setup["fit_in"]
    return sh2signal_fwd(setup["fit_out"], signal2sh_fwd(fin, x_sub))


def predict(setup, x_sub: torch.Tensor, batch=65536) -> torch.Tensor:
    net = setup["net"]
    out = torch.empty((x_sub.shape[0], net.plan_out.n_dw), dtype=torch.float32, device=x_sub.device)
    for lo in range(0, x_sub.shape[0], batch):
        hi = min(x_sub.shape[0], lo + batch)
        out[lo:hi] = net.forward(x_sub[lo:hi])
    return out


def run_learned(train_voxels=1 << 22, eval_voxels=262144, epochs=8, lr=2e-3, batch=8192, precision="bf16",
                form="folded", device="cuda:0", log=sys.stderr, bf16_activations=True, relu_bits=False):
    dev = torch.device(device)
    t0 = time.perf_counter()
    S = learned_setup(train_voxels, eval_voxels, precision, form, device, batch, bf16_activations=bf16_activations,
                      relu_bits=relu_bits)
    w, acq, cols, net = S["w"], S["acq"], S["cols"], S["net"]
    xtr, ctr = _gen(acq, train_voxels, w, dg.STREAM_DATA)
    xev, cev = _gen(acq, eval_voxels, w, dg.STREAM_HELDOUT)
    print(f"[learned] generated {train_voxels} + {eval_voxels} voxels in {time.perf_counter() - t0:.1f} s",
          file=log, flush=True)
    xs_tr = torch.from_numpy(np.ascontiguousarray(xtr[:, cols])).to(dev)
    y_tr = torch.from_numpy(ctr).to(dev)
    xs_ev = torch.from_numpy(np.ascontiguousarray(xev[:, cols])).to(dev)
    y_ev = torch.from_numpy(cev).to(dev)
    x_ev_full = torch.from_numpy(xev).to(dev)
    del xtr, ctr, xev, cev
    g = torch.Generator(device="cpu").manual_seed(w.config)
    nb = train_voxels // batch
    torch.cuda.synchronize()
    t_train = time.perf_counter()
    steps = 0
    for ep in range(epochs):
        perm = torch.randperm(train_voxels, generator=g)[: nb * batch].view(nb, batch).to(dev)
        lr_ep = lr * (0.5 ** (ep // max(1, epochs // 3)))
        for bi in range(nb):
            ids = perm[bi]
            net.train_step(xs_tr.index_select(0, ids), y_tr.index_select(0, ids), lr=lr_ep)
            steps += 1
        torch.cuda.synchronize()
        print(f"[learned] epoch {ep + 1}/{epochs} loss {float(net.loss):.6f} "
              f"({time.perf_counter() - t_train:.1f} s)", file=log, flush=True)
    train_s = time.perf_counter() - t_train
    final_loss = float(net.loss)  # evaluation below may reallocate the network's buffers
    torch.cuda.synchronize()
    t_inf = time.perf_counter()
    pred = predict(S, xs_ev)
    torch.cuda.synchronize()
    inf_s = time.perf_counter() - t_inf
    fit = plain_fit(S, xs_ev)
    fit0 = plain_fit(S, xs_ev, lam0=True)
    res = {
        "workload": w.name, "train_voxels": train_voxels, "eval_voxels": eval_voxels, "epochs": epochs,
        "batch": batch, "optimizer": f"Adam lr {lr} halved every {max(1, epochs // 3)} epochs", "precision": precision,
        "lsc_form": form, "relu_backward_mask": "bits" if net.relu_bits else "activation",
        "nrmse_net_vs_clean": nrmse(pred, y_ev), "nrmse_fit_vs_clean": nrmse(fit, y_ev),
        "nrmse_fit_lambda0_vs_clean": nrmse(fit0, y_ev),
        "nrmse_net_vs_noisy": nrmse(pred, x_ev_full), "nrmse_fit_vs_noisy": nrmse(fit, x_ev_full),
        "train_voxels_per_s": steps * batch / train_s, "inference_voxels_per_s": eval_voxels / inf_s,
        "final_train_loss": final_loss,
    }
    return res, S, net


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["learned"])
    ap.add_argument("--train-voxels", type=int, default=1 << 22)
    ap.add_argument("--eval-voxels", type=int, default=262144)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--form", default="folded")
    ap.add_argument("--relu-mask", choices=["bits", "activation"], default="activation")
    a = ap.parse_args()
    res, _, _ = run_learned(a.train_voxels, a.eval_voxels, a.epochs, a.lr, precision=a.precision, form=a.form,
                            relu_bits=a.relu_mask == "bits")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
