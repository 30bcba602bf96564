#!/usr/bin/env python3
"""Throughput of the DELIMIT hot path on one MI355X.

One step = forward + backward of the three-shell stack over 1,048,576
synthetic voxels resident in HBM:
  Signal2SH (3 shells x 90 directions, SH order 8)
  -> LSC 3->32 (two rings of 8 points, 30 deg) -> ReLU -> LSC 32->3
  -> SH2Signal -> q-space MSE against the noise-free signal
  -> backward through every layer (input, weight and bias gradients).

Prints one JSON line: voxels/s, the roofline position of the dominant
kernel (per-launch durations from HIP events recorded by the library during
a second, instrumented pass over the same steps), and the FP64 CPU oracle
timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--precision fp32|bf16]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxels/s fwd+bwd Signal2SH+LSC+SH2Signal, 3×90 dirs, L=8; % roofline"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["c2", "c4", "sweep"], default="c2",
                    help="c2: three-shell stack fwd+bwd over 2^20 voxels (the headline); "
                         "c4: four-layer training step (fwd, MSE, bwd, Adam) on 8192-voxel batches")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="fp32")
    ap.add_argument("--form", choices=["folded", "resample"], default="folded",
                    help="LSC evaluation: folded linear map, or the paper's resample/row-dot/refit order")
    ap.add_argument("--voxels", type=int, default=None, help="override the voxel count (default: the workload's)")
    ap.add_argument("--chunk", type=int, default=1 << 17, help="LSC voxels per workspace pass")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--fp32-activations", action="store_true",
                    help="BF16: keep the hidden LSC activations in float32 (default: bfloat16 storage)")
    ap.add_argument("--unfused-head", action="store_true",
                    help="run the loss head as SH2Signal, MSE and SH2Signal adjoint in three calls")
    ap.add_argument("--relu-mask", choices=["auto", "bits", "activation"], default="auto",
                    help="source of the hidden ReLU's backward mask: one bit per element written by the forward, or "
                         "the stored activation (auto: bits for the 1M-voxel BF16 step, which is memory-bound; the "
                         "activation in FP32, where the extra epilogue work costs more than the saved reads, and for "
                         "the 8192-voxel four-layer step, whose activations stay in cache)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--with-copy-calibration", action="store_true",
                    help="after the timed steps, copy a 1 GiB buffer 3 times (reference for HBM byte counters)")
    return ap.parse_args()


def make_data(w, V, chunk=1 << 16):
    import datagen as dg

    acq = dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
    n = acq.dw_bvecs.shape[0]
    x = np.empty((V, n), dtype=np.float32)
    clean = np.empty((V, n), dtype=np.float32)

    def one(ci):
        lo = ci * chunk
        hi = min(V, lo + chunk)
        b = dg.stick_ball_batch(acq, hi - lo, w.nf_max, w.snr, dg.rng_for(w.config, dg.STREAM_DATA, ci),
                                dtype=np.float32)
        x[lo:hi] = b.x
        clean[lo:hi] = b.clean

    nchunks = (V + chunk - 1) // chunk
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        list(ex.map(one, range(nchunks)))
    return acq, x, clean


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_stack_folded_hbm_traffic.txt")


def kernel_source_hash():
    """sha256 prefix of the library's kernel and launch sources (as recorded with the counters)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1808_01517_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(tag, prec):
    """HBM bytes per launch of `tag` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, or None when that summary was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    except OSError:
        return None
    recorded = next((ln[1] for ln in lines if ln[0] == "source_sha256"), None)
    if recorded != kernel_source_hash():
        return None
    for ln in lines:
        if ln[0] == "traffic" and ln[1] == prec and ln[2] == tag:
            return float(ln[3])
    return None


def roofline(tag, ms, launches, nbytes, flops, prec):
    t = ms / 1e3
    hbm_time = nbytes / (HBM_PEAK_GBS * 1e9)
    mfma_time = flops / (MFMA_PEAK_TFLOPS[prec] * 1e12)
    if mfma_time > hbm_time:
        ach = flops / t / 1e12
        return {"kernel": tag, "bound": "mfma", "achieved": round(ach, 2), "peak": MFMA_PEAK_TFLOPS[prec],
                "unit": "TFLOP/s", "frac": round(ach / MFMA_PEAK_TFLOPS[prec], 4), "traffic": None,
                "launches": launches, "avg_launch_ms": round(ms / launches, 4),
                "alg_flops_per_launch": flops / launches, "alg_bytes_per_launch": nbytes / launches}
    ach = nbytes / t / 1e9
    return {"kernel": tag, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "launches": launches,
            "avg_launch_ms": round(ms / launches, 4), "alg_bytes_per_launch": nbytes / launches,
            "alg_flops_per_launch": flops / launches}


def cpu_baseline(w, acq, target_s):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload."""
    import datagen as dg
    from oracle import lsc as olsc
    from oracle import sh as osh
    from oracle import stack as ostack

    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover - threadpoolctl is optional
        cores = os.cpu_count() or 1
    plan = osh.SHPlan(acq.bvecs, acq.bvals, w.sh_order, w.lb_lambda)
    g = dg.lsc_sampled_gradients(w)
    layers = []
    ch = w.channels
    for k in range(len(ch) - 1):
        p = olsc.LSCPlan(g, w.sh_order_lsc_in, w.sh_order_lsc_out, w.kernel_sizes, w.angular_distance, w.lb_lambda)
        W, b = dg.lsc_weights(w.config, k, ch[k], ch[k + 1], p.T)
        layers.append(ostack.Layer(p, W, b, k < len(ch) - 2))
    net = ostack.Stack(plan, layers, plan)
    nmax = 16384
    batch = dg.stick_ball_batch(acq, nmax, w.nf_max, w.snr, dg.rng_for(w.config, dg.STREAM_HELDOUT, 0))
    t0 = time.perf_counter()
    net.loss_and_grads(batch.x[:128], batch.clean[:128])
    per_vox = (time.perf_counter() - t0) / 128
    n = int(min(nmax, max(256, target_s / max(per_vox, 1e-9))))
    n = (n // 256) * 256
    t0 = time.perf_counter()
    for lo in range(0, n, 1024):
        hi = min(n, lo + 1024)
        net.loss_and_grads(batch.x[lo:hi], batch.clean[lo:hi])
    dt = time.perf_counter() - t0
    return {"value": round(n / dt, 2), "unit": "voxels/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n} voxels of the same workload (stack forward + MSE + backward), NumPy float64, "
                      f"1024-voxel chunks, {dt:.1f} s"}


def bench_c4(args):
    """Training steps of the four-layer network; each batch has its own
    distorted gradient table (plan tables rebuilt in float64 and uploaded on
    the stream) and its own voxels; layers 1 and 3 recompute their outputs."""
    import torch

    import datagen as dg
    from paper_1808_01517_amd import apps

    dev = torch.device("cuda:0")
    prec, form = args.precision, args.form
    w = dg.C4
    B = w.voxels
    half = prec == "bf16" and form == "folded" and not args.fp32_activations
    bits = args.relu_mask == "bits"  # auto: the activation mask at 8 192-voxel batches
    net, acq = apps.c4_network(prec, form, recompute=(0, 2), batch=B, bf16_activations=half, relu_bits=bits)
    nb = 8
    batches = []
    for i in range(nb):
        dacq, x, clean = apps.c4_batch(acq, i, B)
        batches.append((dacq.bvecs, torch.from_numpy(x).to(dev), torch.from_numpy(clean).to(dev)))

    def step(i):
        bvecs, x, clean = batches[i % nb]
        net.plan_in.update_gradients(bvecs)
        net.train_step(x, clean, lr=1e-4)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for i in range(args.steps):
        step(args.warmup + i)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    result = {"metric": "voxels/s training step (fwd + MSE + bwd + Adam), 4-layer LSC 3-32-64-32-3, 3x90 dirs, L=8",
              "value": round(B / (ms / 1e3), 1), "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f32" if prec == "fp32" else "bf16", "data": "synthetic",
              "config": {"workload": w.name, "batch": B, "lsc_channels": list(w.channels), "sh_order": w.sh_order,
                         "distortion_deg": 3.0, "recompute_layers": [1, 3], "lsc_form": form, "precision": prec,
                         "hidden_activation_storage": "bf16" if half else "f32",
                         "relu_backward_mask": "bits" if net.relu_bits else "activation"}}
    if not args.no_kernel_timing:
        import paper_1808_01517_amd as dl
        dl.timing_reset()
        dl.timing_enable(True)
        for i in range(args.steps):
            step(i)
        torch.cuda.synchronize()
        dl.timing_enable(False)
        rep = dl.timing_report()
        top = max(rep.items(), key=lambda kv: kv[1][0])
        result["roofline"] = roofline(top[0], *top[1], prec)
        result["kernels"] = {t: {"ms_per_step": round(v[0] / args.steps, 4), "launches_per_step": v[1] // args.steps}
                             for t, v in sorted(rep.items(), key=lambda kv: -kv[1][0])}
    print(json.dumps(result), flush=True)


def bench_sweep(args):
    """Transform-only order sweep (the paper's Fig. 1 experiment re-done):
    Signal2SH then SH2Signal on the three-shell table at SH orders 2..12,
    450 000 synthetic voxels (about one brain scan), FP32 and BF16, next to
    the FP64 oracle on the host cores.  One JSON line with a row per order."""
    import torch

    import datagen as dg
    import paper_1808_01517_amd as dl
    from oracle import sh as osh

    dev = torch.device("cuda:0")
    w = dg.C2
    V = args.voxels or 450_000
    acq, x_h, _ = make_data(w, V)
    x = torch.from_numpy(x_h).to(dev)
    rows = []
    for L in (2, 4, 6, 8, 10, 12):
        plan = dl.SHPlan(acq.bvecs, acq.bvals, L, w.lb_lambda)
        c = torch.empty((V, plan.n_shells, plan.K), dtype=torch.float32, device=dev)
        xr = torch.empty_like(x)
        row = {"sh_order": L, "K": plan.K}
        # oracle on the host: the same round trip in float64 on a bounded sample
        n = min(V, 32768)
        oplan = osh.SHPlan(acq.bvecs, acq.bvals, L, w.lb_lambda)
        xs = x_h[:n].astype(np.float64)
        t0 = time.perf_counter()
        xo = osh.sh2signal(oplan, osh.signal2sh(oplan, xs))
        tc = time.perf_counter() - t0
        row["oracle_voxels_per_s"] = round(n / tc, 1)
        for prec in ("fp32", "bf16"):
            def rt():
                dl.signal2sh_fwd(plan, x, out=c, precision=prec)
                dl.sh2signal_fwd(plan, c, out=xr, precision=prec)
            for _ in range(args.warmup):
                rt()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                rt()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            dl.timing_reset()
            dl.timing_enable(True)
            rt()
            torch.cuda.synchronize()
            dl.timing_enable(False)
            rep = dl.timing_report()
            nbytes = sum(v[2] for v in rep.values())
            err = float(np.linalg.norm(xr[:n].double().cpu().numpy() - xo) / np.linalg.norm(xo))
            row[prec] = {"ms": round(ms, 4), "voxels_per_s": round(V / (ms / 1e3), 1),
                         "hbm_frac": round(nbytes / (ms / 1e3) / (HBM_PEAK_GBS * 1e9), 4),
                         "rel_err_vs_oracle": err}
        rows.append(row)
        print(f"[sweep] L={L} K={plan.K}: fp32 {row['fp32']['ms']:.3f} ms, bf16 {row['bf16']['ms']:.3f} ms, "
              f"oracle {row['oracle_voxels_per_s']:.0f} voxels/s", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "voxels/s Signal2SH + SH2Signal round trip by SH order", "unit": "voxels/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "data": "synthetic",
                      "config": {"workload": "order-sweep-3shell-90dir", "voxels": V, "shells": 3,
                                 "dirs_per_shell": 90, "lb_lambda": w.lb_lambda,
                                 "oracle_sample_voxels": min(V, 32768),
                                 "oracle_threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))},
                      "rows": rows}), flush=True)


def main():
    args = parse()
    if args.workload in ("c4", "sweep"):
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        (bench_c4 if args.workload == "c4" else bench_sweep)(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the layers are per-voxel and this build "
              "measures a single GPU's share; see the sharding notes in the design document.", file=sys.stderr)
        sys.exit(2)
    import torch

    import datagen as dg
    import paper_1808_01517_amd as dl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = dg.C2
    V = args.voxels or w.voxels
    prec = args.precision
    t_gen = time.perf_counter()
    acq, x_h, clean_h = make_data(w, V)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] generated {V} voxels x {x_h.shape[1]} dirs in {t_gen:.1f} s", file=sys.stderr, flush=True)

    plan = dl.SHPlan(acq.bvecs, acq.bvals, w.sh_order, w.lb_lambda)
    g = dg.lsc_sampled_gradients(w)
    ch = w.channels
    layers = []
    for k in range(len(ch) - 1):
        p = dl.LSCPlan(g, w.sh_order_lsc_in, w.sh_order_lsc_out, w.kernel_sizes, w.angular_distance, w.lb_lambda)
        W, b = dg.lsc_weights(w.config, k, ch[k], ch[k + 1], p.T)
        layers.append((p, torch.from_numpy(W.astype(np.float32)).to(dev), torch.from_numpy(b.astype(np.float32)).to(dev),
                       k < len(ch) - 2))
    x = torch.from_numpy(x_h).to(dev)
    tgt = torch.from_numpy(clean_h).to(dev)
    del x_h, clean_h
    S, K = plan.n_shells, plan.K
    f32 = dict(dtype=torch.float32, device=dev)
    # BF16: the hidden activations and their gradients are stored in bfloat16
    # (every contraction rounds them to bfloat16 on load, so no value changes)
    half = prec == "bf16" and args.form == "folded" and not args.fp32_activations
    act_dt = [torch.bfloat16 if half and 0 < k < len(layers) and (ch[k] * layers[k - 1][0].K_out) % 8 == 0
              else torch.float32 for k in range(len(layers) + 1)]
    acts = [torch.empty((V, S, K), **f32)] + [torch.empty((V, ch[k + 1], p.K_out), dtype=act_dt[k + 1], device=dev)
                                              for k, (p, _, _, _) in enumerate(layers)]
    grads = [torch.empty_like(a) for a in acts]
    # a hidden ReLU's backward mask travels as one bit per element
    use_bits = args.relu_mask == "bits" or (args.relu_mask == "auto" and prec == "bf16")
    bits = [dl.relu_bits_like(acts[k + 1]) if args.form == "folded" and relu and use_bits
            and (ch[k + 1] * p.K_out) % 16 == 0 else None for k, (p, _, _, relu) in enumerate(layers)]
    bits = [None] + bits
    fused_head = dl.sh2signal_mse_supported(plan) and not args.unfused_head
    xhat = None if fused_head else torch.empty_like(x)
    dxhat = None if fused_head else torch.empty_like(x)
    head_ws = torch.empty(dl.lib().dlm_sh2signal_mse_workspace_bytes(plan.handle, V), dtype=torch.uint8, device=dev)
    dx = torch.empty_like(x)
    dWs = [torch.empty_like(Wk) for _, Wk, _, _ in layers]
    dbs = [torch.empty_like(bk) for _, _, bk, _ in layers]
    loss = torch.empty((), **f32)
    mse_ws = torch.empty(dl.lib().dlm_mse_workspace_bytes(x.numel()), dtype=torch.uint8, device=dev)
    form = args.form
    ws_bytes = max(dl.lsc_workspace_bytes(p, ch[k], ch[k + 1], min(V, args.chunk), prec, form)
                   for k, (p, _, _, _) in enumerate(layers))
    ws = dl.Workspace(ws_bytes, dev)

    def step():
        dl.signal2sh_fwd(plan, x, out=acts[0], precision=prec)
        for k, (p, Wk, bk, relu) in enumerate(layers):
            dl.lsc_fwd(p, acts[k], Wk, bk, relu=relu, out=acts[k + 1], precision=prec, workspace=ws, form=form,
                       relu_bits=bits[k + 1])
        if fused_head:  # x^ and its gradient never go through HBM
            dl.sh2signal_mse_fwd_bwd(plan, acts[-1], tgt, precision=prec, outs=(loss, grads[-1], head_ws))
        else:
            dl.sh2signal_fwd(plan, acts[-1], out=xhat, precision=prec)
            dl.mse_fwd_bwd(xhat, tgt, outs=(loss, dxhat, mse_ws))
            dl.sh2signal_bwd(plan, dxhat, out=grads[-1], precision=prec)
        for k in range(len(layers) - 1, -1, -1):
            p, Wk, bk, relu = layers[k]
            # the ReLU after layer k-1 is applied by layer k's adjoint as it writes grads[k]
            relu_in = k > 0 and layers[k - 1][3]
            relu_out = relu and k == len(layers) - 1
            dl.lsc_bwd(p, acts[k], Wk, grads[k + 1], a_out=acts[k + 1], relu=relu_out, relu_in=relu_in,
                       precision=prec, workspace=ws, outs=(grads[k], dWs[k], dbs[k]), form=form,
                       relu_bits=bits[k] if relu_in else None)
        dl.signal2sh_bwd(plan, grads[0], out=dx, precision=prec)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(st)
    for _ in range(args.steps):
        step()
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    value = V * args.steps / (ms_total / 1e3)
    print(f"[bench] {args.steps} steps: {ms_step:.2f} ms/step (wall {wall / args.steps * 1e3:.2f} ms/step), "
          f"loss {float(loss):.5f}", file=sys.stderr, flush=True)

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == "fp32" else "bf16", "data": "synthetic",
        "config": {"workload": w.name, "voxels": V, "shells": len(w.shell_b), "dirs_per_shell": w.dirs_per_shell,
                   "b0_volumes": w.n_b0, "sh_order": w.sh_order, "lsc_channels": list(ch),
                   "kernel_sizes": list(w.kernel_sizes), "angular_distance_deg": 30.0, "lsc_form": form,
                   "precision": prec, "lsc_chunk_voxels": min(V, args.chunk),
                   "loss_head": "fused" if fused_head else "unfused",
                   "hidden_activation_storage": "bf16" if torch.bfloat16 in act_dt else "f32",
                   "relu_backward_mask": "bits" if any(b is not None for b in bits) else "activation"},
    }

    if not args.no_kernel_timing:
        dl.timing_reset()
        dl.timing_enable(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        dl.timing_enable(False)
        rep = dl.timing_report()
        kern = {t: {"ms_per_step": round(v[0] / args.steps, 3), "launches_per_step": v[1] // args.steps,
                    "GB/s": round(v[2] / (v[0] / 1e3) / 1e9, 1) if v[0] > 0 else None,
                    "TFLOP/s": round(v[3] / (v[0] / 1e3) / 1e12, 2) if v[0] > 0 else None}
                for t, v in sorted(rep.items(), key=lambda kv: -kv[1][0])}
        top = max(rep.items(), key=lambda kv: kv[1][0])
        result["roofline"] = roofline(top[0], *top[1], prec)
        if form == "folded" and V == w.voxels:
            # counters were taken on this workload in the folded form only
            result["roofline"]["traffic"] = measured_traffic(top[0], prec)
            result["roofline"]["traffic_source"] = os.path.relpath(TRAFFIC_FILE, ROOT)
        roof_s = sum(max(v[2] / (HBM_PEAK_GBS * 1e9), v[3] / (MFMA_PEAK_TFLOPS[prec] * 1e12)) for v in rep.values())
        result["step_roofline_frac"] = round(roof_s / args.steps / (ms_step / 1e3), 4)
        result["kernels"] = kern
    if args.with_copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes_per_dispatch"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        del src, dst
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, acq, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
