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
a second, instrumented pass over the same steps), the same for the other
precision under its own key ("bf16" when the line is FP32), the copy and
MFMA peaks measured on this GPU, and the FP64 CPU oracle timed on the host
cores (the stack on a fixed slice, on one thread, and the transforms alone).

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
    ap.add_argument("--single-precision", action="store_true",
                    help="time only --precision (default: the other precision of the same workload as well, "
                         "reported under its own key)")
    ap.add_argument("--no-peaks", action="store_true", help="skip the copy-kernel and MFMA-loop peak measurement")
    ap.add_argument("--fp32-activations", action="store_true",
                    help="BF16: keep the hidden LSC activations in float32 (default: bfloat16 storage)")
    ap.add_argument("--unfused-head", action="store_true",
                    help="run the loss head as SH2Signal, MSE and SH2Signal adjoint in three calls")
    ap.add_argument("--relu-mask", choices=["auto", "bits", "activation"], default="auto",
                    help="source of the hidden ReLU's backward mask: one bit per element written by the forward, or "
                         "the stored activation (auto: bits for the 1M-voxel step in both precisions; the activation "
                         "for the 8192-voxel four-layer step, whose activations stay in cache)")
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


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _median_time(fn, runs, warmup=1):
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), ts


def cpu_baseline(w, acq, x_all, slice_voxels=4096, chunk=1024, runs=5, one_thread_voxels=256):
    """The FP64 oracle, as it stands, timed on the host cores:
    * the stack forward + MSE + backward on a fixed slice of the workload
      (slice_voxels voxels in chunk-voxel pieces), median of `runs` after one
      warm-up: `value`, in the GPU line's unit;
    * the same on one thread (one_thread_voxels voxels, median of 3);
    * Signal2SH + SH2Signal alone on every voxel of the batch, median of
      `runs` after one warm-up."""
    import datagen as dg
    from oracle import lsc as olsc
    from oracle import sh as osh
    from oracle import stack as ostack
    from threadpoolctl import threadpool_info, threadpool_limits

    cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count() or 1])
    plan = osh.SHPlan(acq.bvecs, acq.bvals, w.sh_order, w.lb_lambda)
    g = dg.lsc_sampled_gradients(w)
    layers = []
    ch = w.channels
    for k in range(len(ch) - 1):
        p = olsc.LSCPlan(g, w.sh_order_lsc_in, w.sh_order_lsc_out, w.kernel_sizes, w.angular_distance, w.lb_lambda)
        W, b = dg.lsc_weights(w.config, k, ch[k], ch[k + 1], p.T)
        layers.append(ostack.Layer(p, W, b, k < len(ch) - 2))
    net = ostack.Stack(plan, layers, plan)
    batch = dg.stick_ball_batch(acq, slice_voxels, w.nf_max, w.snr, dg.rng_for(w.config, dg.STREAM_HELDOUT, 0))

    def stack(n, step):
        for lo in range(0, n, step):
            net.loss_and_grads(batch.x[lo:lo + step], batch.clean[lo:lo + step])

    t_stack, ts = _median_time(lambda: stack(slice_voxels, chunk), runs)
    with threadpool_limits(limits=1):
        t_one, _ = _median_time(lambda: stack(one_thread_voxels, one_thread_voxels), 3)
    V = x_all.shape[0]
    x64 = x_all.astype(np.float64)
    t_tr, _ = _median_time(lambda: osh.sh2signal(plan, osh.signal2sh(plan, x64)), runs)
    del x64
    return {"value": round(slice_voxels / t_stack, 2), "unit": "voxels/s", "cores": int(cores), "kind": "oracle",
            "sample": f"stack forward + MSE + backward (NumPy float64) on a fixed {slice_voxels}-voxel slice of "
                      f"the same workload in {chunk}-voxel chunks, median of {runs} runs after 1 warm-up "
                      f"({t_stack:.2f} s per run, {min(ts):.2f}-{max(ts):.2f} s)",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "one_thread": {"value": round(one_thread_voxels / t_one, 2), "unit": "voxels/s", "cores": 1,
                           "sample": f"{one_thread_voxels} voxels, median of 3 after 1 warm-up"},
            "transforms_only": {"value": round(V / t_tr, 1), "unit": "voxels/s", "cores": int(cores),
                                "sample": f"Signal2SH + SH2Signal on all {V} voxels, median of {runs} after 1 "
                                          f"warm-up ({t_tr:.2f} s per run)"}}


def measure_peaks(dev, copy_bytes=1 << 31, runs=5):
    """Copy-kernel bandwidth and MFMA-loop rates measured on this GPU (best
    of `runs` after a warm-up), beside the spec-sheet peaks."""
    import torch

    import paper_1808_01517_amd as dl

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(runs):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        return best

    src = torch.empty(copy_bytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    ms = timed(lambda: dl.peak_copy(src, dst))
    ok = bool(torch.equal(src, dst))
    del src, dst
    out = {"hbm_copy_GBs": round(2 * copy_bytes / (ms / 1e3) / 1e9, 1), "hbm_copy_bytes": 2 * copy_bytes,
           "copy_verified": ok, "spec_hbm_GBs": HBM_PEAK_GBS}
    blocks = 1024
    buf = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    for prec, iters in (("fp32", 20000), ("bf16", 20000)):
        flops = float(dl.lib().dlm_peak_mfma_flops(dl.precision_code(prec), blocks, iters))
        ms = timed(lambda: dl.peak_mfma(prec, blocks, iters, buf))
        out[f"{prec}_mfma_TFLOPs"] = round(flops / (ms / 1e3) / 1e12, 1)
        out[f"spec_{prec}_mfma_TFLOPs"] = MFMA_PEAK_TFLOPS[prec]
    return out


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


def c2_step(prec, form, args, plan, layers, ch, x, tgt, dev):
    """Buffers and the step function of the three-shell stack in one
    precision: forward, fused loss head, backward of every layer."""
    import torch

    import paper_1808_01517_amd as dl

    V = x.shape[0]
    S, K = plan.n_shells, plan.K
    f32 = dict(dtype=torch.float32, device=dev)
    # BF16: the hidden activations and their gradients are stored in bfloat16
    # (every contraction rounds them to bfloat16 on load, so no value changes)
    half = prec == "bf16" and form == "folded" and not args.fp32_activations
    act_dt = [torch.bfloat16 if half and 0 < k < len(layers) and (ch[k] * layers[k - 1][0].K_out) % 8 == 0
              else torch.float32 for k in range(len(layers) + 1)]
    acts = [torch.empty((V, S, K), **f32)] + [torch.empty((V, ch[k + 1], p.K_out), dtype=act_dt[k + 1], device=dev)
                                              for k, (p, _, _, _) in enumerate(layers)]
    grads = [torch.empty_like(a) for a in acts]
    # a hidden ReLU's backward mask travels as one bit per element
    use_bits = args.relu_mask in ("bits", "auto")
    bits = [dl.relu_bits_like(acts[k + 1]) if form == "folded" and relu and use_bits
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
    mse_ws = None if fused_head else torch.empty(dl.lib().dlm_mse_workspace_bytes(x.numel()), dtype=torch.uint8,
                                                 device=dev)
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

    config = {"precision": prec, "loss_head": "fused" if fused_head else "unfused",
              "hidden_activation_storage": "bf16" if torch.bfloat16 in act_dt else "f32",
              "relu_backward_mask": "bits" if any(b is not None for b in bits) else "activation"}
    return step, loss, config


def time_c2(step, loss, prec, form, args, V, full_size):
    """W untimed steps, then K steps between HIP events on the stream the
    library launches on; then (unless disabled) the same K steps again with
    the library's per-launch events for the per-kernel figures."""
    import torch

    import paper_1808_01517_amd as dl

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(st)
    for _ in range(args.steps):
        step()
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    out = {"value": round(V * args.steps / (ms_total / 1e3), 1), "ms_per_step": round(ms_step, 3)}
    print(f"[bench] {prec}: {args.steps} steps: {ms_step:.2f} ms/step (wall {wall / args.steps * 1e3:.2f} ms/step), "
          f"loss {float(loss):.5f}", file=sys.stderr, flush=True)
    if args.no_kernel_timing:
        return out
    dl.timing_reset()
    dl.timing_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dl.timing_enable(False)
    rep = dl.timing_report()
    peak = MFMA_PEAK_TFLOPS[prec]
    kern = {}
    for t, v in sorted(rep.items(), key=lambda kv: -kv[1][0]):
        sec = v[0] / 1e3
        kern[t] = {"ms_per_step": round(v[0] / args.steps, 3), "launches_per_step": v[1] // args.steps,
                   "GB/s": round(v[2] / sec / 1e9, 1) if sec > 0 else None,
                   "TFLOP/s": round(v[3] / sec / 1e12, 2) if sec > 0 else None,
                   "hbm_frac": round(v[2] / sec / 1e9 / HBM_PEAK_GBS, 3) if sec > 0 else None,
                   "mfma_frac": round(v[3] / sec / 1e12 / peak, 3) if sec > 0 else None}
    top = max(rep.items(), key=lambda kv: kv[1][0])
    out["roofline"] = roofline(top[0], *top[1], prec)
    if form == "folded" and full_size:
        # counters were taken on this workload in the folded form only
        out["roofline"]["traffic"] = measured_traffic(top[0], prec)
        out["roofline"]["traffic_source"] = os.path.relpath(TRAFFIC_FILE, ROOT)
    roof_s = sum(max(v[2] / (HBM_PEAK_GBS * 1e9), v[3] / (peak * 1e12)) for v in rep.values())
    out["step_roofline_frac"] = round(roof_s / args.steps / (ms_step / 1e3), 4)
    out["kernels"] = kern
    return out


def with_measured_peak(roof, peaks, prec):
    """The roofline's achieved rate also against the peak measured on this GPU."""
    if not roof or not peaks:
        return roof
    key = "hbm_copy_GBs" if roof["bound"] == "hbm" else f"{prec}_mfma_TFLOPs"
    roof["measured_peak"] = peaks[key]
    roof["frac_of_measured_peak"] = round(roof["achieved"] / peaks[key], 4)
    return roof


def main():
    args = parse()
    if args.workload in ("c4", "sweep"):
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        (bench_c4 if args.workload == "c4" else bench_sweep)(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the layers are per-voxel and the benchmark "
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
    form = args.form
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
    del clean_h
    full_size = V == w.voxels

    step, loss, cfg = c2_step(prec, form, args, plan, layers, ch, x, tgt, dev)
    main_res = time_c2(step, loss, prec, form, args, V, full_size)
    del step
    result = {
        "metric": METRIC, "value": main_res["value"], "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main_res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == "fp32" else "bf16", "data": "synthetic",
        "config": {"workload": w.name, "voxels": V, "shells": len(w.shell_b), "dirs_per_shell": w.dirs_per_shell,
                   "b0_volumes": w.n_b0, "sh_order": w.sh_order, "lsc_channels": list(ch),
                   "kernel_sizes": list(w.kernel_sizes), "angular_distance_deg": 30.0, "lsc_form": form,
                   "lsc_chunk_voxels": min(V, args.chunk), **cfg},
    }
    for k in ("roofline", "step_roofline_frac", "kernels"):
        if k in main_res:
            result[k] = main_res[k]
    if not args.single_precision:
        # the other precision of the same workload, same data, same run
        other = "bf16" if prec == "fp32" else "fp32"
        torch.cuda.empty_cache()
        step, loss, cfg_o = c2_step(other, form, args, plan, layers, ch, x, tgt, dev)
        res_o = time_c2(step, loss, other, form, args, V, full_size)
        del step
        res_o = {"dtype": "f32" if other == "fp32" else "bf16", **res_o, "config": cfg_o}
        result[other] = res_o
    del x, tgt
    torch.cuda.empty_cache()
    if not args.no_peaks:
        peaks = measure_peaks(dev)
        result["measured_peaks"] = peaks
        with_measured_peak(result.get("roofline"), peaks, prec)
        for other in ("fp32", "bf16"):
            if other in result:
                with_measured_peak(result[other].get("roofline"), peaks, other)
    if args.with_copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes_per_dispatch"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        del src, dst
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host cores", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w, acq, x_h)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
