"""The allocation-free fused loss head (dlm_sh2signal_mse_fwd_bwd_noalloc)
against the workspace entry point (dlm_sh2signal_mse_fwd_bwd) through the C
ABI: bitwise the same loss, gradient and signal, on two calls in a row (the
second with a smaller batch, so it runs over what the first left in the
shared static array), on shells of unequal size, and the FP64 oracle's
bounds; sizes beyond the static array are refused."""
import ctypes as C

import numpy as np
import pytest
import torch

import datagen as dg
import paper_1808_01517_amd as dl
from paper_1808_01517_amd._lib import DLM_BF16, DLM_EWORKSPACE, DLM_FP32, DLM_OK
from oracle import sh as osh
from oracle import stack as ostack
from parity_util import TOL, check

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _p(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _mixed_acquisition():
    dirs = [dg.perturb_directions(dg.fibonacci_hemisphere(n), 2.0, dg.rng_for(61, 1, s))
            for s, n in enumerate((17, 45, 96))]
    shell_b = [1000.0, 2000.0, 3000.0]
    bvecs = np.concatenate([np.zeros((2, 3))] + dirs)
    bvals = np.concatenate([np.zeros(2)] + [np.full(d.shape[0], b) for b, d in zip(shell_b, dirs)])
    return dg.Acquisition(bvecs=bvecs, bvals=bvals, shell_b=shell_b, shell_dirs=dirs, n_b0=2)


def _run_both(plan, c, tgt, prec):
    lib = dl.lib()
    V = c.shape[0]
    pc = DLM_BF16 if prec == "bf16" else DLM_FP32
    loss_a = torch.empty((), device=DEV)
    dc_a = torch.empty_like(c)
    x_a = torch.empty_like(tgt)
    ws = torch.empty(lib.dlm_sh2signal_mse_workspace_bytes(plan.handle, V), dtype=torch.uint8, device=DEV)
    st = lib.dlm_sh2signal_mse_fwd_bwd(plan.handle, _p(c), _p(tgt), V, _p(loss_a), _p(dc_a), _p(x_a), _p(ws),
                                       ws.numel(), pc, _stream())
    assert st == DLM_OK, lib.dlm_last_error()
    loss_b = torch.full((), 7.0, device=DEV)
    dc_b = torch.full_like(c, 7.0)
    x_b = torch.full_like(tgt, 7.0)
    st = lib.dlm_sh2signal_mse_fwd_bwd_noalloc(plan.handle, _p(c), _p(tgt), V, _p(loss_b), _p(dc_b), _p(x_b), pc,
                                                _stream())
    assert st == DLM_OK, lib.dlm_last_error()
    torch.cuda.synchronize()
    return (loss_a, dc_a, x_a), (loss_b, dc_b, x_b)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("table", ["c2", "mixed"])
def test_noalloc_loss_head_matches_workspace_entry_point(prec, table):
    if table == "c2":
        w = dg.C2
        acq = dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
    else:
        acq = _mixed_acquisition()
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
    for V in (3000 + 13, 1000 + 7):  # the second call is smaller
        batch = dg.stick_ball_batch(acq, V, 3, 20.0, dg.rng_for(62, 2, V))
        other = dg.stick_ball_batch(acq, V, 3, 20.0, dg.rng_for(62, 2, V + 1))
        c64 = osh.signal2sh(oplan, batch.x).astype(np.float32).astype(np.float64)
        t64 = other.clean.astype(np.float32).astype(np.float64)
        (la, dca, xa), (lb, dcb, xb) = _run_both(plan, cuda(c64), cuda(t64), prec)
        assert lb.item() == la.item()
        assert torch.equal(dcb, dca) and torch.equal(xb, xa)
        xr = osh.sh2signal(oplan, c64)
        l_ref, dxh = ostack.mse(xr, t64)
        check("xhat", xb, xr, prec)
        check("dc", dcb, osh.sh2signal_adjoint(oplan, dxh), prec)
        assert abs(lb.item() - l_ref) / l_ref <= TOL[prec]


def test_noalloc_loss_head_refuses_batches_beyond_its_scratch():
    w = dg.C2
    acq = dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
    lib = dl.lib()
    cap = lib.dlm_sh2signal_mse_static_scratch_bytes()
    assert cap == 4 << 20
    # the largest batch that fits (the workspace grows with V), and one more
    # 16-voxel tile
    lo, hi = 16, 16
    while lib.dlm_sh2signal_mse_workspace_bytes(plan.handle, hi) <= cap:
        lo, hi = hi, 2 * hi
    while hi - lo > 16:
        mid = (lo + hi) // 32 * 16
        if lib.dlm_sh2signal_mse_workspace_bytes(plan.handle, mid) <= cap:
            lo = mid
        else:
            hi = mid
    V = lo
    assert lib.dlm_sh2signal_mse_workspace_bytes(plan.handle, V) <= cap
    assert lib.dlm_sh2signal_mse_workspace_bytes(plan.handle, V + 16) > cap
    assert V > 5_000_000  # a million-voxel batch fits many times over
    dummy = torch.zeros(16, device=DEV)
    st = lib.dlm_sh2signal_mse_fwd_bwd_noalloc(plan.handle, _p(dummy), _p(dummy), V + 16, _p(dummy), _p(dummy), None,
                                                DLM_FP32, _stream())
    assert st == DLM_EWORKSPACE
    assert b"static scratch" in lib.dlm_last_error()
