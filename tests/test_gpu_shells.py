"""GPU parity of the SH transforms on multi-shell tables whose shells differ
in size (Sec. 2.3.1: several b-values, each shell its own gradient table),
and of plans that only evaluate the basis (Sec. 2.2: SH2Signal onto any N
resampled directions, also fewer than the K coefficients).

Shells of unequal size take a different launch sequence from the uniform
three-shell table: one launch per shell with per-shell signal, coefficient
and table offsets.  The tables interleave the shells' volumes and the b0
volumes, so the shell-major reordering and the b0 gather of the fused
normalisation are exercised too.  Voxel counts leave ragged tiles.
"""
import numpy as np
import pytest
import torch

import datagen as dg
import paper_1808_01517_amd as dl
from paper_1808_01517_amd._lib import DLM_ESINGULAR, DLM_OK
from paper_1808_01517_amd.layers import SH2Signal
from oracle import sh as osh
from oracle import stack as ostack
from parity_util import check, fmt, rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# (shell b-values, directions per shell, b0 volumes, seed)
CASES = {
    "17-45-96": ((1000.0, 2000.0, 3000.0), (17, 45, 96), 3, 41),
    "30-60": ((700.0, 2500.0), (30, 60), 2, 42),
}


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _interleave(shell_b, sd, labels):
    bvecs = np.zeros((labels.size, 3))
    bvals = np.zeros(labels.size)
    nxt = [0] * len(sd)
    for i, s in enumerate(labels):
        if s >= 0:
            bvecs[i] = sd[s][nxt[s]]
            bvals[i] = shell_b[s]
            nxt[s] += 1
    return bvecs, bvals


def interleaved_acquisition(shell_b, dirs, n_b0, seed):
    """Shells of the given sizes plus b0 volumes in a seeded interleaved
    table order; each shell's volumes keep their relative order, so the
    plan's shell-major layout lists shell s as shell_dirs[s]."""
    sd = [dg.perturb_directions(dg.fibonacci_hemisphere(n), 2.0, dg.rng_for(seed, 1, s))
          for s, n in enumerate(dirs)]
    labels = np.concatenate([np.full(n_b0, -1)] + [np.full(n, s) for s, n in enumerate(dirs)])
    labels = dg.rng_for(seed, 1, 99).permutation(labels)
    bvecs, bvals = _interleave(shell_b, sd, labels)
    acq = dg.Acquisition(bvecs=bvecs, bvals=bvals, shell_b=list(shell_b), shell_dirs=sd, n_b0=n_b0)
    return acq, labels


def raw_volumes(batch, labels, scale=640.0):
    """Raw signal in table order: b0 volumes and S0-scaled diffusion-weighted
    volumes interleaved as the table lists them."""
    V = batch.x.shape[0]
    s0 = batch.raw_b0.mean(axis=1, keepdims=True)
    dw = batch.x * s0
    raw = np.empty((V, labels.size))
    raw[:, labels < 0] = batch.raw_b0
    raw[:, labels >= 0] = 0.0
    # shell-major column of each table position
    counts = [int((labels == s).sum()) for s in range(labels.max() + 1)]
    offs = np.concatenate([[0], np.cumsum(counts)])
    nxt = [0] * len(counts)
    for i, s in enumerate(labels):
        if s >= 0:
            raw[:, i] = dw[:, offs[s] + nxt[s]]
            nxt[s] += 1
    return raw * scale


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("L", [4, 8])
@pytest.mark.parametrize("case", list(CASES))
def test_unequal_shells_transforms(prec, L, case):
    shell_b, dirs, n_b0, seed = CASES[case]
    acq, labels = interleaved_acquisition(shell_b, dirs, n_b0, seed)
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    assert plan.has_fit and oplan.has_fit
    assert [s[0] for s in plan.shells] == list(dirs) == oplan.dirs
    for s in range(len(dirs)):
        assert np.array_equal(plan.shells[s][2], oplan.shell_idx[s])
    V = 1000 + 7
    batch = dg.stick_ball_batch(acq, V, 3, 20.0, dg.rng_for(seed, 2, L))
    x = batch.x.astype(np.float32).astype(np.float64)
    errs = {}
    c = dl.signal2sh_fwd(plan, cuda(x), precision=prec)
    check("c", c, osh.signal2sh(oplan, x), prec, errs)
    xr = dl.sh2signal_fwd(plan, c, precision=prec)
    check("x", xr, osh.sh2signal(oplan, c.double().cpu().numpy()), prec, errs)
    rng = np.random.default_rng(seed + L)
    dc = rng.standard_normal((V, len(dirs), plan.K)).astype(np.float32).astype(np.float64)
    check("s2sh_bwd", dl.signal2sh_bwd(plan, cuda(dc), precision=prec), osh.signal2sh_adjoint(oplan, dc), prec, errs)
    dx = rng.standard_normal((V, plan.n_dw)).astype(np.float32).astype(np.float64)
    check("sh2s_bwd", dl.sh2signal_bwd(plan, cuda(dx), precision=prec), osh.sh2signal_adjoint(oplan, dx), prec, errs)
    # b0 normalisation fused into the load, raw volumes in table order
    raw = raw_volumes(batch, labels).astype(np.float32).astype(np.float64)
    c_raw = dl.signal2sh_fwd_raw(plan, cuda(raw), precision=prec)
    check("c_raw", c_raw, osh.signal2sh(oplan, osh.normalize_b0(raw, acq.bvals, oplan)), prec, errs)
    print(f"[parity] shells {case} order {L} {prec}: " + fmt(errs), flush=True)


@pytest.mark.parametrize("case", list(CASES))
def test_unequal_shells_update_gradients(case):
    """A fresh seeded distortion of every direction, rebuilt in float64 and
    uploaded in stream order, gives the fresh oracle plan's results."""
    shell_b, dirs, n_b0, seed = CASES[case]
    acq, labels = interleaved_acquisition(shell_b, dirs, n_b0, seed)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
    V = 500 + 3
    x = dg.stick_ball_batch(acq, V, 3, 20.0, dg.rng_for(seed, 2, 5)).x.astype(np.float32).astype(np.float64)
    xg = cuda(x)
    c_old = dl.signal2sh_fwd(plan, xg)
    dirs_new = dg.distort_acquisition(acq, 3.0, dg.rng_for(seed, dg.STREAM_DISTORT, 1)).shell_dirs
    bvecs_new, bvals_new = _interleave(shell_b, dirs_new, labels)  # the same table order
    assert np.array_equal(bvals_new, acq.bvals)
    plan.update_gradients(bvecs_new)
    oplan = osh.SHPlan(bvecs_new, bvals_new, 8, 0.006)
    for prec in ("fp32", "bf16"):
        c = dl.signal2sh_fwd(plan, xg, precision=prec)
        check("c", c, osh.signal2sh(oplan, x), prec)
        check("x", dl.sh2signal_fwd(plan, c, precision=prec), osh.sh2signal(oplan, c.double().cpu().numpy()), prec)
    assert rel(c_old, osh.signal2sh(oplan, x)) > 1e-4  # the tables really changed


def _eval_only_acq(dirs, seed):
    sd = [dg.perturb_directions(dg.fibonacci_hemisphere(n), 2.0, dg.rng_for(seed, 1, s)) for s, n in enumerate(dirs)]
    shell_b = [1000.0 * (s + 1) for s in range(len(dirs))]
    bvecs = np.concatenate(sd)
    bvals = np.concatenate([np.full(n, b) for n, b in zip(dirs, shell_b)])
    return dg.Acquisition(bvecs=bvecs, bvals=bvals, shell_b=shell_b, shell_dirs=sd, n_b0=0)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("dirs", [(30,), (17, 30), (17, 60)])
def test_sh2signal_onto_fewer_directions_than_coefficients(prec, dirs):
    """Order 8 (K = 45) at lambda = 0 onto shells of 17, 30 or 60 directions:
    every shell with N < K has no fit (in (17, 60) one shell does and one
    does not).  The plan evaluates: SH2Signal, its adjoint and the fused
    loss head match the oracle; every call that needs the fit is refused
    with DLM_ESINGULAR before any launch."""
    acq = _eval_only_acq(dirs, 51)
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, 8, 0.0)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, 8, 0.0)
    assert not plan.has_fit and not oplan.has_fit
    lib = dl.lib()
    assert lib.dlm_sh_plan_fit_status(plan.handle) == DLM_ESINGULAR
    assert b"singular" in lib.dlm_last_error()
    B0, P0 = plan.matrices(0)
    assert P0 is None and np.abs(B0 - oplan.B[0]).max() < 1e-12
    V, S = 300 + 5, len(dirs)
    rng = np.random.default_rng(7)
    c = rng.standard_normal((V, S, plan.K)).astype(np.float32).astype(np.float64)
    errs = {}
    check("x", dl.sh2signal_fwd(plan, cuda(c), precision=prec), osh.sh2signal(oplan, c), prec, errs)
    dx = rng.standard_normal((V, plan.n_dw)).astype(np.float32).astype(np.float64)
    check("dc", dl.sh2signal_bwd(plan, cuda(dx), precision=prec), osh.sh2signal_adjoint(oplan, dx), prec, errs)
    tgt = rng.standard_normal((V, plan.n_dw)).astype(np.float32).astype(np.float64)
    loss, dch, xhat = dl.sh2signal_mse_fwd_bwd(plan, cuda(c), cuda(tgt), need_xhat=True, precision=prec)
    xr = osh.sh2signal(oplan, c)
    l_ref, dxh = ostack.mse(xr, tgt)
    check("head_x", xhat, xr, prec, errs)
    check("head_dc", dch, osh.sh2signal_adjoint(oplan, dxh), prec, errs)
    assert abs(loss.item() - l_ref) / l_ref <= (2e-2 if prec == "bf16" else 1e-5)
    print(f"[parity] evaluation-only plan {dirs} {prec}: " + fmt(errs), flush=True)
    sig = torch.zeros((V, plan.n_dw), device=DEV)
    for call in (lambda: dl.signal2sh_fwd(plan, sig, precision=prec),
                 lambda: dl.signal2sh_bwd(plan, torch.zeros((V, S, plan.K), device=DEV), precision=prec)):
        with pytest.raises(dl.DelimitError) as e:
            call()
        assert e.value.status == DLM_ESINGULAR
    with pytest.raises(np.linalg.LinAlgError):
        osh.signal2sh(oplan, np.zeros((1, plan.n_dw)))


def test_sh2signal_module_onto_30_directions():
    """The SH2Signal layer (built at lambda = 0, as evaluation needs no fit)
    takes order-8 coefficients onto a 30-direction table."""
    acq = _eval_only_acq((30,), 52)
    mod = SH2Signal(8, acq.bvecs, acq.bvals)
    c = np.random.default_rng(8).standard_normal((77, 45)).astype(np.float32).astype(np.float64)
    out = mod(cuda(c))
    ref = osh.sh2signal(osh.SHPlan(acq.bvecs, acq.bvals, 8, 0.0), c[:, None, :])
    check("x", out, ref, "fp32")


def test_update_gradients_keeps_an_existing_fit():
    """A plan with a fit refuses a table whose fit is singular and keeps its
    tables; an evaluation-only plan takes any table of the same shells."""
    acq = _eval_only_acq((30,), 53)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, 4, 0.0)  # K = 15 < 30: has a fit
    assert plan.has_fit
    x = cuda(np.random.default_rng(9).uniform(0.1, 1.0, (64, 30)))
    c0 = dl.signal2sh_fwd(plan, x)
    same = np.tile([[0.0, 0.0, 1.0]], (30, 1))  # one direction 30 times: rank 1
    with pytest.raises(dl.DelimitError) as e:
        plan.update_gradients(same)
    assert e.value.status == DLM_ESINGULAR
    assert plan.has_fit
    assert torch.equal(dl.signal2sh_fwd(plan, x), c0)
    ev = dl.SHPlan(acq.bvecs, acq.bvals, 8, 0.0)
    assert not ev.has_fit
    dacq = dg.distort_acquisition(acq, 3.0, dg.rng_for(53, dg.STREAM_DISTORT, 2))
    ev.update_gradients(dacq.bvecs)
    assert dl.lib().dlm_sh_plan_fit_status(ev.handle) == DLM_ESINGULAR
    c = np.random.default_rng(10).standard_normal((64, 1, 45))
    check("x", dl.sh2signal_fwd(ev, cuda(c)), osh.sh2signal(osh.SHPlan(dacq.bvecs, dacq.bvals, 8, 0.0), c), "fp32")
    assert dl.lib().dlm_sh_plan_fit_status(plan.handle) == DLM_OK
