"""The table-resident FP32 kernels (large batches: persistent blocks that
copy every shell's fragment tables into LDS once) against their other forms
(small batches; DLM_SHELL_RESIDENT=0 forces those) and against the FP64
oracle: the loss head, and Signal2SH, with the SH2Signal and
Signal2SH-adjoint contractions of the same large batch beside them.

The loss head's two forms run the same per-item arithmetic on the same
fragments, so they must agree bit for bit: loss, gradient and x^ (the BF16
head and the contractions over the coefficients have one form, so there
the comparison is of a call with itself).  Signal2SH's other form is the
tiled core, whose summation order differs: it is held to the oracle only.  The batch (90,007 voxels of the three-shell 90-direction order-8
table) is large enough for the resident form and leaves a ragged 16-voxel
tile; a batch of unequal shells (17/45/96, one launch per shell, 270,021
voxels) takes it shell by shell.
"""
import os

import numpy as np
import pytest
import torch

import datagen as dg
import paper_1808_01517_amd as dl
from oracle import sh as osh
from oracle import stack as ostack

from parity_util import TOL, check, fmt

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
V_BIG = 90_000 + 7  # 16,877 wave items of 3 shells: above the resident form's threshold


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _acq(kind):
    if kind == "c2":
        w = dg.C2
        return dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
    dirs = [dg.perturb_directions(dg.fibonacci_hemisphere(n), 2.0, dg.rng_for(7, 0, s))
            for s, n in enumerate((17, 45, 96))]
    shell_b = [1000.0, 2000.0, 3000.0]
    bvecs = np.concatenate([np.zeros((2, 3))] + dirs, axis=0)
    bvals = np.concatenate([np.zeros(2)] + [np.full(d.shape[0], b) for b, d in zip(shell_b, dirs)])
    return dg.Acquisition(bvecs=bvecs, bvals=bvals, shell_b=shell_b, shell_dirs=dirs, n_b0=2)


def _run(plan, c, tgt, dcoef, prec):
    coef = dl.signal2sh_fwd(plan, tgt, precision=prec) if plan.has_fit else None
    x = dl.sh2signal_fwd(plan, c, precision=prec)
    dx = dl.signal2sh_bwd(plan, dcoef, precision=prec)
    loss, dc, xhat = dl.sh2signal_mse_fwd_bwd(plan, c, tgt, need_xhat=True, precision=prec)
    torch.cuda.synchronize()
    return x, dx, loss, dc, xhat, coef


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("kind", ["c2", "mixed"])
def test_resident_tables_match_short_blocks_and_oracle(prec, kind):
    acq = _acq(kind)
    L = 8
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    V = V_BIG if kind == "c2" else 3 * V_BIG  # one launch per shell: each must reach the threshold
    rng = np.random.default_rng(77)
    c = rng.standard_normal((V, len(plan.shells), plan.K)).astype(np.float32).astype(np.float64)
    tgt = osh.sh2signal(oplan, rng.standard_normal(c.shape)).astype(np.float32).astype(np.float64)
    dcoef = rng.standard_normal(c.shape).astype(np.float32).astype(np.float64)
    cg, tg, dg_ = cuda(c), cuda(tgt), cuda(dcoef)
    res = _run(plan, cg, tg, dg_, prec)
    os.environ["DLM_SHELL_RESIDENT"] = "0"
    try:
        short = _run(plan, cg, tg, dg_, prec)
    finally:
        del os.environ["DLM_SHELL_RESIDENT"]
    for name, a, b in zip(("x", "dx", "loss", "dc", "xhat"), res[:5], short[:5]):
        assert torch.equal(a, b), f"{kind} {prec}: {name} differs between the two forms"
    x, dx, loss, dc, xhat, coef = res
    errs = {}
    c_ref = osh.signal2sh(oplan, tgt)
    check("c", coef, c_ref, prec, errs)
    check("c_other_form", short[5], c_ref, prec, errs)
    x_ref = osh.sh2signal(oplan, c)
    check("x", x, x_ref, prec, errs)
    check("dx", dx, osh.signal2sh_adjoint(oplan, dcoef), prec, errs)
    l_ref, dxh_ref = ostack.mse(x_ref, tgt)
    check("xhat", xhat, x_ref, prec, errs)
    check("dc", dc, osh.sh2signal_adjoint(oplan, dxh_ref), prec, errs)
    errs["loss"] = abs(loss.item() - l_ref) / l_ref
    print(f"[parity] resident tables {kind} {prec}, V={V}: " + fmt(errs), flush=True)
    assert errs["loss"] <= TOL[prec]


def test_resident_loss_head_across_table_sizes():
    """The resident FP32 loss head raises the kernel's dynamic-LDS limit to
    the largest table it has met and caches its fit per table size: a
    three-shell plan (110 KB of tables), then a two-shell plan (74 KB), then
    the three-shell plan again must all run resident and match the oracle
    (a limit lowered for the two-shell plan would make the third launch
    fail)."""
    w = dg.C2
    three = dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
    two = dg.make_acquisition(w.config, w.shell_b[:2], w.dirs_per_shell, w.perturb_deg, w.n_b0)
    rng = np.random.default_rng(78)
    for acq, V in ((three, V_BIG), (two, 2 * V_BIG), (three, V_BIG)):
        oplan = osh.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
        plan = dl.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
        c = rng.standard_normal((V, len(plan.shells), plan.K)).astype(np.float32).astype(np.float64)
        tgt = osh.sh2signal(oplan, rng.standard_normal(c.shape)).astype(np.float32).astype(np.float64)
        loss, dc, xhat = dl.sh2signal_mse_fwd_bwd(plan, cuda(c), cuda(tgt), need_xhat=True, precision="fp32")
        torch.cuda.synchronize()
        x_ref = osh.sh2signal(oplan, c)
        l_ref, dxh_ref = ostack.mse(x_ref, tgt)
        errs = {}
        check("xhat", xhat, x_ref, "fp32", errs)
        check("dc", dc, osh.sh2signal_adjoint(oplan, dxh_ref), "fp32", errs)
        errs["loss"] = abs(loss.item() - l_ref) / l_ref
        print(f"[parity] resident loss head, {len(plan.shells)} shells, V={V}: " + fmt(errs), flush=True)
        assert errs["loss"] <= TOL["fp32"]
