"""GPU parity of the fused q-space loss head (SH2Signal, MSE, SH2Signal
adjoint in one pass) against the FP64 oracle's three steps in a row.

Cases: the three-shell 90-direction order-8 table, a one-shell 30-direction
order-4 table, and shells of unequal size (17, 45 and 96 directions: a ragged
direction tile, and the largest shell the fused kernel takes), each with a
voxel count that leaves a ragged 16-voxel tile.
"""
import numpy as np
import pytest
import torch

import datagen as dg
import paper_1808_01517_amd as dl
from oracle import sh as osh
from oracle import stack as ostack

from parity_util import TOL, check, fmt, rel, row_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _mixed_acquisition():
    """Three shells of 17, 45 and 96 directions plus two b0 volumes."""
    dirs = [dg.perturb_directions(dg.fibonacci_hemisphere(n), 2.0, dg.rng_for(7, 0, s))
            for s, n in enumerate((17, 45, 96))]
    shell_b = [1000.0, 2000.0, 3000.0]
    bvecs = np.concatenate([np.zeros((2, 3))] + dirs, axis=0)
    bvals = np.concatenate([np.zeros(2)] + [np.full(d.shape[0], b) for b, d in zip(shell_b, dirs)])
    return dg.Acquisition(bvecs=bvecs, bvals=bvals, shell_b=shell_b, shell_dirs=dirs, n_b0=2)


def _case(name):
    if name == "c2":
        w = dg.C2
        acq = dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
        return acq, w.sh_order, 3000 + 13
    if name == "c1":
        w = dg.C1
        acq = dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
        return acq, w.sh_order, 4096 + 37
    return _mixed_acquisition(), 8, 1000 + 7


def _inputs(acq, oplan, V, seed, near_fit=False):
    """SH coefficients of noisy stick-ball signals and a target.

    Default: the clean signal of an independent batch, so the residual
    x^ - target is as large as the signal (a network early in training).
    near_fit: the clean signal of the same voxels, so the residual is the
    noise alone (a network that has converged); x^ - target then cancels
    most of x^, and rounding in x^ grows, relative to the residual, by the
    ratio ||x^|| / ||x^ - target||."""
    batch = dg.stick_ball_batch(acq, V, 3, 20.0, dg.rng_for(seed, 2, 0))
    c = osh.signal2sh(oplan, batch.x).astype(np.float32).astype(np.float64)
    other = batch if near_fit else dg.stick_ball_batch(acq, V, 3, 20.0, dg.rng_for(seed, 2, 1))
    tgt = other.clean.astype(np.float32).astype(np.float64)
    return c, tgt


def _head_errors(plan, oplan, c, tgt, prec):
    loss, dc, xhat = dl.sh2signal_mse_fwd_bwd(plan, cuda(c), cuda(tgt), need_xhat=True, precision=prec)
    xhat_ref = osh.sh2signal(oplan, c)
    l_ref, dxh_ref = ostack.mse(xhat_ref, tgt)
    dc_ref = osh.sh2signal_adjoint(oplan, dxh_ref)
    errs = {"xhat": (rel(xhat, xhat_ref), row_err(xhat, xhat_ref)), "loss": abs(loss.item() - l_ref) / l_ref,
            "dc": (rel(dc, dc_ref), row_err(dc, dc_ref))}
    kappa = float(np.linalg.norm(xhat_ref) / np.linalg.norm(xhat_ref - tgt))
    return errs, kappa, (loss, dc, xhat), (xhat_ref, dc_ref)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("case", ["c2", "c1", "mixed"])
def test_loss_head_matches_oracle(prec, case):
    acq, L, V = _case(case)
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    assert dl.sh2signal_mse_supported(plan)
    c, tgt = _inputs(acq, oplan, V, 21)
    errs, kappa, (loss, dc, xhat), (xhat_ref, dc_ref) = _head_errors(plan, oplan, c, tgt, prec)
    print(f"[parity] loss head {case} {prec} (kappa {kappa:.1f}): " + fmt(errs), flush=True)
    check("xhat", xhat, xhat_ref, prec)
    check("dc", dc, dc_ref, prec)
    assert errs["loss"] <= TOL[prec], errs
    # the same call without x^ gives the same loss and gradient bit for bit
    loss2, dc2, none = dl.sh2signal_mse_fwd_bwd(plan, cuda(c), cuda(tgt), precision=prec)
    assert none is None
    assert loss2.item() == loss.item()
    assert torch.equal(dc2, dc)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_loss_head_near_fit(prec):
    """Residual = noise only.  x^ keeps its own bound; the loss and dc,
    functions of the residual, are held to the bound scaled by
    kappa = ||x^|| / ||x^ - target|| (the cancellation in x^ - target)."""
    acq, L, V = _case("c2")
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    c, tgt = _inputs(acq, oplan, V, 24, near_fit=True)
    errs, kappa, (_, dc, xhat), (xhat_ref, dc_ref) = _head_errors(plan, oplan, c, tgt, prec)
    print(f"[parity] loss head near fit {prec} (kappa {kappa:.1f}): " + fmt(errs), flush=True)
    assert kappa > 3.0  # the case does exercise cancellation
    check("xhat", xhat, xhat_ref, prec)
    check("dc", dc, dc_ref, prec, scale=kappa)
    assert errs["loss"] <= TOL[prec] * kappa, errs


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_loss_head_matches_unfused_composition(prec):
    """Fused head vs dlm_sh2signal_fwd -> dlm_mse_fwd_bwd -> dlm_sh2signal_bwd
    on the GPU: the same arithmetic in a different summation order."""
    acq, L, V = _case("c2")
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    c, tgt = _inputs(acq, oplan, V, 22)
    cg, tg = cuda(c), cuda(tgt)
    loss, dc, xhat = dl.sh2signal_mse_fwd_bwd(plan, cg, tg, need_xhat=True, precision=prec)
    xu = dl.sh2signal_fwd(plan, cg, precision=prec)
    lu, dxu = dl.mse_fwd_bwd(xu, tg)
    dcu = dl.sh2signal_bwd(plan, dxu, precision=prec)
    assert rel(xhat, xu) <= 1e-6 and row_err(xhat, xu) <= 1e-5
    assert abs(loss.item() - lu.item()) <= 1e-5 * abs(lu.item())
    check("dc", dc, dcu, prec)


@pytest.mark.parametrize("V", [1, 17, 16 * 1400 + 5])
def test_loss_head_batch_sizes(V):
    """One voxel, one full 16-voxel tile plus one, and more per-wave partials
    than one block sums (22 405 voxels x 3 shells = 4 203 waves > 4 096: the
    two-pass sum)."""
    acq, L, _ = _case("c2")
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    c, tgt = _inputs(acq, oplan, V, 23)
    loss, dc, _ = dl.sh2signal_mse_fwd_bwd(plan, cuda(c), cuda(tgt))
    l_ref, dxh_ref = ostack.mse(osh.sh2signal(oplan, c), tgt)
    assert abs(loss.item() - l_ref) / l_ref <= TOL["fp32"]
    check("dc", dc, osh.sh2signal_adjoint(oplan, dxh_ref), "fp32")


def test_loss_head_rejects_empty_batch_and_large_orders():
    acq, L, _ = _case("c2")
    plan = dl.SHPlan(acq.bvecs, acq.bvals, L, 0.006)
    empty = torch.zeros((0, plan.n_shells, plan.K), device=DEV)
    with pytest.raises(dl.DelimitError):
        dl.sh2signal_mse_fwd_bwd(plan, empty, torch.zeros((0, plan.n_dw), device=DEV))
    # order 10 has K = 66 coefficients, beyond the fused kernel's 64
    big = dl.SHPlan(acq.bvecs, acq.bvals, 10, 0.006)
    assert not dl.sh2signal_mse_supported(big)
    c = torch.zeros((16, big.n_shells, big.K), device=DEV)
    with pytest.raises(dl.DelimitError):
        dl.sh2signal_mse_fwd_bwd(big, c, torch.zeros((16, big.n_dw), device=DEV))
