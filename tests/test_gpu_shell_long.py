"""BF16 reductions over a shell's directions (Signal2SH, the SH2Signal
adjoint) on batches large enough for the per-shell kernel with two 16-voxel
blocks per wave (below that size the tiled core runs them), against the
FP64 oracle with norm-wise and per-voxel bounds.

Cases: the three-shell 90-direction order-8 table (one launch for the three
equal shells, 133,157 voxels: the last wave holds one partial block), and
shells of 17, 45 and 96 directions (one launch per shell, 140,003 voxels:
96 is the longest reduction this path takes, 17 and 45 go to the
coefficient-sized kernel).
"""
import numpy as np
import pytest
import torch

import datagen as dg
import paper_1808_01517_amd as dl
from oracle import sh as osh

from parity_util import check, fmt

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _acq(kind):
    if kind == "c2":
        w = dg.C2
        return dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0), 2048 * 64 + 2048 + 37
    dirs = [dg.perturb_directions(dg.fibonacci_hemisphere(n), 2.0, dg.rng_for(9, 0, s))
            for s, n in enumerate((17, 45, 96))]
    shell_b = [1000.0, 2000.0, 3000.0]
    bvecs = np.concatenate([np.zeros((2, 3))] + dirs, axis=0)
    bvals = np.concatenate([np.zeros(2)] + [np.full(d.shape[0], b) for b, d in zip(shell_b, dirs)])
    return dg.Acquisition(bvecs=bvecs, bvals=bvals, shell_b=shell_b, shell_dirs=dirs, n_b0=2), 140_003


@pytest.mark.parametrize("kind", ["c2", "mixed"])
def test_bf16_long_reductions_on_large_batches(kind):
    acq, V = _acq(kind)
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
    rng = np.random.default_rng(93)
    c = rng.standard_normal((V, plan.n_shells, plan.K))
    x = osh.sh2signal(oplan, c).astype(np.float32).astype(np.float64)
    dx = rng.standard_normal(x.shape).astype(np.float32).astype(np.float64)
    coef = dl.signal2sh_fwd(plan, cuda(x), precision="bf16")
    dc = dl.sh2signal_bwd(plan, cuda(dx), precision="bf16")
    torch.cuda.synchronize()
    errs = {}
    check("c", coef, osh.signal2sh(oplan, x), "bf16", errs)
    check("dc", dc, osh.sh2signal_adjoint(oplan, dx), "bf16", errs)
    print(f"[parity] BF16 long reductions {kind}, V={V}: " + fmt(errs), flush=True)
