"""BF16 reductions over a shell's directions (Signal2SH, the SH2Signal
adjoint) on batches large enough for the per-shell kernel with two 16-voxel
blocks per wave (below that size the tiled core runs them), against the
FP64 oracle with norm-wise and per-voxel bounds.

Cases: the three-shell 90-direction order-8 table (one launch for the three
equal shells, 133,157 voxels: the last wave holds one partial block), and
shells of 17, 45 and 96 directions (one launch per shell, 140,003 voxels:
96 is the longest reduction this path takes, 17 and 45 go to the
coefficient-sized kernel).  A second test holds the BF16 per-shell
contractions with two blocks per wave bitwise to their one-block form.
"""
import os

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


@pytest.mark.parametrize("V", [45_000 + 33, 1000 + 7])
def test_bf16_pairs_match_single_blocks(V):
    """BF16 per-shell contractions with two 16-voxel blocks per wave against
    DLM_SHELL_PAIRS=0 (one block per wave): the same per-block arithmetic,
    so every output must agree bit for bit.  Both batches have an odd number
    of 16-voxel blocks (the last pair is half empty); 45,033 voxels put the
    three-shell Signal2SH and SH2Signal adjoint on the per-shell kernel,
    1,007 keep them on the tiled core."""
    w = dg.C2
    acq = dg.make_acquisition(w.config, w.shell_b, w.dirs_per_shell, w.perturb_deg, w.n_b0)
    oplan = osh.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
    plan = dl.SHPlan(acq.bvecs, acq.bvals, 8, 0.006)
    assert ((V + 15) // 16) % 2 == 1
    rng = np.random.default_rng(95)
    c = cuda(rng.standard_normal((V, plan.n_shells, plan.K)))
    x = cuda(osh.sh2signal(oplan, rng.standard_normal((V, plan.n_shells, plan.K))))
    dx = cuda(rng.standard_normal((V, plan.n_dw)))

    def run():
        out = [dl.signal2sh_fwd(plan, x, precision="bf16"), dl.sh2signal_bwd(plan, dx, precision="bf16"),
               dl.signal2sh_bwd(plan, c, precision="bf16"), dl.sh2signal_fwd(plan, c, precision="bf16")]
        torch.cuda.synchronize()
        return out

    pairs = run()
    os.environ["DLM_SHELL_PAIRS"] = "0"
    try:
        single = run()
    finally:
        del os.environ["DLM_SHELL_PAIRS"]
    names = ("signal2sh", "sh2signal_adjoint", "signal2sh_adjoint", "sh2signal")
    for name, a, b in zip(names, pairs, single):
        assert torch.equal(a, b), f"V={V}: {name} differs between two blocks and one block per wave"
    print(f"[parity] BF16 pairs vs single blocks, V={V}: bitwise equal", flush=True)
