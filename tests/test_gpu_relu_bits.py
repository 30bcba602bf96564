"""ReLU bits: the forward of a stacked layer writes one bit per output
element (its sign after the fused ReLU) beside the activation, and the next
layer's adjoint masks its input gradient with those bits instead of reading
the activation again.  The mask is the same predicate (stored value > 0), so
every result is bit-identical to the activation-mask path, and both meet the
oracle at the precision's bound.  Rows of 1440 entries (32 channels x 45
order-8 coefficients, 90 sixteen-bit words) and ragged batches.
"""
import numpy as np
import pytest
import torch

import datagen as dg
import paper_1808_01517_amd as dl
from oracle import lsc as olsc

from parity_util import check, fmt

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _plan(L=8, ks=(8, 8), m=90):
    g = dg.fibonacci_hemisphere(m)
    return olsc.LSCPlan(g, L, L, ks, np.deg2rad(30), 0.006), dl.LSCPlan(g, L, L, ks, np.deg2rad(30), 0.006)


def _weights(seed, C, O, T):
    W, b = dg.lsc_weights(seed, 0, C, O, T)
    return W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)


def pack_bits(a: torch.Tensor) -> np.ndarray:
    """Host packing of [a > 0] (rows of a multiple of 16 entries) into uint16
    words, bit b of word w = entry 16 w + b."""
    pos = (a.float().cpu().numpy().reshape(a.shape[0], -1) > 0).astype(np.uint16)
    pos = pos.reshape(a.shape[0], -1, 16)
    return (pos << np.arange(16, dtype=np.uint16)).sum(axis=2, dtype=np.uint16)


def words(bits: torch.Tensor) -> np.ndarray:
    return bits.cpu().numpy().view(np.uint16)


@pytest.mark.parametrize("V", [1, 33, 203])
@pytest.mark.parametrize("prec,store", [("fp32", torch.float32), ("bf16", torch.float32), ("bf16", torch.bfloat16)])
def test_forward_writes_relu_bits(prec, store, V):
    oplan, plan = _plan()
    W, b = _weights(21, 3, 32, plan.T)
    a = np.random.default_rng(V).standard_normal((V, 3, plan.K_in))
    ag, Wg, bg = cuda(a), cuda(W), cuda(b)
    ref_out = dl.lsc_fwd(plan, ag, Wg, bg, relu=True, precision=prec, form="folded", out_dtype=store)
    bits = dl.relu_bits_like(ref_out)
    assert tuple(bits.shape) == (V, 90)
    bits.fill_(-1)  # every word is overwritten
    out = dl.lsc_fwd(plan, ag, Wg, bg, relu=True, precision=prec, form="folded", out_dtype=store, relu_bits=bits)
    torch.cuda.synchronize()
    assert torch.equal(out, ref_out)
    got, want = words(bits), pack_bits(out)
    assert np.array_equal(got, want), f"{int((got != want).sum())} words differ"
    assert 0 < (out > 0).float().mean().item() < 1
    out_ref, _ = olsc.lsc_forward(oplan, a.astype(np.float32).astype(np.float64), W, b, True)
    check("out", out.float(), out_ref, prec)


@pytest.mark.parametrize("O", [3, 64])
@pytest.mark.parametrize("prec,store", [("fp32", torch.float32), ("bf16", torch.float32), ("bf16", torch.bfloat16)])
def test_backward_with_relu_bits_matches_activation_mask(prec, store, O):
    """Layer 1 (3 -> 32, ReLU) writes a_1 and its bits; layer 2 (32 -> O)
    takes the input-gradient mask from the bits.  da_in, dW and dbias equal
    those of the activation-mask path bit for bit."""
    oplan, plan = _plan()
    V = 203
    W1, b1 = _weights(22, 3, 32, plan.T)
    W2, b2 = _weights(23, 32, O, plan.T)
    x = cuda(np.random.default_rng(5).standard_normal((V, 3, plan.K_in)))
    W1g, b1g, W2g = cuda(W1), cuda(b1), cuda(W2)
    a1 = torch.empty((V, 32, plan.K_out), dtype=store, device=DEV)
    bits = dl.relu_bits_like(a1)
    dl.lsc_fwd(plan, x, W1g, b1g, relu=True, precision=prec, form="folded", out=a1, relu_bits=bits)
    out_half = prec == "bf16" and (O * plan.K_out) % 8 == 0 and store == torch.bfloat16
    da = cuda(np.random.default_rng(6).standard_normal((V, O, plan.K_out)))
    if out_half:
        da = da.to(torch.bfloat16)
    g_m, dW_m, db_m = dl.lsc_bwd(plan, a1, W2g, da, relu_in=True, precision=prec, form="folded")
    g_b, dW_b, db_b = dl.lsc_bwd(plan, a1, W2g, da, relu_in=True, precision=prec, form="folded", relu_bits=bits)
    torch.cuda.synchronize()
    assert torch.equal(g_b, g_m)
    assert torch.equal(dW_b, dW_m) and torch.equal(db_b, db_m)
    assert bool((g_b[a1 <= 0] == 0).all())
    a64 = a1.double().cpu().numpy()
    _, z = olsc.lsc_forward(oplan, a64, W2, b2, False)
    da_ref, dW_ref, db_ref = olsc.lsc_backward(oplan, a64, W2, z, da.double().cpu().numpy(), False)
    errs = {}
    check("da_in", g_b.float(), da_ref * (a64 > 0), prec, errs)
    check("dW", dW_b, dW_ref, prec, errs, kind="sum")
    check("db", db_b, db_ref, prec, errs, kind="sum")
    print(f"[parity] relu bits bwd {prec} store={store} O={O}: " + fmt(errs), flush=True)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_relu_bits_on_short_rows(prec):
    """Order 2 (6 coefficients), 3 -> 16 -> 3: rows of 96 entries (6 words),
    the narrow-tile configuration of the streaming core in both directions."""
    oplan, plan = _plan(L=2, ks=(6, 6), m=30)
    V = 517
    W1, b1 = _weights(26, 3, 16, plan.T)
    W2, b2 = _weights(27, 16, 3, plan.T)
    x = np.random.default_rng(8).standard_normal((V, 3, plan.K_in))
    W1g, b1g, W2g = cuda(W1), cuda(b1), cuda(W2)
    a1 = dl.lsc_fwd(plan, cuda(x), W1g, b1g, relu=True, precision=prec, form="folded")
    bits = dl.relu_bits_like(a1)
    assert tuple(bits.shape) == (V, 6)
    bits.fill_(-1)
    a1b = dl.lsc_fwd(plan, cuda(x), W1g, b1g, relu=True, precision=prec, form="folded", relu_bits=bits)
    torch.cuda.synchronize()
    assert torch.equal(a1b, a1)
    assert np.array_equal(words(bits), pack_bits(a1))
    da = cuda(np.random.default_rng(9).standard_normal((V, 3, plan.K_out)))
    g_m, dW_m, db_m = dl.lsc_bwd(plan, a1, W2g, da, relu_in=True, precision=prec, form="folded")
    g_b, dW_b, db_b = dl.lsc_bwd(plan, a1, W2g, da, relu_in=True, precision=prec, form="folded", relu_bits=bits)
    torch.cuda.synchronize()
    assert torch.equal(g_b, g_m) and torch.equal(dW_b, dW_m) and torch.equal(db_b, db_m)
    a64 = a1.double().cpu().numpy()
    _, z = olsc.lsc_forward(oplan, a64, W2, b2, False)
    da_ref, _, _ = olsc.lsc_backward(oplan, a64, W2, z, da.double().cpu().numpy(), False)
    check("da_in", g_b, da_ref * (a64 > 0), prec)


def test_relu_bits_rejects_unsupported():
    oplan, plan = _plan()
    V = 16
    W1, b1 = _weights(24, 3, 32, plan.T)
    W3, b3 = _weights(25, 32, 3, plan.T)
    x = cuda(np.random.default_rng(7).standard_normal((V, 3, plan.K_in)))
    W1g, b1g, W3g, b3g = cuda(W1), cuda(b1), cuda(W3), cuda(b3)
    a1 = dl.lsc_fwd(plan, x, W1g, b1g, relu=True, form="folded")
    bits = dl.relu_bits_like(a1)
    with pytest.raises(dl.DelimitError):  # no fused ReLU
        dl.lsc_fwd(plan, x, W1g, b1g, relu=False, form="folded", relu_bits=bits)
    with pytest.raises(dl.DelimitError):  # resample form
        dl.lsc_fwd(plan, x, W1g, b1g, relu=True, form="resample", relu_bits=bits)
    with pytest.raises(ValueError):  # wrong shape
        dl.lsc_fwd(plan, x, W1g, b1g, relu=True, form="folded", relu_bits=bits[:, :45])
    with pytest.raises(ValueError):  # 3 x 45 entries per row: not a multiple of 16
        dl.relu_bits_like(x)
    dl.lsc_fwd(plan, x, W1g, b1g, relu=True, form="folded", relu_bits=bits)
    da = torch.ones((V, 3, plan.K_out), device=DEV)
    with pytest.raises(dl.DelimitError):  # bits without relu_in
        dl.lsc_bwd(plan, a1, W3g, da, form="folded", relu_bits=bits)
    out3 = dl.lsc_fwd(plan, a1, W3g, b3g, relu=True, form="folded")
    with pytest.raises(dl.DelimitError):  # bits with the output-side ReLU
        dl.lsc_bwd(plan, a1, W3g, da, a_out=out3, relu=True, relu_in=True, form="folded", relu_bits=bits)
    with pytest.raises(dl.DelimitError):  # resample form
        dl.lsc_bwd(plan, a1, W3g, da, relu_in=True, form="resample", relu_bits=bits)
    empty = torch.zeros((0, 32, plan.K_in), device=DEV)
    e_bits = dl.relu_bits_like(empty)
    g0, dW0, db0 = dl.lsc_bwd(plan, empty, W3g, torch.zeros((0, 3, plan.K_out), device=DEV), relu_in=True,
                              form="folded", relu_bits=e_bits)
    assert g0.shape[0] == 0 and float(dW0.abs().max()) == 0.0 and float(db0.abs().max()) == 0.0


@pytest.mark.parametrize("case", [(3, 32, 8, 1000 + 77), (5, 16, 6, 517)])
@pytest.mark.parametrize("prec,store", [("fp32", torch.float32), ("bf16", torch.float32), ("bf16", torch.bfloat16)])
def test_short_reduction_kernel_matches_tiled_core(case, prec, store, monkeypatch):
    """The folded GEMMs with a short reduction (C * K_in or O * K_out in
    129..160: the forward of a layer with few input channels, the input
    gradient of a layer with few output channels) run on a kernel that keeps
    its rows of A in registers; DLM_TILED_ONLY=1 sends them to the tiled
    core.  Both accumulate in the same order: outputs, ReLU bits and input
    gradients are bitwise equal, with a ragged last block of rows."""
    C, O, L, V = case
    oplan, plan = _plan(L=L)
    W1, b1 = _weights(31, C, O, plan.T)
    W2, _ = _weights(32, O, C, plan.T)
    x = cuda(np.random.default_rng(12).standard_normal((V, C, plan.K_in)))
    d = cuda(np.random.default_rng(13).standard_normal((V, C, plan.K_out)))
    W1g, b1g, W2g = cuda(W1), cuda(b1), cuda(W2)

    def run():
        a1 = torch.empty((V, O, plan.K_out), dtype=store, device=DEV)
        bits = dl.relu_bits_like(a1)
        dl.lsc_fwd(plan, x, W1g, b1g, relu=True, out=a1, precision=prec, form="folded", relu_bits=bits)
        g, _, _ = dl.lsc_bwd(plan, a1, W2g, d, relu_in=True, precision=prec, form="folded", relu_bits=bits,
                             need_weight_grad=False, need_bias_grad=False)
        torch.cuda.synchronize()
        return a1, bits, g

    monkeypatch.delenv("DLM_TILED_ONLY", raising=False)
    fast = run()
    monkeypatch.setenv("DLM_TILED_ONLY", "1")
    tiled = run()
    for name, u, w in zip(("a_out", "bits", "da_in"), fast, tiled):
        assert torch.equal(u, w), name
    monkeypatch.delenv("DLM_TILED_ONLY")
    out_ref, _ = olsc.lsc_forward(oplan, x.double().cpu().numpy(), W1, b1, True)
    check("a_out", fast[0].float(), out_ref, prec)
