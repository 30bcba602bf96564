"""MI355X-native DELIMIT layers (Koppers & Merhof, arXiv:1808.01517).

Thin Python binding over libdelimit.so (C ABI in include/delimit.h): plans
hold the float64-built tables on the device, and each call hands device
pointers of torch tensors plus the current HIP stream to the library.
PyTorch supplies device memory and streams only; every step of Signal2SH,
SH2Signal and the local spherical convolution runs in the library's HIP
kernels.  There is no CPU or PyTorch fallback: without the built library
every call raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import DLM_BF16, DLM_FP32, DLM_LSC_FOLDED, DLM_LSC_RESAMPLE, DelimitError, check, dptr, lib

__all__ = [
    "SHPlan", "LSCPlan", "precision_code", "signal2sh_fwd", "signal2sh_bwd", "sh2signal_fwd", "sh2signal_bwd",
    "lsc_fwd", "lsc_bwd", "lsc_workspace_bytes", "mse_fwd_bwd", "adam_step", "Workspace", "DelimitError",
    "sh_basis", "sh_fit_matrix", "lsc_kernel_points", "timing_enable", "timing_reset", "timing_report",
    "form_code", "DEFAULT_FORM", "signal2sh_fwd_raw", "relmse_fwd_bwd", "sh2signal_mse_supported",
    "sh2signal_mse_fwd_bwd", "peak_copy", "peak_mfma",
]


DEFAULT_FORM = "folded"


def form_code(f) -> int:
    if f in (DLM_LSC_RESAMPLE, "resample"):
        return DLM_LSC_RESAMPLE
    if f in (DLM_LSC_FOLDED, "folded", None):
        return DLM_LSC_FOLDED
    raise ValueError(f"unknown LSC form {f!r}")


def precision_code(p) -> int:
    if p in (DLM_FP32, "fp32", "f32", torch.float32, None):
        return DLM_FP32
    if p in (DLM_BF16, "bf16", torch.bfloat16):
        return DLM_BF16
    raise ValueError(f"unknown precision {p!r}")


def _stream(t: torch.Tensor):
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _f32_dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32 (got {t.dtype})")
    return t.contiguous()


def _act_dev(t: torch.Tensor, name: str) -> torch.Tensor:
    """An LSC activation: float32, or bfloat16 (BF16 folded form only)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError(f"{name} must be float32 or bfloat16 (got {t.dtype})")
    return t.contiguous()


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ------------------------------------------------------------ host tables
def sh_basis(sh_order: int, dirs) -> np.ndarray:
    d = _c64(dirs).reshape(-1, 3)
    K = (sh_order + 1) * (sh_order + 2) // 2
    out = np.zeros((d.shape[0], K))
    check(lib().dlm_sh_basis(sh_order, dptr(d), d.shape[0], dptr(out)))
    return out


def sh_fit_matrix(sh_order: int, dirs, lb_lambda: float) -> np.ndarray:
    d = _c64(dirs).reshape(-1, 3)
    K = (sh_order + 1) * (sh_order + 2) // 2
    out = np.zeros((K, d.shape[0]))
    check(lib().dlm_sh_fit_matrix(sh_order, dptr(d), d.shape[0], float(lb_lambda), dptr(out)))
    return out


def lsc_kernel_points(dirs, kernel_sizes, angular_distance: float) -> np.ndarray:
    d = _c64(dirs).reshape(-1, 3)
    ks = (C.c_int * len(kernel_sizes))(*[int(k) for k in kernel_sizes])
    T = 1 + sum(int(k) for k in kernel_sizes)
    out = np.zeros((d.shape[0], T, 3))
    check(lib().dlm_lsc_kernel_points(dptr(d), d.shape[0], ks, len(kernel_sizes), float(angular_distance), dptr(out)))
    return out


# ------------------------------------------------------------------ plans
class SHPlan:
    """Per-shell SH basis / regularised fit of one gradient table on the device."""

    def __init__(self, bvecs, bvals, sh_order: int, lb_lambda: float = 0.006, b0_max: float = 50.0,
                 shell_rel_tol: float = 0.05):
        bv = _c64(bvecs).reshape(-1, 3)
        bl = _c64(bvals).reshape(-1)
        if bl.shape[0] != bv.shape[0]:
            raise ValueError("bvecs and bvals differ in length")
        h = C.c_void_p()
        check(lib().dlm_sh_plan_create(dptr(bv), dptr(bl), bv.shape[0], int(sh_order), float(lb_lambda),
                                       float(b0_max), float(shell_rel_tol), C.byref(h)))
        self._h = h
        # bound now: __del__ may run during interpreter teardown, when module
        # globals such as lib() are already gone
        self._destroy = lib().dlm_sh_plan_destroy
        self.sh_order = int(sh_order)
        self.n_total = bv.shape[0]
        # False for an evaluation-only plan (a shell's fit is singular, e.g.
        # fewer directions than coefficients at lb_lambda = 0): SH2Signal and
        # its adjoint work, Signal2SH calls raise DelimitError
        self.has_fit = lib().dlm_sh_plan_fit_status(h) == _lib.DLM_OK
        S, K, n = C.c_int(), C.c_int(), C.c_int64()
        check(lib().dlm_sh_plan_info(h, C.byref(S), C.byref(K), C.byref(n)))
        self.n_shells, self.K, self.n_dw = S.value, K.value, n.value
        self.shells = []
        for s in range(self.n_shells):
            nd, b = C.c_int64(), C.c_double()
            check(lib().dlm_sh_plan_shell(h, s, C.byref(nd), C.byref(b), None))
            idx = np.zeros(nd.value, dtype=np.int64)
            check(lib().dlm_sh_plan_shell(h, s, None, None, idx.ctypes.data_as(C.POINTER(C.c_int64))))
            self.shells.append((nd.value, b.value, idx))

    @property
    def handle(self):
        return self._h

    def matrices(self, shell: int):
        """(B_s [N_s][K], P_s [K][N_s]) in float64; P_s is None on an
        evaluation-only plan."""
        n = self.shells[shell][0]
        B = np.zeros((n, self.K))
        if not self.has_fit:
            check(lib().dlm_sh_plan_matrices(self._h, shell, dptr(B), None))
            return B, None
        P = np.zeros((self.K, n))
        check(lib().dlm_sh_plan_matrices(self._h, shell, dptr(B), dptr(P)))
        return B, P

    def update_gradients(self, bvecs, stream=None):
        bv = _c64(bvecs).reshape(-1, 3)
        if bv.shape[0] != self.n_total:
            raise ValueError("update_gradients needs the same number of volumes")
        st = C.c_void_p(stream if stream is not None else torch.cuda.current_stream().cuda_stream)
        check(lib().dlm_sh_plan_update_gradients(self._h, dptr(bv), st))
        self.has_fit = lib().dlm_sh_plan_fit_status(self._h) == _lib.DLM_OK

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = None


class LSCPlan:
    """Cyclic-kernel geometry, resampling basis and refit of one LSC layer."""

    def __init__(self, sampled_gradients, sh_order_in: int, sh_order_out: int, kernel_sizes,
                 angular_distance: float, lb_lambda: float = 0.006):
        g = _c64(sampled_gradients).reshape(-1, 3)
        ks = [int(k) for k in kernel_sizes]
        arr = (C.c_int * max(1, len(ks)))(*ks)
        h = C.c_void_p()
        check(lib().dlm_lsc_plan_create(dptr(g), g.shape[0], int(sh_order_in), int(sh_order_out), arr, len(ks),
                                        float(angular_distance), float(lb_lambda), C.byref(h)))
        self._h = h
        self._destroy = lib().dlm_lsc_plan_destroy  # see SHPlan.__init__
        T, Ki, Ko, m = C.c_int(), C.c_int(), C.c_int(), C.c_int64()
        check(lib().dlm_lsc_plan_info(h, C.byref(T), C.byref(Ki), C.byref(Ko), C.byref(m)))
        self.T, self.K_in, self.K_out, self.m = T.value, Ki.value, Ko.value, m.value
        self.kernel_sizes = tuple(ks)
        self.sh_order_in, self.sh_order_out = int(sh_order_in), int(sh_order_out)

    @property
    def handle(self):
        return self._h

    def tables(self):
        pts = np.zeros((self.m, self.T, 3))
        Bnb = np.zeros((self.m * self.T, self.K_in))
        Pm = np.zeros((self.K_out, self.m))
        check(lib().dlm_lsc_plan_tables(self._h, dptr(pts), dptr(Bnb), dptr(Pm)))
        return pts, Bnb, Pm

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = None


# -------------------------------------------------------------- workspace
class Workspace:
    """Caller-owned device scratch for the LSC calls (a torch uint8 buffer)."""

    def __init__(self, nbytes: int, device="cuda"):
        self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=device)

    @property
    def nbytes(self) -> int:
        return self.buf.numel()

    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())


def lsc_workspace_bytes(plan: LSCPlan, C_in: int, O: int, V_chunk: int, precision="fp32", form=DEFAULT_FORM) -> int:
    out = C.c_size_t()
    check(lib().dlm_lsc_workspace_bytes(plan.handle, int(C_in), int(O), int(V_chunk), form_code(form),
                                        precision_code(precision), C.byref(out)))
    return out.value


_ws_cache: dict = {}


def _default_ws(plan: LSCPlan, C_in: int, O: int, V: int, prec: int, device, form) -> Workspace:
    """A workspace shared by the calls on one stream (resample form: up to
    65536 voxels per pass).  Keyed by device and stream: calls on one stream
    run in order, so they may share scratch; calls on different streams get
    their own.  Growing it frees the old buffer through torch's caching
    allocator, which reuses it only after the stream's queued work."""
    need = lsc_workspace_bytes(plan, C_in, O, min(max(V, 1), 1 << 16), prec, form)
    key = (str(device), torch.cuda.current_stream(device).cuda_stream)
    ws = _ws_cache.get(key)
    if ws is None or ws.nbytes < need:
        ws = Workspace(need, device)
        _ws_cache[key] = ws
    return ws


# ---------------------------------------------------------- SH transforms
def _sh_call(fn, plan: SHPlan, inp: torch.Tensor, out_shape, out, precision):
    inp = _f32_dev(inp, "input")
    V = inp.shape[0]
    if out is None:
        out = torch.empty(out_shape, dtype=torch.float32, device=inp.device)
    check(fn(plan.handle, _ptr(inp), _ptr(out), V, precision_code(precision), _stream(inp)))
    return out


def signal2sh_fwd(plan: SHPlan, x: torch.Tensor, out=None, precision="fp32") -> torch.Tensor:
    """x [V][N_dw] -> c [V][S][K]."""
    if x.dim() != 2 or x.shape[1] != plan.n_dw:
        raise ValueError(f"x must be [V, {plan.n_dw}]")
    return _sh_call(lib().dlm_signal2sh_fwd, plan, x, (x.shape[0], plan.n_shells, plan.K), out, precision)


def signal2sh_bwd(plan: SHPlan, dc: torch.Tensor, out=None, precision="fp32") -> torch.Tensor:
    if dc.dim() != 3 or tuple(dc.shape[1:]) != (plan.n_shells, plan.K):
        raise ValueError(f"dc must be [V, {plan.n_shells}, {plan.K}]")
    return _sh_call(lib().dlm_signal2sh_bwd, plan, dc, (dc.shape[0], plan.n_dw), out, precision)


def signal2sh_fwd_raw(plan: SHPlan, raw: torch.Tensor, out=None, precision="fp32") -> torch.Tensor:
    """raw [V][n_total] (creation-table volume order, b0 volumes included) ->
    c [V][S][K], with the b0 normalisation fused into the load."""
    raw = _f32_dev(raw, "raw")
    if raw.dim() != 2 or raw.shape[1] != plan.n_total:
        raise ValueError(f"raw must be [V, {plan.n_total}]")
    V = raw.shape[0]
    if out is None:
        out = torch.empty((V, plan.n_shells, plan.K), dtype=torch.float32, device=raw.device)
    ws = torch.empty(lib().dlm_signal2sh_raw_workspace_bytes(V), dtype=torch.uint8, device=raw.device)
    check(lib().dlm_signal2sh_fwd_raw(plan.handle, _ptr(raw), _ptr(out), V, _ptr(ws), ws.numel(),
                                      precision_code(precision), _stream(raw)))
    return out


def sh2signal_fwd(plan: SHPlan, c: torch.Tensor, out=None, precision="fp32") -> torch.Tensor:
    """c [V][S][K] -> x [V][N_dw]."""
    if c.dim() != 3 or tuple(c.shape[1:]) != (plan.n_shells, plan.K):
        raise ValueError(f"c must be [V, {plan.n_shells}, {plan.K}]")
    return _sh_call(lib().dlm_sh2signal_fwd, plan, c, (c.shape[0], plan.n_dw), out, precision)


def sh2signal_bwd(plan: SHPlan, dx: torch.Tensor, out=None, precision="fp32") -> torch.Tensor:
    if dx.dim() != 2 or dx.shape[1] != plan.n_dw:
        raise ValueError(f"dx must be [V, {plan.n_dw}]")
    return _sh_call(lib().dlm_sh2signal_bwd, plan, dx, (dx.shape[0], plan.n_shells, plan.K), out, precision)


# -------------------------------------------------------------------- LSC
def relu_bits_like(a: torch.Tensor) -> torch.Tensor:
    """An int16 [V][N/16] buffer for the ReLU bits of activations a [V][...]
    (N entries per row, a multiple of 16)."""
    n = a[0].numel() if a.shape[0] else int(np.prod(a.shape[1:]))
    if n % 16:
        raise ValueError(f"ReLU bits need rows of a multiple of 16 entries, got {n}")
    return torch.empty((a.shape[0], n // 16), dtype=torch.int16, device=a.device)


def _bits_dev(bits, V, n, name):
    if bits is None:
        return None
    if bits.dtype != torch.int16 or not bits.is_cuda or not bits.is_contiguous() or tuple(bits.shape) != (V, n // 16):
        raise ValueError(f"{name} must be a contiguous int16 device tensor of shape ({V}, {n // 16})")
    return bits


def lsc_fwd(plan: LSCPlan, a_in: torch.Tensor, W: torch.Tensor, bias=None, relu: bool = False, out=None,
            precision="fp32", workspace: Workspace | None = None, form=DEFAULT_FORM,
            out_dtype=torch.float32, relu_bits=None) -> torch.Tensor:
    """a_in [V][C][K_in], W [O][C][T] (or [O][C][1][T]), bias [O] -> a_out [V][O][K_out].
    a_in and a_out (`out`, else `out_dtype`) may be bfloat16 with precision
    "bf16" in the folded form: activations stored in bfloat16.
    relu_bits (with relu, folded form): an int16 [V][O*K_out/16] tensor that
    receives bit n%16 of word n/16 = [a_out[v].flat[n] > 0]."""
    a_in = _act_dev(a_in, "a_in")
    W = _f32_dev(W, "W").reshape(W.shape[0], W.shape[1], -1)
    V, Cin, Kin = a_in.shape
    O = W.shape[0]
    if Kin != plan.K_in or W.shape[1] != Cin or W.shape[2] != plan.T:
        raise ValueError(f"shapes: a_in {tuple(a_in.shape)}, W {tuple(W.shape)}, plan K_in={plan.K_in} T={plan.T}")
    if bias is not None:
        bias = _f32_dev(bias, "bias")
        if bias.numel() != O:
            raise ValueError("bias must have O entries")
    prec = precision_code(precision)
    ws = workspace or _default_ws(plan, Cin, O, V, prec, a_in.device, form)
    if out is None:
        out = torch.empty((V, O, plan.K_out), dtype=out_dtype, device=a_in.device)
    out = _act_dev(out, "out")
    io = (_lib.DLM_IO_IN_BF16 if a_in.dtype == torch.bfloat16 else 0) | \
        (_lib.DLM_IO_OUT_BF16 if out.dtype == torch.bfloat16 else 0)
    relu_bits = _bits_dev(relu_bits, V, O * plan.K_out, "relu_bits")
    check(lib().dlm_lsc_fwd_io(plan.handle, _ptr(a_in), Cin, _ptr(W), _ptr(bias), O, _ptr(out), V, int(bool(relu)),
                               io, _ptr(relu_bits), form_code(form), ws.ptr(), ws.nbytes, prec, _stream(a_in)))
    return out


def lsc_bwd(plan: LSCPlan, a_in: torch.Tensor, W: torch.Tensor, da_out: torch.Tensor, a_out=None, relu=False,
            need_input_grad=True, need_weight_grad=True, need_bias_grad=True, precision="fp32",
            workspace: Workspace | None = None, outs=None, form=DEFAULT_FORM, relu_in=False, relu_bits=None):
    """Returns (da_in or None, dW [O][C][T] or None, dbias [O] or None).
    relu: the forward fused a ReLU into a_out (da_out is masked by a_out > 0).
    relu_in: a_in is a ReLU output; da_in is returned masked by a_in > 0 (the
    gradient of the previous layer's pre-activation).
    `outs` = (da_in, dW, dbias) preallocated tensors (entries may be None).
    Activations may be bfloat16 (precision "bf16", folded form): da_in takes
    a_in's dtype, a_out (when given) must have da_out's.
    relu_bits (with relu_in, folded form): the ReLU bits lsc_fwd wrote for
    a_in; the relu_in mask is read from them instead of a_in (same result)."""
    a_in = _act_dev(a_in, "a_in")
    W = _f32_dev(W, "W").reshape(W.shape[0], W.shape[1], -1)
    da_out = _act_dev(da_out, "da_out")
    if relu:
        a_out = _act_dev(a_out, "a_out")
    V, Cin, _ = a_in.shape
    O = W.shape[0]
    prec = precision_code(precision)
    ws = workspace or _default_ws(plan, Cin, O, V, prec, a_in.device, form)
    dev = a_in.device
    o_da, o_dW, o_db = outs if outs is not None else (None, None, None)
    da_in = (o_da if o_da is not None else torch.empty_like(a_in)) if need_input_grad else None
    need_dW = need_weight_grad or need_bias_grad
    dW = (o_dW if o_dW is not None else torch.empty((O, Cin, plan.T), dtype=torch.float32, device=dev)) \
        if need_dW else None
    db = (o_db if o_db is not None else torch.empty((O,), dtype=torch.float32, device=dev)) if need_bias_grad else None
    flags = (_lib.DLM_RELU_OUT if relu else 0) | (_lib.DLM_RELU_IN if relu_in else 0)
    if da_in is not None and da_in.dtype != a_in.dtype:
        raise ValueError("da_in must have a_in's dtype")
    io = (_lib.DLM_IO_IN_BF16 if a_in.dtype == torch.bfloat16 else 0) | \
        (_lib.DLM_IO_OUT_BF16 if da_out.dtype == torch.bfloat16 else 0)
    relu_bits = _bits_dev(relu_bits, V, Cin * plan.K_in, "relu_bits")
    check(lib().dlm_lsc_bwd_io(plan.handle, _ptr(a_in), Cin, _ptr(W), O, _ptr(a_out if relu else None), _ptr(da_out),
                               _ptr(da_in), _ptr(dW), _ptr(db), V, flags, io, _ptr(relu_bits), form_code(form),
                               ws.ptr(), ws.nbytes, prec, _stream(a_in)))
    return da_in, (dW if need_weight_grad else None), db


# --------------------------------------------------------------- training
def mse_fwd_bwd(pred: torch.Tensor, target: torch.Tensor, need_grad: bool = True, outs=None):
    """(loss device scalar, dpred) for loss = mean((pred - target)^2).
    `outs` = (loss, dpred, workspace) preallocated tensors."""
    pred = _f32_dev(pred, "pred")
    target = _f32_dev(target, "target")
    if pred.shape != target.shape:
        raise ValueError("pred and target differ in shape")
    n = pred.numel()
    if outs is not None:
        loss, dpred, ws = outs
    else:
        ws = torch.empty(lib().dlm_mse_workspace_bytes(n), dtype=torch.uint8, device=pred.device)
        loss = torch.empty((), dtype=torch.float32, device=pred.device)
        dpred = torch.empty_like(pred) if need_grad else None
    check(lib().dlm_mse_fwd_bwd(_ptr(pred), _ptr(target), n, _ptr(loss), _ptr(dpred), _ptr(ws), ws.numel(),
                                _stream(pred)))
    return loss, dpred


def sh2signal_mse_supported(plan: SHPlan) -> bool:
    """Whether the fused loss head takes this plan (<= 96 directions per
    shell, K <= 64)."""
    return bool(lib().dlm_sh2signal_mse_supported(plan.handle))


def sh2signal_mse_fwd_bwd(plan: SHPlan, c: torch.Tensor, target: torch.Tensor, need_xhat: bool = False,
                          precision="fp32", outs=None, xhat_out=None):
    """The q-space loss head in one pass: (loss device scalar, dc [V][S][K],
    xhat [V][N_dw] or None) for xhat = SH2Signal(c) and loss =
    mean((xhat - target)^2), dc its gradient.  `outs` = (loss, dc, workspace)
    preallocated tensors; `xhat_out` a preallocated xhat (implies need_xhat)."""
    c = _f32_dev(c, "c")
    target = _f32_dev(target, "target")
    if c.dim() != 3 or tuple(c.shape[1:]) != (plan.n_shells, plan.K):
        raise ValueError(f"c must be [V, {plan.n_shells}, {plan.K}]")
    V = c.shape[0]
    if tuple(target.shape) != (V, plan.n_dw):
        raise ValueError(f"target must be [{V}, {plan.n_dw}]")
    if outs is not None:
        loss, dc, ws = outs
    else:
        ws = torch.empty(lib().dlm_sh2signal_mse_workspace_bytes(plan.handle, V), dtype=torch.uint8,
                         device=c.device)
        loss = torch.empty((), dtype=torch.float32, device=c.device)
        dc = torch.empty_like(c)
    xhat = xhat_out
    if xhat is not None:
        if tuple(xhat.shape) != (V, plan.n_dw) or xhat.dtype != torch.float32 or not xhat.is_contiguous():
            raise ValueError(f"xhat_out must be a contiguous float32 [{V}, {plan.n_dw}] tensor")
    elif need_xhat:
        xhat = torch.empty((V, plan.n_dw), dtype=torch.float32, device=c.device)
    check(lib().dlm_sh2signal_mse_fwd_bwd(plan.handle, _ptr(c), _ptr(target), V, _ptr(loss), _ptr(dc), _ptr(xhat),
                                          _ptr(ws), ws.numel(), precision_code(precision), _stream(c)))
    return loss, dc, xhat


def relmse_fwd_bwd(pred: torch.Tensor, target: torch.Tensor, eps: float = 1e-3, need_grad: bool = True):
    """(loss device scalar, dpred) for loss = mean(((pred - target) / (|target| + eps))^2)."""
    pred = _f32_dev(pred, "pred")
    target = _f32_dev(target, "target")
    if pred.shape != target.shape:
        raise ValueError("pred and target differ in shape")
    n = pred.numel()
    ws = torch.empty(lib().dlm_mse_workspace_bytes(n), dtype=torch.uint8, device=pred.device)
    loss = torch.empty((), dtype=torch.float32, device=pred.device)
    dpred = torch.empty_like(pred) if need_grad else None
    check(lib().dlm_relmse_fwd_bwd(_ptr(pred), _ptr(target), n, float(eps), _ptr(loss), _ptr(dpred), _ptr(ws),
                                   ws.numel(), _stream(pred)))
    return loss, dpred


def peak_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """The reference copy kernel: dst <- src (device tensors of equal byte size)."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("peak_copy needs contiguous device tensors")
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("peak_copy buffers differ in size")
    check(lib().dlm_peak_copy(_ptr(src), _ptr(dst), n, _stream(src)))


def peak_mfma(precision, blocks: int, iters: int, out: torch.Tensor) -> float:
    """Run the reference MFMA loop; returns the flops it does.  out: float32
    device tensor of at least lib().dlm_peak_mfma_out_floats(blocks) entries."""
    if out.dtype != torch.float32 or not out.is_cuda or out.numel() < lib().dlm_peak_mfma_out_floats(blocks):
        raise ValueError("out must be a float32 device tensor of blocks * 256 entries")
    prec = precision_code(precision)
    check(lib().dlm_peak_mfma(prec, int(blocks), int(iters), _ptr(out), _stream(out)))
    return float(lib().dlm_peak_mfma_flops(prec, int(blocks), int(iters)))


def timing_enable(on: bool = True) -> None:
    """Record a HIP event pair around every library launch (measurement only)."""
    check(lib().dlm_timing_enable(int(bool(on))))


def timing_reset() -> None:
    check(lib().dlm_timing_reset())


def timing_report() -> dict:
    """{tag: (total_ms, launches, algorithmic_bytes, algorithmic_flops)}; waits for recorded events."""
    n = lib().dlm_timing_count()
    out = {}
    for i in range(n):
        buf = C.create_string_buffer(128)
        ms, cnt, b, f = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
        check(lib().dlm_timing_entry(i, buf, 128, C.byref(ms), C.byref(cnt), C.byref(b), C.byref(f)))
        out[buf.value.decode()] = (ms.value, cnt.value, b.value, f.value)
    return out


def adam_step(w: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr=1e-3, beta1=0.9,
              beta2=0.999, eps=1e-8):
    for t, nm in ((w, "w"), (g, "g"), (m, "m"), (v, "v")):
        if not t.is_contiguous() or t.dtype != torch.float32 or not t.is_cuda:
            raise ValueError(f"{nm} must be a contiguous float32 CUDA tensor")
    check(lib().dlm_adam_step(_ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), float(lr), float(beta1), float(beta2),
                              float(eps), int(step), _stream(w)))
