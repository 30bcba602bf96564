"""Error measures of the GPU parity tests (imported by the test modules).

Every comparison with the FP64 oracle is held to two bounds:

* norm-wise over the whole tensor, ||out - ref||_F / ||ref||_F:
  FP32 form <= 1e-5, BF16 form <= 2e-2 (the tolerances the workloads state);
* per voxel, for every per-voxel result (signals, coefficients,
  activations and their gradients; rows = first axis),
  max_v ||out_v - ref_v|| / max(||ref_v||, FLOOR * rms_v ||ref_v||);
  for sums over voxels (weight and bias gradients, kind="sum"), the largest
  entry error against the largest entry, max |out - ref| / max |ref|:
  FP32 <= 1e-4, BF16 <= 5e-2 for either.

The second bound catches what the first cannot: one wholly wrong voxel
among a few thousand moves the norm-wise error by only ~1/sqrt(V), but its
own row error is ~1 (and one wrong weight-gradient entry of typical size
is ~0.3 of the largest).  The floor keeps rows whose reference is near zero
(a voxel whose gradient the ReLU almost wholly masks) from turning rounding
of the size of the typical row into a large ratio.  A weight gradient's
entries are sums over voxels that may cancel, so a per-channel ratio would
measure that cancellation rather than the kernel; hence the max-normalised
entry error there.  Emulating the BF16 operand rounding on the CPU for the
SH transforms gives per-voxel errors of 1-3x the norm-wise error (max
6e-3), well inside 5e-2.
"""
from __future__ import annotations

import numpy as np

TOL = {"fp32": 1e-5, "bf16": 2e-2}
VOXEL_TOL = {"fp32": 1e-4, "bf16": 5e-2}
FLOOR = 0.1


def to64(a) -> np.ndarray:
    if hasattr(a, "detach"):
        return a.detach().double().cpu().numpy()
    return np.asarray(a, dtype=np.float64)


def rel(out, ref) -> float:
    """Norm-wise relative error over the whole tensor."""
    o, r = to64(out), to64(ref)
    return float(np.linalg.norm(o - r) / max(np.linalg.norm(r), 1e-300))


def row_err(out, ref, floor: float = FLOOR) -> float:
    """Largest per-row relative error (rows = first axis), each row's norm
    floored at `floor` times the RMS row norm."""
    o, r = to64(out), to64(ref)
    if o.shape != r.shape:
        raise ValueError(f"shapes differ: {o.shape} vs {r.shape}")
    if o.size == 0:
        return 0.0
    o = o.reshape(o.shape[0], -1)
    r = r.reshape(r.shape[0], -1)
    nr = np.linalg.norm(r, axis=1)
    ne = np.linalg.norm(o - r, axis=1)
    fl = max(floor * float(np.sqrt(np.mean(nr ** 2))), 1e-300)
    return float(np.max(ne / np.maximum(nr, fl)))


def entry_err(out, ref) -> float:
    """Largest entry error relative to the largest reference entry."""
    o, r = to64(out), to64(ref)
    if o.shape != r.shape:
        raise ValueError(f"shapes differ: {o.shape} vs {r.shape}")
    if o.size == 0:
        return 0.0
    return float(np.max(np.abs(o - r)) / max(float(np.max(np.abs(r))), 1e-300))


def check(name: str, out, ref, prec: str, errs: dict | None = None, scale: float = 1.0,
          kind: str = "voxel") -> tuple[float, float]:
    """Assert both bounds for `prec` ("fp32"/"bf16"), each times `scale`;
    record (norm-wise, per-voxel or entry) under `name` in `errs`.
    kind: "voxel" for per-voxel results, "sum" for sums over voxels."""
    if kind not in ("voxel", "sum"):
        raise ValueError(kind)
    e = rel(out, ref)
    v = row_err(out, ref) if kind == "voxel" else entry_err(out, ref)
    if errs is not None:
        errs[name] = (e, v)
    assert e <= TOL[prec] * scale, f"{name}: norm-wise error {e:.3e} > {TOL[prec] * scale:.1e}"
    assert v <= VOXEL_TOL[prec] * scale, f"{name}: {kind} error {v:.3e} > {VOXEL_TOL[prec] * scale:.1e}"
    return e, v


def fmt(errs: dict) -> str:
    """'name norm-wise/per-voxel' pairs for the [parity] log lines."""
    parts = []
    for k, v in errs.items():
        parts.append(f"{k} {v[0]:.2e}/{v[1]:.2e}" if isinstance(v, tuple) else f"{k} {v:.2e}")
    return ", ".join(parts)
