"""Seeded synthetic inputs for the DELIMIT layers.

This module produces *inputs only*: gradient tables, b-values, diffusion
signals, initial weights and direction subsets.  It holds none of the
layers' arithmetic (no spherical-harmonic basis, no least-squares fit, no
local spherical convolution) and imports neither the oracle nor the HIP
package, so both sides can draw identical inputs from it.

The workloads stand in for the paper's data: a full brain scan of about
450 000 voxels (Sec. 2.2, Efficiency paragraph) and Human Connectome
Project volumes (Sec. 3), neither of which is available.  Signals follow a
1-3 fibre stick + ball model with Rician noise, sampled on multi-shell
Fibonacci-hemisphere tables with a small seeded angular perturbation, which
mimics the per-scan distortion of gradient directions (Sec. 1).

Random streams: NumPy PCG64 seeded with SeedSequence([config, stream, index]);
stream 1 = gradient tables (index = shell), 2 = training/bench data
(index = chunk), 3 = held-out data, 4 = per-batch distortion, 5 = weights.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

STREAM_TABLES = 1
STREAM_DATA = 2
STREAM_HELDOUT = 3
STREAM_DISTORT = 4
STREAM_WEIGHTS = 5

DIFFUSIVITY = 1.7e-3  # mm^2/s, stick and ball


def rng_for(config: int, stream: int, index: int = 0) -> np.random.Generator:
    """Independent PCG64 stream for (config, stream, index)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(config), int(stream), int(index)])))


def fibonacci_hemisphere(n: int) -> np.ndarray:
    """n unit vectors on the upper hemisphere (z in (0,1)), golden-angle spiral."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (i + 0.5) / n
    phi = i * np.pi * (3.0 - np.sqrt(5.0))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def _tangent_basis(g: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Orthonormal pair spanning the tangent plane at each row of g."""
    helper = np.where(np.abs(g[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = np.cross(g, helper)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(g, e1)
    return e1, e2


def perturb_directions(g: np.ndarray, max_deg: float, rng: np.random.Generator) -> np.ndarray:
    """Rotate each direction by delta ~ U[0, max_deg] degrees about a uniformly
    random tangent axis (Rodrigues' formula with the axis orthogonal to g)."""
    g = np.asarray(g, dtype=np.float64)
    g = g / np.linalg.norm(g, axis=1, keepdims=True)
    n = g.shape[0]
    delta = np.deg2rad(rng.uniform(0.0, max_deg, size=n))
    beta = rng.uniform(0.0, 2.0 * np.pi, size=n)
    e1, e2 = _tangent_basis(g)
    k = np.cos(beta)[:, None] * e1 + np.sin(beta)[:, None] * e2
    out = g * np.cos(delta)[:, None] + np.cross(k, g) * np.sin(delta)[:, None]
    return out / np.linalg.norm(out, axis=1, keepdims=True)


def random_unit_vectors(n: int, rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@dataclass
class Acquisition:
    """A multi-shell gradient table.

    bvecs/bvals list every volume, b0 volumes first, then the diffusion
    weighted volumes shell by shell (shell-major, increasing b)."""
    bvecs: np.ndarray            # (n_total, 3)
    bvals: np.ndarray            # (n_total,)
    shell_b: list = field(default_factory=list)
    shell_dirs: list = field(default_factory=list)   # per shell (N_s, 3)
    n_b0: int = 0

    @property
    def dw_bvecs(self) -> np.ndarray:
        return np.concatenate(self.shell_dirs, axis=0)

    @property
    def dw_bvals(self) -> np.ndarray:
        return np.concatenate([np.full(d.shape[0], b) for b, d in zip(self.shell_b, self.shell_dirs)])


def make_acquisition(config: int, shell_b, dirs_per_shell: int, max_perturb_deg: float, n_b0: int) -> Acquisition:
    """Per-shell Fibonacci hemisphere tables, each with its own seeded perturbation."""
    base = fibonacci_hemisphere(dirs_per_shell)
    dirs = []
    for s, _ in enumerate(shell_b):
        dirs.append(perturb_directions(base, max_perturb_deg, rng_for(config, STREAM_TABLES, s)))
    b0_vecs = np.zeros((n_b0, 3))
    bvecs = np.concatenate([b0_vecs] + dirs, axis=0)
    bvals = np.concatenate([np.zeros(n_b0)] + [np.full(dirs_per_shell, float(b)) for b in shell_b])
    return Acquisition(bvecs=bvecs, bvals=bvals, shell_b=[float(b) for b in shell_b], shell_dirs=dirs, n_b0=n_b0)


def distort_acquisition(acq: Acquisition, max_deg: float, rng: np.random.Generator) -> Acquisition:
    """A fresh distortion of every diffusion-weighted direction (shell structure kept)."""
    dirs = [perturb_directions(d, max_deg, rng) for d in acq.shell_dirs]
    bvecs = np.concatenate([np.zeros((acq.n_b0, 3))] + dirs, axis=0)
    return Acquisition(bvecs=bvecs, bvals=acq.bvals.copy(), shell_b=list(acq.shell_b), shell_dirs=dirs, n_b0=acq.n_b0)


def _stick_ball_clean(dirs: np.ndarray, bvals: np.ndarray, fracs: np.ndarray, sticks: np.ndarray,
                      nf: np.ndarray, d: float) -> np.ndarray:
    """Noise-free S/S0 for every voxel at every (direction, b) pair.

    fracs: (V, 1+nmax) ball fraction first; sticks: (V, nmax, 3); nf: (V,)."""
    V = fracs.shape[0]
    nmax = sticks.shape[1]
    out = fracs[:, :1] * np.exp(-bvals * d)[None, :]
    for k in range(nmax):
        cos = sticks[:, k, :] @ dirs.T                       # (V, n)
        term = np.exp(-(bvals[None, :] * d) * cos * cos)
        active = (nf > k).astype(np.float64)[:, None]
        out = out + active * fracs[:, 1 + k:2 + k] * term
    return out


def _rician(clean: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    n1 = rng.standard_normal(clean.shape)
    n2 = rng.standard_normal(clean.shape)
    return np.sqrt((clean + sigma * n1) ** 2 + (sigma * n2) ** 2)


@dataclass
class SignalBatch:
    """Synthetic voxels on one acquisition.

    x      : (V, N_dw) b0-normalised noisy DW signal, shell-major
    clean  : (V, N_dw) noise-free S/S0 on the same table
    raw_b0 : (V, n_b0) noisy b0 volumes (empty when n_b0 == 0)
    params : fibre parameters so the same voxels can be re-sampled on
             another table (fracs, sticks, nf)"""
    x: np.ndarray
    clean: np.ndarray
    raw_b0: np.ndarray
    params: tuple


def stick_ball_batch(acq: Acquisition, V: int, nf_max: int, snr: float, rng: np.random.Generator,
                     dtype=np.float64) -> SignalBatch:
    """1..nf_max sticks + a ball, Dirichlet(1,...,1) fractions, uniform fibre
    orientations, S0 = 1, Rician noise sigma = 1/snr, divided by the mean of
    the noisy b0 volumes when the table has any (otherwise S0 = 1 is known)."""
    nf = rng.integers(1, nf_max + 1, size=V)
    alpha = np.ones(1 + nf_max)
    fr = rng.gamma(alpha[None, :].repeat(V, 0))              # Dirichlet via gammas
    mask = np.concatenate([np.ones((V, 1)), (np.arange(nf_max)[None, :] < nf[:, None]).astype(np.float64)], 1)
    fr = fr * mask
    fracs = fr / fr.sum(axis=1, keepdims=True)
    sticks = random_unit_vectors(V * nf_max, rng).reshape(V, nf_max, 3)
    dirs = acq.dw_bvecs
    bv = acq.dw_bvals
    clean = _stick_ball_clean(dirs, bv, fracs, sticks, nf, DIFFUSIVITY)
    sigma = 1.0 / snr
    noisy = _rician(clean, sigma, rng)
    if acq.n_b0 > 0:
        b0 = _rician(np.ones((V, acq.n_b0)), sigma, rng)
        x = noisy / b0.mean(axis=1, keepdims=True)
    else:
        b0 = np.zeros((V, 0))
        x = noisy
    return SignalBatch(x=x.astype(dtype), clean=clean.astype(dtype), raw_b0=b0.astype(dtype),
                       params=(fracs, sticks, nf))


def resample_clean(params: tuple, acq: Acquisition) -> np.ndarray:
    """Noise-free S/S0 of the same voxels on another table."""
    fracs, sticks, nf = params
    return _stick_ball_clean(acq.dw_bvecs, acq.dw_bvals, fracs, sticks, nf, DIFFUSIVITY)


def farthest_point_subset(dirs: np.ndarray, k: int) -> np.ndarray:
    """Greedy farthest-point choice of k of the given axes (antipodal angle
    arccos|g.h|), starting from index 0.  Returns sorted indices."""
    g = dirs / np.linalg.norm(dirs, axis=1, keepdims=True)
    chosen = [0]
    dmin = np.arccos(np.clip(np.abs(g @ g[0]), 0.0, 1.0))
    for _ in range(1, k):
        nxt = int(np.argmax(dmin))
        chosen.append(nxt)
        dmin = np.minimum(dmin, np.arccos(np.clip(np.abs(g @ g[nxt]), 0.0, 1.0)))
    return np.array(sorted(chosen), dtype=np.int64)


def lsc_weights(config: int, layer: int, C: int, O: int, T: int, dtype=np.float64):
    """Seeded U(-1/sqrt(C*T), +1/sqrt(C*T)) kernel [O][C][T] and bias [O]."""
    rng = rng_for(config, STREAM_WEIGHTS, layer)
    bound = 1.0 / np.sqrt(C * T)
    W = rng.uniform(-bound, bound, size=(O, C, T))
    b = rng.uniform(-bound, bound, size=(O,))
    return W.astype(dtype), b.astype(dtype)


# ---------------------------------------------------------------------------
# Workload definitions.  Each mirrors one of the five configurations: sizes,
# shells, orders, channel widths, kernel rings and noise levels.
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    config: int
    shell_b: tuple
    dirs_per_shell: int
    n_b0: int
    perturb_deg: float
    sh_order: int
    lb_lambda: float
    voxels: int
    nf_max: int
    snr: float
    channels: tuple          # LSC widths, first = number of shells
    kernel_sizes: tuple      # points per ring
    angular_distance: float  # radians, outer ring
    sh_order_lsc_in: int
    sh_order_lsc_out: int


C1 = Workload("c1-plain-fp64-1shell-30dir-L4", 0, (1000.0,), 30, 0, 2.0, 4, 0.006, 4096, 2, 30.0,
              (1, 8), (6, 6), np.deg2rad(30.0), 4, 4)
C2 = Workload("c2-3shell-90dir-L8-lsc3-32-3-1Mvox", 1, (1000.0, 2000.0, 3000.0), 90, 18, 2.0, 8, 0.006,
              1 << 20, 3, 20.0, (3, 32, 3), (8, 8), np.deg2rad(30.0), 8, 8)
C4 = Workload("c4-3shell-90dir-L8-lsc3-32-64-32-3-batch8192", 3, (1000.0, 2000.0, 3000.0), 90, 18, 2.0, 8,
              0.006, 8192, 3, 20.0, (3, 32, 64, 32, 3), (8, 8), np.deg2rad(30.0), 8, 8)
C5 = Workload("c5-learned-15of90-L4to8-lsc3-64-64-3", 4, (1000.0, 2000.0, 3000.0), 90, 18, 2.0, 8, 0.006,
              1 << 22, 3, 20.0, (3, 64, 64, 3), (8, 8), np.deg2rad(30.0), 4, 8)


def lsc_sampled_gradients(w: Workload) -> np.ndarray:
    """LSC output directions: the unperturbed Fibonacci hemisphere of the
    workload's per-shell size (the acquired table itself for the one-shell case)."""
    return fibonacci_hemisphere(w.dirs_per_shell)
