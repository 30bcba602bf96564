"""CPU-side checks of libdelimit.so: it loads, exports every symbol the
header declares, its float64 host tables agree with the oracle, and its
argument validation returns the documented status codes.  No kernel runs."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import datagen as dg
from oracle import lsc as olsc
from oracle import sh as osh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1808_01517_amd import _lib
    return _lib


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "delimit.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dlm_[a-z0-9_]+)\s*\(", txt)))


def test_every_header_symbol_is_exported(L):
    lib = L.lib()
    syms = _header_symbols()
    assert len(syms) >= 25
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(L.SIGNATURES), set(syms) ^ set(L.SIGNATURES)


@pytest.mark.parametrize("order", [0, 2, 4, 8, 12, 16])
def test_basis_matches_oracle(L, order):
    g = dg.perturb_directions(dg.fibonacci_hemisphere(60), 3.0, dg.rng_for(5, 1, order))
    K = (order + 1) * (order + 2) // 2
    B = np.zeros((60, K))
    L.check(L.lib().dlm_sh_basis(order, L.dptr(np.ascontiguousarray(g)), 60, L.dptr(B)))
    assert np.abs(B - osh.basis_at(order, g)).max() < 1e-12


@pytest.mark.parametrize("order,n,lam", [(4, 30, 0.006), (8, 90, 0.006), (8, 90, 0.0), (4, 15, 0.006)])
def test_fit_matches_oracle(L, order, n, lam):
    g = dg.perturb_directions(dg.fibonacci_hemisphere(n), 2.0, dg.rng_for(6, 1, n))
    K = (order + 1) * (order + 2) // 2
    P = np.zeros((K, n))
    L.check(L.lib().dlm_sh_fit_matrix(order, L.dptr(np.ascontiguousarray(g)), n, lam, L.dptr(P)))
    ref = osh.fit_matrix(osh.basis_at(order, g), order, lam)
    assert np.abs(P - ref).max() < 1e-9 * max(1.0, np.abs(ref).max())


def test_kernel_points_match_oracle(L):
    g = dg.fibonacci_hemisphere(90)
    ks = (C.c_int * 3)(5, 8, 9)
    pts = np.zeros((90, 23, 3))
    L.check(L.lib().dlm_lsc_kernel_points(L.dptr(np.ascontiguousarray(g)), 90, ks, 3, 0.7, L.dptr(pts)))
    assert np.abs(pts - olsc.kernel_points(g, (5, 8, 9), 0.7)).max() < 1e-14


def test_status_codes(L):
    lib = L.lib()
    g = np.ascontiguousarray(dg.fibonacci_hemisphere(20))
    P = np.zeros((45, 20))
    assert lib.dlm_sh_fit_matrix(8, L.dptr(g), 20, 0.0, L.dptr(P)) == L.DLM_ESINGULAR
    assert b"singular" in lib.dlm_last_error()
    assert lib.dlm_sh_fit_matrix(3, L.dptr(g), 20, 0.0, L.dptr(P)) == L.DLM_EINVAL
    assert lib.dlm_sh_fit_matrix(4, L.dptr(g), 20, -1.0, L.dptr(P)) == L.DLM_EINVAL
    bad = g.copy()
    bad[3] = 0.0
    assert lib.dlm_sh_basis(4, L.dptr(bad), 20, L.dptr(np.zeros((20, 15)))) == L.DLM_EINVAL
    bad[3] = np.nan
    assert lib.dlm_sh_basis(4, L.dptr(bad), 20, L.dptr(np.zeros((20, 15)))) == L.DLM_EINVAL
    ks = (C.c_int * 1)(0)
    assert lib.dlm_lsc_kernel_points(L.dptr(g), 20, ks, 1, 0.5, L.dptr(np.zeros(20 * 3))) == L.DLM_EINVAL
    ks = (C.c_int * 1)(5)
    assert lib.dlm_lsc_kernel_points(L.dptr(g), 20, ks, 1, 4.0, L.dptr(np.zeros(20 * 18))) == L.DLM_EINVAL
    assert lib.dlm_status_str(L.DLM_EWORKSPACE) == b"workspace too small"
    # compute calls validate before touching the device
    assert lib.dlm_signal2sh_fwd(None, None, None, 10, 0, None) == L.DLM_EINVAL
    assert lib.dlm_lsc_fwd(None, None, 3, None, None, 3, None, 10, 0, 0, None, 0, 0, None) == L.DLM_EINVAL
    assert lib.dlm_mse_fwd_bwd(None, None, 0, None, None, None, 0, None) == L.DLM_EINVAL
    assert lib.dlm_adam_step(None, None, None, None, 5, 1e-3, 0.9, 0.999, 1e-8, 0, None) == L.DLM_EINVAL


def _header_param_counts():
    txt = open(os.path.join(ROOT, "include", "delimit.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    out = {}
    for name, params in re.findall(r"\b(dlm_[a-z0-9_]+)\s*\(([^;{}]*?)\)\s*;", txt, flags=re.S):
        params = params.strip()
        out[name] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_header_parameter_counts_match_bindings(L):
    """Every declaration's parameter count equals its ctypes binding's, so a
    signature change on one side cannot go unnoticed."""
    counts = _header_param_counts()
    assert set(counts) == set(L.SIGNATURES), set(counts) ^ set(L.SIGNATURES)
    bad = {n: (c, len(L.SIGNATURES[n][1])) for n, c in counts.items() if c != len(L.SIGNATURES[n][1])}
    assert not bad, bad


def test_relu_bits_host_helpers(L):
    import torch

    import paper_1808_01517_amd as dl
    a = torch.empty((7, 32, 45))
    b = dl.relu_bits_like(a)
    assert b.dtype == torch.int16 and tuple(b.shape) == (7, 90)
    assert tuple(dl.relu_bits_like(torch.empty((0, 64, 45))).shape) == (0, 180)
    with pytest.raises(ValueError):  # 3 x 45 entries per row
        dl.relu_bits_like(torch.empty((4, 3, 45)))
    with pytest.raises(ValueError):  # bits must live on the device
        dl._bits_dev(b, 7, 32 * 45, "relu_bits")
    assert dl._bits_dev(None, 7, 32 * 45, "relu_bits") is None
    # the entry points validate their plan before touching the device
    lib = L.lib()
    assert lib.dlm_lsc_fwd_io(None, None, 32, None, None, 3, None, 10, 1, 0, None, 1, None, 0, 0, None) == L.DLM_EINVAL
    assert lib.dlm_lsc_bwd_io(None, None, 32, None, 3, None, None, None, None, None, 10, 2, 0, None, 1, None, 0, 0,
                              None) == L.DLM_EINVAL
    # a bits pointer with no plan: rejected before anything is dereferenced
    words = (C.c_uint16 * 8)()
    assert lib.dlm_lsc_fwd_io(None, None, 3, None, None, 32, None, 10, 1, 0, words, 1, None, 0, 0, None) == L.DLM_EINVAL
    assert lib.dlm_lsc_bwd_io(None, None, 32, None, 3, None, None, None, None, None, 10, 2, 0, words, 1, None, 0, 0,
                              None) == L.DLM_EINVAL
