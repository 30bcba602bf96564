"""The library's float64 host code (csrc/host_tables.cpp: SH basis, fits,
shell grouping, cyclic-kernel points, bfloat16 rounding) built with g++
-fsanitize=address,undefined and run on ordinary and edge inputs
(tests/host/sanitize_host_tables.cpp).  Any sanitizer report fails the
test; the printed values are checked against closed forms."""
import math
import os
import shutil
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def run(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "sanitize_host_tables")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "sanitize_host_tables.cpp"),
           os.path.join(ROOT, "paper_1808_01517_amd", "csrc", "host_tables.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    return r


def test_runs_clean_under_sanitizers(run):
    assert run.returncode == 0, run.stderr[-2000:]
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr


def test_values_match_closed_forms(run):
    lines = {}
    for ln in run.stdout.splitlines():
        parts = ln.split()
        lines.setdefault(parts[0], []).append(parts[1:])
    for L, s in lines["basis"]:
        want = sum((2 * l + 1) / (4 * math.pi) for l in range(0, int(L) + 1, 2))  # addition theorem
        assert abs(float(s) - want) < 1e-11
    for L, m, lam, ok, dev in lines["fit"]:
        K = (int(L) + 1) * (int(L) + 2) // 2
        if float(lam) > 0:
            assert ok == "1"  # the penalty makes every fit exist
        elif int(m) < K:
            assert ok == "0"  # fewer directions than coefficients
        else:
            assert ok == "1" and float(dev) < 1e-9  # P B = I
    assert lines["shells"][0] == ["3", "2@1005.0", "2@1995.0", "2@2995.0"]
    assert lines["shells_b0"][0] == ["0"]
    assert all(float(w) < 1e-14 for _, w in lines["points"])
    # round to nearest even on the float32 bits (ties to even, overflow to
    # infinity), NaN quiet: 1, 1 + 2^-8 (tie, down), 1 + 3 2^-8 (tie, up),
    # -2.5, 3e38 (largest finite range), 1e-40 (subnormal), +-0, inf, NaN
    want = []
    for f in (1.0, 1.00390625, 1.01171875, -2.5, 3.0e38, 1e-40, 0.0, -0.0, math.inf):
        u = struct.unpack("<I", struct.pack("<f", f))[0]
        want.append(f"{((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF:04x}")
    assert lines["bf16"][0][:9] == want
    assert want[:5] == ["3f80", "3f80", "3f82", "c020", "7f62"] and want[5] == "0001"
    nan = int(lines["bf16"][0][9], 16)
    assert nan & 0x7F80 == 0x7F80 and nan & 0x7F  # still a NaN
    assert lines["bf16d"][0] == ["3f80", "ff80"]
