"""Host replay of the tile engine's index arithmetic (tests/layout_check.cpp, built here with
hipcc; no GPU): LDS layout regions inside the layout and disjoint, fragment-ordered and
D-slot indices inside their buffers, fragment offsets a bijection, the activation scratch
index inside one workgroup's stride, for FP64, FP32, FP16 and BF16 at every tile width and
the workloads' network shapes."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_tile_engine_indices_stay_in_bounds(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "layout_check")
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-x", "hip",
                        os.path.join(HERE, "layout_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok "), out.stdout
