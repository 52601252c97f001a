"""Host-side parts of bench.py (no GPU): the one-GPU refusal, the byte model of the
roofline and the dtype labels."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_residual_pass_bytes_clinical():
    """The dominant kernel's algorithmic bytes on the clinical plan: every stored entry
    once (int32 index, FP32 D and L), the fluence once, 78 bytes of per-row data."""
    R, C, nnz = 457_793, 12_000, 154_936_615
    b = bench.algorithmic_bytes("fwd_resid", R, C, nnz, 4, 0, 0, 0, 0)
    assert b == nnz * 12 + 4 * C + 78 * R == 1_894_995_234
    # 16-bit values with 16-bit indices: 6 bytes per entry
    b16 = bench.algorithmic_bytes("fwd_resid", R, C, nnz, 2, 0, 0, 0, 0, ib=2)
    assert b16 == nnz * 6 + 4 * C + 78 * R


def test_objective_passes_price_the_view():
    R, C, nnz = 1000, 100, 50_000
    full = bench.algorithmic_bytes("fwd_obj", R, C, nnz, 4, 0, 0, 100, 0)
    view = bench.algorithmic_bytes("fwd_obj", R, C, nnz, 4, 0, 0, 100, 5_000)
    assert view == 5_000 * 12 + 4 * C + 100 * 30 and full == nnz * 12 + 4 * C + R * 30
    assert bench.algorithmic_bytes("scatter", R, C, nnz, 4, 0, 0, 0, 0) == 0
    with pytest.raises(KeyError):
        bench.algorithmic_bytes("no_such_kernel", R, C, nnz, 4, 0, 0, 0, 0)


def test_dtype_labels():
    assert bench.dtype_of("f32") == "f32"
    assert "f16" in bench.dtype_of("f16") and "outside" not in bench.dtype_of("f16")
    for st in ("bf16", "bf16i16"):
        assert "outside" in bench.dtype_of(st)
