"""The bench's algorithmic byte model and its contract checks (CPU only)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("precision,expected", [("fp32", 470), ("fp32c", 408), ("fp16s", 370), ("bf16s", 370),
                                                ("fp64", 816)])
def test_channel_bytes_per_cell(precision, expected):
    """D3Q19 channel with a body force: populations read and written once,
    J, 6 g^{ij}, 54 coefficient words and 3 a_ext words; FP32 storage adds the
    6 lo words of g^{ij} and the deviation modes 19 16-bit references."""
    assert bench.algorithmic_bytes_per_cell(19, 3, precision, True) == expected


def test_fp32_mode_always_reads_a_ext():
    """Without a body force the FP32 mode still reads the a_ext words (they
    carry the rest-state compensation of the coefficient rounding); the O-grid
    adds the far-field U_inf words."""
    assert bench.algorithmic_bytes_per_cell(19, 3, "fp32", False, True) == 152 + (1 + 6 + 54 + 3 + 3 + 6) * 4 + 38
    assert bench.algorithmic_bytes_per_cell(19, 3, "fp32c", False, True) == 152 + (1 + 6 + 54 + 3) * 4


def test_batch_bytes_per_cell():
    """D2Q9 FP32 with deviation storage: 72 + 25 words x 4 + 18 = 190."""
    assert bench.algorithmic_bytes_per_cell(9, 2, "fp32", True) == 190


def test_moving_bytes_per_cell():
    """Moving D3Q19 mesh, FP64: 19 populations read and written (304 bytes),
    J, 6 g^{ij}, 9 g^i and 27 box words of g_i (344 bytes); D2Q9: 144 + (1 +
    3 + 4 + 12) x 8."""
    assert bench.moving_bytes_per_cell(19, 3) == 648
    assert bench.moving_bytes_per_cell(9, 2) == 304


def test_moving_basis_bytes():
    """D3Q19 on a 4x3x2 mesh (box 6x5x4 = 120 nodes): 3 words read and 9
    written per box node, 1 + 18 words written per cell."""
    assert bench.moving_basis_bytes(3, 24, 120) == 8 * (120 * 12 + 24 * 19)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
