"""bench.py on the host: more than one GPU is refused before any GPU work,
and the byte counts it prices launches with are the method's figures."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_algorithmic_bytes():
    # five FP32 pools read and written plus the 6-slot int32 table
    assert bench.BYTES_FUSED_F32 == 5 * 4 * 2 + 6 * 4 == 64
    # the same in FP64
    assert bench.BYTES_FUSED_F64 == 5 * 8 * 2 + 6 * 4 == 104
