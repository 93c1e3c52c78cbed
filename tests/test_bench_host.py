"""Host logic of bench.py (no GPU): the adjoint stage's roofline picks the nearer of its two roofs
and carries the other fraction along."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_adjoint_roof_bandwidth_side():
    r = bench.adjoint_roof(4.0e9, 1.0e9, 1.0e-3)          # 4 TB/s against 1 TFLOP/s
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(4000.0 / bench.HBM_PEAK_GBS, abs=1e-4)
    assert r["mfma_frac"] == pytest.approx(1.0 / bench.FP64_MFMA_PEAK_TF, abs=1e-4)


def test_adjoint_roof_matrix_core_side():
    r = bench.adjoint_roof(1.0e9, 40.0e9, 1.0e-3)         # 1 TB/s against 40 TFLOP/s
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(40.0)
    assert r["frac"] == pytest.approx(40.0 / bench.FP64_MFMA_PEAK_TF, abs=1e-4)
    assert r["hbm_frac"] == pytest.approx(1000.0 / bench.HBM_PEAK_GBS, abs=1e-4)
