"""The benchmark's byte model (host only): the per-stage algorithmic bytes sum
to 12 (N_g + N_r) + 50 R + 34 C per mock, the CPU-baseline line fit recovers a
known line, and the oracle picks are the smallest, the two medians and the
largest mock."""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_stage_bytes_sum_to_pipeline_bytes():
    for ng in (1_000_000, 3_370_000, 8_000_000):
        m = bench.stage_model(ng, 10 * ng)
        total = m["paint"] + m["fft"] + m["bin"] + m["contract"]
        assert total == bench.pipeline_bytes(ng, 10 * ng)
    R, C = 256 ** 3 * 4, 256 * 256 * 129 * 8
    assert bench.pipeline_bytes(0, 0) == 50 * R + 34 * C


def test_paint_roofline_per_launch():
    m = {"paint": 2 * (12 * 11_000_000 + 4 * 256 ** 3 * 4)}
    r = bench.paint_roofline(m, {"ms": 4 * 0.25, "launches": 4})
    assert r["per_launch"] == m["paint"] / 4
    assert abs(r["achieved"] - r["per_launch"] / 0.25e-3 / 1e9) < 1e-9


def test_fit_line_and_picks():
    x = np.array([1.0, 2.0, 5.0, 9.0])
    a, b = bench.fit_line(x, 3.0 * x + 7.0)
    assert abs(a - 3.0) < 1e-12 and abs(b - 7.0) < 1e-12
    sizes = np.array([5, 1, 9, 3, 7, 2])
    assert bench.cpu_picks(sizes) == [1, 3, 0, 2]
