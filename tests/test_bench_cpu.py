"""Host logic of bench.py (no GPU): shape parsing for --shapes, the one-GPU guard, the
algorithmic bytes the roofline is priced on, and the precision block's error statistics."""
import numpy as np
import pytest

import bench


def test_parse_shape():
    assert bench.parse_shape("cf16:64") == ("cf16", 64, 1, False, 3072)
    assert bench.parse_shape("cf32:10x2m") == ("cf32", 10, 2, True, 3000)   # the paper's mixed form
    assert bench.parse_shape("cf16:100") == ("cf16", 100, 1, False, 3000)   # 3072 % 100 != 0
    assert bench.parse_shape("cf16:61@2989") == ("cf16", 61, 1, False, 2989)
    for bad in ("cf8:64", "cf16:64@3000", "cf16:10x3"):                    # T % M, C % F
        with pytest.raises(ValueError):
            bench.parse_shape(bad)


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_algorithmic_bytes():
    # the FP32 baseline: 75 264 streams x (3072 x 32 B + 48 flag bytes + 36 B of average and weight)
    assert bench.algorithmic_bytes(1176 * 64, 3072, 64, 32) == 1176 * 64 * (3072 * 32 + 48 + 36) == 7405074432
    # windows of 10 x 2: one flag byte per window of a channel pair
    assert bench.algorithmic_bytes(1176 * 64, 3000, 10, 16, F=2) == 1176 * 64 * (3000 * 16 + 36) + 1176 * 32 * 300


def test_stat_errors_count_one_sided_non_finite_apart():
    stats = np.array([[[1.0, 0.2, 0.3], [np.nan, 0.1, 0.1], [np.inf, 0.5, 0.5], [np.nan, 0.4, 0.4]]], np.float32)
    ref = {"tau": np.array([[1.0, 2.0, np.inf, np.nan]]), "r_re": np.array([[0.2, 0.1, 0.5, 0.4]]),
           "r_im": np.array([[0.3, 0.1, 0.5, 0.4]])}
    e = bench.stat_errors(stats, ref)
    assert e["tau"]["nonfinite_one_side_frac"] == 0.25      # NaN against 2.0 only
    assert e["tau"]["max"] == 0.0                            # over windows finite on both sides
    assert e["r_re"]["max"] < 1e-7 and e["r_re"]["nonfinite_one_side_frac"] == 0.0
