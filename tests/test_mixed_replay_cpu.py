"""The kernel-order replay of the mixed form (tests/mixed_replay.py) against the oracle's
sequential form (oracle/mixed.py) on the CPU: identical up to the derived order bound, and
both binary16 values.  Pins the tolerance the GPU test uses, which is derived, not fitted."""
import math

import numpy as np
import pytest

import oracle
from tests.mixed_replay import U16, lanes_for, mixed_stats_tree, r_order_bound


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * math.sqrt(0.5)


@pytest.mark.parametrize("M,F", [(10, 2), (5, 4), (20, 1), (16, 1), (16, 2)])
def test_tree_order_within_bound_of_sequential(M, F):
    rng = np.random.default_rng(7 + M * F)
    C, T = 4 * F, 40 * M
    vis = (_cn(rng, (6, C, T, 4)) * np.exp(rng.normal(0, 0.5, (6, C, 1, 1)))).astype(np.complex64)
    # a polarised pulse in part of the windows: sums near W, where binary16 ulps are largest
    vis[:, :F, ::3] += np.array([1.0, 0.4 + 0.3j, 0.4 - 0.3j, 0.5], np.complex64) * 4
    p = oracle.Params(M=M, F=F, d=1.9).f32()
    K, S, L = lanes_for(M, F)
    tau_t, re_t, im_t = mixed_stats_tree(vis, M, F, p.d, p.eps)
    tau_s, re_s, im_s = oracle.mixed_window_stats(oracle.window_view(vis, M, F), p.d, p.eps)
    for v in (tau_t, re_t, im_t):
        fin = np.isfinite(v)
        assert np.array_equal(v[fin].astype(np.float16).astype(np.float32), v[fin])   # binary16 values
    bound = r_order_bound(M * F, K, L)
    for t, s in ((re_t, re_s), (im_t, im_s)):
        diff = np.abs(t.astype(np.float64) - s.astype(np.float64))
        assert diff.max() <= bound, (diff.max(), bound)
        print(f"{M}x{F}: K={K} L={L}: max |r_tree - r_seq| {diff.max():.2e} (bound {bound:.2e}), "
              f"identical in {np.mean(diff == 0):.3f} of windows")
    # tau: identical S1, S2 roundings except where an FP32 sum lands on the other side of a
    # binary16 rounding boundary: one binary16 ulp of the ratio, times the prefactor
    fin = np.isfinite(tau_s)
    assert np.array_equal(np.isfinite(tau_t), fin)
    pre = (M * F * p.d + 1) / (M * F - 1)
    ulp = 2 * U16 * np.maximum(1.0, np.abs(tau_s[fin].astype(np.float64)) / pre + 1)
    assert np.all(np.abs(tau_t[fin].astype(np.float64) - tau_s[fin]) <= 2 * pre * ulp + 4 * U16 * np.abs(tau_s[fin]))
