"""Why the adaptive state (the per-stream running null mean and variance of each statistic,
an extension the paper names as future work in Section 5) is kept in float64 on the GPU.

The integration's own moments (at most T / 2 windows) are summed in float32 by the kernels;
the running state they are merged into (Chan, Golub & LeVeque 1979) lives for the whole
observation.  This replays both designs in NumPy on synthetic null statistics, 48 windows
per integration as in the 48-station, M = 64 workload, against the FP64 oracle's
``AdaptiveState``: a float32 state drifts past the 1e-5 tolerance within a few 1e4
integrations (its M2, a sum that only grows, gains a rounding of about its own ulp at every
merge), while a float64 state fed float32 integration moments stays within 1e-7.
The GPU side of the same run is ``tests/test_gpu_adaptive.py::test_long_run_state_error``.
"""
import numpy as np

import oracle

F32 = np.float32


def _batch32(x):
    """One integration's moments in float32 (count, mean, sum of squared deviations)."""
    x32 = x.astype(F32)
    m = x32.mean(axis=-2, dtype=F32)
    d = (x32 - m[..., None, :]).astype(F32)
    return x.shape[-2], m, (d * d).sum(axis=-2, dtype=F32)


def test_float32_state_drifts_float64_state_does_not():
    rng = np.random.default_rng(5)
    S, nW, K = 8, 48, 30000
    ref = oracle.AdaptiveState((S,))
    keep = np.ones((S, nW), bool)
    n32, m32, s32 = np.zeros(S, F32), np.zeros((S, 3), F32), np.zeros((S, 3), F32)
    n64, m64, s64 = np.zeros(S, np.uint64), np.zeros((S, 3)), np.zeros((S, 3))
    for _ in range(K):
        x = np.stack([rng.normal(1.0, 0.18, (S, nW)), np.abs(rng.normal(0.0, 0.12, (S, nW))),
                      np.abs(rng.normal(0.0, 0.12, (S, nW)))], -1)            # tau, r_re, r_im
        ref.update(x, keep)
        nb, mb, sb = _batch32(x)
        # float32 state, float32 count (the former design)
        n1 = (n32 + F32(nb)).astype(F32)
        fb = (F32(nb) / n1).astype(F32)
        cross = (n32 * fb).astype(F32)
        d = (mb - m32).astype(F32)
        m32 = (m32 + d * fb[:, None]).astype(F32)
        s32 = (s32 + sb + d * d * cross[:, None]).astype(F32)
        n32 = n1
        # float64 state, exact count (the kernels' state_merge)
        fb = nb / (n64 + nb).astype(np.float64)
        cross = n64.astype(np.float64) * fb
        d = mb.astype(np.float64) - m64
        m64 = m64 + d * fb[:, None]
        s64 = s64 + sb.astype(np.float64) + d * d * cross[:, None]
        n64 = n64 + np.uint64(nb)
    assert np.array_equal(n64, ref.n)

    def rel(a, b):
        return float((np.abs(a - b) / np.maximum(np.abs(b), 1e-300)).max())

    e32 = max(rel(m32, ref.mean), rel(s32, ref.m2))
    e64 = max(rel(m64, ref.mean), rel(s64, ref.m2))
    print(f"after {K} integrations: float32 state {e32:.2e}, float64 state {e64:.2e}")
    assert e32 > 1e-5, e32          # the float32 state leaves the tolerance
    assert e64 < 1e-7, e64          # the float64 state does not
