"""Input cases shared by the GPU parity tests and their CPU-side checks (no GPU needed here)."""
from __future__ import annotations

import math

import numpy as np

import oracle
import synth
from tests.gpu_helpers import TOL_F16_TOTAL, TOL_F32, stat_error


def thresholds_for(M, d=2.1):
    """Plan thresholds near the 2.5 / 97.5 % null quantiles (SK) and the 95 % DS quantile."""
    sd = 1.7 / math.sqrt(M)
    return dict(d=d, s_low=max(0.05, 1.0 - 2.0 * sd), s_high=1.0 + 2.3 * sd,
                gamma=min(0.95, math.sqrt(7.815 / (3 * M))))


def scene_vis(N, C, T, seed, rfi_channels=(1,), inr=8.0, duty=(40, 7)):
    env = synth.pulse_train(T, duty[0], duty[1], 3)
    sc = synth.Scene(N, C, T, seed, rho=0.1,
                     rfi=[synth.Rfi(list(rfi_channels), inr, 0.7, 0.2, env, f0=0.11)])
    return synth.correlate(synth.make_voltages(sc))


def storage_error(vis, op: "oracle.Params") -> float:
    """Largest statistic error that complex-half storage alone causes: the oracle on the
    FP16-rounded input against the oracle on the complex64 input (relative, as stat_error)."""
    a = oracle.screen(vis, op)
    b = oracle.screen(synth.to_cf16(vis), op)
    return max(float(stat_error(b[k], a[k]).max()) for k in ("tau", "r_re", "r_im"))


def cf16_total_tolerance(vis, op: "oracle.Params") -> float:
    """Total-error tolerance of complex-half storage: 3e-3, unless the storage rounding alone
    already exceeds it (short windows, where (W d + 1) / (W - 1) amplifies it: W = 2 on these
    inputs); then what storage causes plus the 1e-5 of FP32 arithmetic.  A kernel within 1e-5
    of the oracle on the FP16 bytes cannot do better than that."""
    s = storage_error(vis, op)
    return TOL_F16_TOTAL if s <= TOL_F16_TOTAL - TOL_F32 else s + TOL_F32


def exempt_shapes():
    """The complex-half parity cases with windows of fewer than 16 samples, built exactly as
    tests/test_gpu_screen.py builds them: (label, vis, oracle.Params)."""
    out = []
    for M in (2, 4, 8):
        T = M * max(3, 1600 // M)
        out.append((f"M={M}", scene_vis(2, 5, T, seed=M), oracle.Params(M=M, **thresholds_for(M))))
    for M, T in ((3, 300), (10, 400)):
        out.append((f"M={M}", scene_vis(2, 3, T, seed=M + 7, duty=(60, 20)),
                    oracle.Params(M=M, **thresholds_for(M))))
    return out
