"""Writes tests/golden/plain_case_oracle.npz: the FP64 oracle's statistics, flags, masked
averages and weights for the plain case (4 stations, 16 channels, 256 samples, M = 16,
seed 0; a 10 %-duty polarised pulse train at 10 dB in channels 3 and 11).

Calls only the oracle and the seeded generator.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

PARAMS = dict(M=16, d=2.1, s_low=0.15, s_high=1.98, gamma=0.4)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plain_case_oracle.npz")


def compute():
    vis = synth.correlate(synth.make_voltages(synth.scene_plain(0)))
    out = oracle.screen(vis, oracle.Params(**PARAMS))
    return vis, out


if __name__ == "__main__":
    _, out = compute()
    np.savez_compressed(OUT, tau=out["tau"], r_re=out["r_re"], r_im=out["r_im"], flags=out["flags"],
                        avg=out["avg"], weight=out["weight"],
                        params=np.array([PARAMS[k] for k in ("M", "d", "s_low", "s_high", "gamma")]))
    print("wrote", OUT)
