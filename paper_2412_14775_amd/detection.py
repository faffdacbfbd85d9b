"""Detection quality of the screen on synthetic data with known RFI (Section 4.2).

False-alarm probability  Pfa = flagged RFI-free windows / RFI-free windows,
missed-detection probability Pmd = unflagged RFI windows / RFI windows,
for the SK test alone, the DS test alone and both (ORed), as a function of the
interference-to-noise ratio, for polarised and for unpolarised RFI.  A window
counts as an RFI window when any of its samples holds RFI.

Every screen runs on the GPU through librfi; thresholds come from calibration
on an RFI-free realisation of the same array (the fine-tuning of Section 2.3).
Uses the repository's seeded generator ``synth`` (imported on call).
"""
from __future__ import annotations

import numpy as np


def _scene(synth, seed, N, C, T, inr_db, polarized, rng, model="voltage"):
    """Narrow-duration and narrowband sources at random places; pol_frac U[0.5, 0.9] when
    polarised (at most 90 % polarised, as at the horizon), fully unpolarised otherwise.
    model "voltage": injected into the station voltages (per-sample polarisation wanders
    around the mean state); model "post": added after correlation with a fixed coherency of
    that degree of polarisation (the simulation model of Section 4.2)."""
    srcs = []
    for _ in range(3):                                     # narrow duration, 1-2 channels
        start = int(rng.integers(0, T - 60))
        length = int(rng.integers(10, 60))
        env = synth.burst_envelope(T, [start], [length])
        c0 = int(rng.integers(0, C - 1))
        chans = [c0, c0 + 1] if rng.random() < 0.5 else [c0]
        srcs.append(synth.Rfi(chans, inr_db, float(rng.uniform(0, np.pi)), float(rng.uniform(-np.pi / 4, np.pi / 4)),
                              env, f0=float(rng.uniform(-0.5, 0.5)), unpolarized=not polarized,
                              pol_frac=float(rng.uniform(0.5, 0.9)) if polarized else 1.0))
    c = int(rng.integers(0, C))                            # narrowband, pulsed
    srcs.append(synth.Rfi([c], inr_db, float(rng.uniform(0, np.pi)), float(rng.uniform(-np.pi / 4, np.pi / 4)),
                          synth.pulse_train(T, int(rng.integers(100, 400)), int(rng.integers(10, 40)), 0),
                          f0=float(rng.uniform(-0.5, 0.5)), unpolarized=not polarized,
                          pol_frac=float(rng.uniform(0.5, 0.9)) if polarized else 1.0))
    if model == "post":
        post = [synth.PostRfi(s.channels, s.inr_db, s.theta, s.chi, s.envelope,
                              0.0 if s.unpolarized else s.pol_frac) for s in srcs]
        return synth.Scene(N, C, T, seed, rho=0.1, post_rfi=post)
    return synth.Scene(N, C, T, seed, rho=0.1, rfi=srcs)


def _window_truth(truth, M, F):
    C, T = truth.shape
    t = truth.reshape(C // F, F, T // M, M)
    return t.any(axis=(1, 3))                              # [C/F, T/M]


def detection_study(inrs_db=(-10, -5, 0, 5, 10, 20), realizations=4, N=6, C=16, T=2000, M=10, F=2,
                    fmt="cf32", pfa_sk=0.01, pfa_ds=0.01, seed=0, model="voltage"):
    """Pfa / Pmd table for SK, DS and BOTH, polarised and unpolarised RFI."""
    import torch

    import synth
    from . import rfi

    B = N * (N + 1) // 2
    dev = torch.device("cuda:0")

    def to_dev(vis):
        a = vis.view(np.float32).reshape(vis.shape + (2,))
        if fmt == "cf16":
            a = a.astype(np.float16)
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    base = rfi.rfi_params_default(n_stations=N, n_baselines=B, n_channels=C, n_samples=T, block_m=M,
                                  block_f=F, vis_format=rfi.RFI_VIS_CF16 if fmt == "cf16" else rfi.RFI_VIS_CF32,
                                  sk_d=2.0)
    null = synth.correlate(synth.make_voltages(synth.scene_null(N, C, T, seed=seed + 99_991)))
    cal = rfi.calibrate_on_null(base, to_dev(null), pfa_sk, pfa_ds)
    methods = {"SK": rfi.RFI_OPT_NO_DS, "DS": rfi.RFI_OPT_NO_SK, "BOTH": 0}
    rows = []
    rng = np.random.default_rng(seed)
    for polarized in (True, False):
        for ii, inr in enumerate(inrs_db):
            counts = {m: np.zeros(4, np.int64) for m in methods}     # fa, clean, md, rfi
            for k in range(realizations):
                sc = _scene(synth, seed * 100_000 + 1000 * ii + 17 * k + (0 if polarized else 500), N, C, T,
                            float(inr), polarized, rng, model)
                vis = to_dev(synth.correlate_scene(sc, synth.make_voltages(sc)))
                truth = _window_truth(synth.rfi_truth(sc), M, F)      # same for every baseline
                for name, opt in methods.items():
                    p = rfi.rfi_params_default(**{**base.as_dict(), **cal, "options": opt})
                    plan = rfi.Plan(p)
                    out = plan.alloc_outputs(flags=True, stats=False)
                    plan.screen(vis, out["avg"], out["weight"], out["flags"], None)
                    torch.cuda.synchronize()
                    flagged = out["flags"].cpu().numpy() != 0          # [B, C/F, T/M]
                    plan.close()
                    tr = np.broadcast_to(truth, flagged.shape)
                    counts[name] += [np.sum(flagged & ~tr), np.sum(~tr), np.sum(~flagged & tr), np.sum(tr)]
            for name, c in counts.items():
                rows.append(dict(polarized=polarized, inr_db=float(inr), method=name,
                                 pfa=float(c[0] / max(c[1], 1)), pmd=float(c[2] / max(c[3], 1)),
                                 rfi_windows=int(c[3])))
    return dict(calibration=cal, window=f"{M} x {F}", stations=N, channels=C, samples=T, model=model, rows=rows)


def format_table(study) -> str:
    lines = ["| RFI | INR (dB) | Pfa SK | Pmd SK | Pfa DS | Pmd DS | Pfa BOTH | Pmd BOTH |",
             "|---|---|---|---|---|---|---|---|"]
    by = {}
    for r in study["rows"]:
        by.setdefault((r["polarized"], r["inr_db"]), {})[r["method"]] = r
    for (pol, inr), m in by.items():
        lines.append(f"| {'polarised' if pol else 'unpolarised'} | {inr:g} | "
                     + " | ".join(f"{m[k]['pfa']:.3f} | {m[k]['pmd']:.3f}" for k in ("SK", "DS", "BOTH")) + " |")
    return "\n".join(lines)
