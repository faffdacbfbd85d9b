"""Benchmark of the online SK + DS RFI screen on one MI355X.

Workload (one step = one integration screened = one rfi_screen call):
  48 stations (1176 baselines incl. autos), 64 channels, 3072 samples per 1 s
  integration, window M = 64, complex64 visibilities (7.40 GB), synthetic
  voltage-level noise with sky correlation 0.1 and pulsed, randomly polarised
  RFI in 5 % of the channels.  The same array stored as complex half (3.70 GB)
  is timed as the precision form.

Prints one JSON line: samples screened per second (complex64 form = ``value``),
the complex-half form, per-integration latency p50 / p99 against the 1 s
deadline, the HBM roofline of the screen kernel (HIP events on the launch
stream), the read-bandwidth probe, and the FP64 oracle timed on the host's
cores on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       python bench.py --shapes cf16:64 cf16:10x2 cf32:10x2m ... [--steps K] [--warmup W]
         (times only the listed window shapes; for profiling single kernels)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
N_STATIONS, N_CHANNELS, N_SAMPLES, BLOCK_M = 48, 64, 3072, 64
SEED = 1
# plan thresholds for M = 64 (null quantiles of this generator: SK 2.5 / 97.5 %, DS 95 %)
PLAN = dict(sk_d=2.2, sk_low=0.656, sk_high=1.487, ds_gamma=0.202)
CPU_SAMPLE_BASELINES = 1176         # baselines (x all 64 channels): the whole integration, 15-20 s of CPU work on 16 cores


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for name in ("screen.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_2412_14775_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n_streams: int, T: int, M: int, sample_bytes: int, F: int = 1) -> int:
    """Bytes one screen must move: every sample read once, one flag byte per window (of F
    channels), average (8 floats) and weight (1 float) per stream."""
    return n_streams * (T * sample_bytes + 36) + n_streams // F * (T // M)


# ----------------------------------------------------------------------------- CPU baseline

_CPU_VIS = None
_CPU_M = BLOCK_M


def _oracle_chunk(bounds):
    import oracle
    b0, b1 = bounds
    p = oracle.Params(M=_CPU_M, d=PLAN["sk_d"], s_low=PLAN["sk_low"], s_high=PLAN["sk_high"],
                      gamma=PLAN["ds_gamma"])
    out = oracle.screen(_CPU_VIS[b0:b1], p)
    return int((out["flags"] != 0).sum())


def _time_oracle(vis: np.ndarray, M: int, workers: int, per_task: int = 2) -> float:
    """Seconds the oracle takes over ``vis`` [B, C, T, 4] in a pool of ``workers`` processes
    (forked before any GPU use; ``per_task`` baselines per task)."""
    global _CPU_VIS, _CPU_M
    _CPU_VIS, _CPU_M = vis, M
    chunks = [(i, min(i + per_task, vis.shape[0])) for i in range(0, vis.shape[0], per_task)]
    try:
        with mp.get_context("fork").Pool(workers) as pool:
            pool.map(_oracle_chunk, chunks[:workers])              # warm the workers
            t0 = time.perf_counter()
            pool.map(_oracle_chunk, chunks, chunksize=1)
            return time.perf_counter() - t0
    finally:
        _CPU_VIS = None


def cpu_baseline(e: np.ndarray) -> dict:
    """FP64 oracle on bounded samples of two workloads, in a process pool over every core this
    process may run on.  Data generation is outside the timed region; only the oracle's
    compute is timed.
      * the FP32 baseline (48 stations, 64 channels, 3072 samples, M = 64): CPU_SAMPLE_BASELINES
        of its 1176 baselines (seeded; all of them by default, the whole integration), all
        channels and samples;
      * the 64-station mixed case (2080 baselines, 256 channels, M = 64): a seeded 1 % of its
        (baseline, channel) streams (21 baselines, all channels), extrapolated as samples/s."""
    try:
        workers = len(os.sched_getaffinity(0))
    except AttributeError:
        workers = os.cpu_count() or 1
    rng = np.random.default_rng(1234)
    bl = np.sort(rng.choice(synth.n_baselines(N_STATIONS), CPU_SAMPLE_BASELINES, replace=False))
    vis = synth.correlate(e, bl)                                   # [Bs, C, T, 4] complex64
    n = vis.shape[0] * vis.shape[1] * vis.shape[2]
    dt = _time_oracle(vis, BLOCK_M, workers)
    del vis
    sc3 = synth.scene_mixed(3)
    bl3 = np.sort(np.random.default_rng(4321).choice(sc3.n_baselines, 21, replace=False))
    vis3 = synth.correlate(synth.make_voltages(sc3), bl3)          # 1.0 % of the streams
    n3 = vis3.shape[0] * vis3.shape[1] * vis3.shape[2]
    dt3 = _time_oracle(vis3, 64, workers, per_task=1)
    del vis3
    return {"value": n / dt, "unit": "samples/s", "cores": workers, "kind": "oracle",
            "host_cpu_count": os.cpu_count(),
            "sample": f"{len(bl)} of 1176 baselines x 64 channels x 3072 samples "
                      f"({n / 1e6:.1f} M samples, complex64, M=64), FP64 NumPy oracle, "
                      f"{workers} worker processes (all cores this process may use; os.cpu_count() "
                      f"= {os.cpu_count()}), {dt:.2f} s wall",
            "mixed_case_c3": {"value": n3 / dt3, "unit": "samples/s", "cores": workers,
                              "sample": f"21 of 2080 baselines x 256 channels x 3072 samples "
                                        f"(1.0 % of the streams, {n3 / 1e6:.1f} M samples, M=64), "
                                        f"{dt3:.2f} s wall; samples/s extrapolate to the whole "
                                        f"26.2 GB integration"}}


PREC_BASELINES = 16                 # seeded baselines (x all channels) for the precision block
TF_PLAN = dict(sk_d=2.2, sk_low=0.42, sk_high=2.0, ds_gamma=0.40)   # 10 x 2 windows (W = 20)


def precision_references(e: np.ndarray, e3000: np.ndarray) -> dict:
    """FP64 oracle outputs of a seeded sample of baselines (one autocorrelation and crosses,
    all channels) of the FP32-baseline workload (its complex64 bytes, and the same bytes
    rounded to complex half) and of the 10 x 2 workload (3000 samples).  The GPU screens
    exactly these bytes: bench.py writes them over the same baselines of the device arrays."""
    import oracle
    rng = np.random.default_rng(99)
    B = synth.n_baselines(N_STATIONS)
    bl = np.sort(np.concatenate([[0], rng.choice(np.arange(1, B), PREC_BASELINES - 1, replace=False)]))
    v = synth.correlate(e, bl)
    p = oracle.Params(M=BLOCK_M, d=PLAN["sk_d"], s_low=PLAN["sk_low"], s_high=PLAN["sk_high"],
                      gamma=PLAN["ds_gamma"])
    keep = ("tau", "r_re", "r_im", "flags")
    ref32 = oracle.screen(v, p)
    ref16 = oracle.screen(synth.to_cf16(v), p)
    v3000 = synth.correlate(e3000, bl)
    p10 = oracle.Params(M=10, F=2, d=TF_PLAN["sk_d"], s_low=TF_PLAN["sk_low"], s_high=TF_PLAN["sk_high"],
                        gamma=TF_PLAN["ds_gamma"])
    ref10 = oracle.screen(v3000, p10)
    return dict(bl=bl, vis=v, vis3000=v3000, ref32={k: ref32[k] for k in keep},
                ref16={k: ref16[k] for k in keep}, ref10={k: ref10[k] for k in keep})


def stat_errors(stats: np.ndarray, ref: dict) -> dict:
    """max and p99 over windows of |gpu - oracle| / max(1, |oracle|) per statistic, over the
    windows where both are finite; windows that are NaN or infinite on one side only (the
    paper's mixed form overflows binary16 where W S2 is large) are counted apart, as a
    fraction, and windows non-finite on both sides count as equal."""
    out = {}
    for k, name in enumerate(("tau", "r_re", "r_im")):
        g = stats[..., k].astype(np.float64)
        o = ref[name]
        fin = np.isfinite(g) & np.isfinite(o)
        one_side = np.isfinite(g) != np.isfinite(o)
        err = np.abs(g[fin] - o[fin]) / np.maximum(1.0, np.abs(o[fin]))
        out[name] = {"max": float(np.max(err)) if err.size else 0.0,
                     "p99": float(np.percentile(err, 99)) if err.size else 0.0,
                     "nonfinite_one_side_frac": float(np.mean(one_side))}
    return out


def flag_disagreement(a: np.ndarray, b: np.ndarray) -> dict:
    """Windows whose flag bits differ, and windows flagged on one side only (the flag mask,
    the measure of the paper's Section 4.3 comparison)."""
    return {"bits": float(np.mean(a != b)), "mask": float(np.mean((a != 0) != (b != 0)))}


# ----------------------------------------------------------------------------- GPU

SETTLE_MS = 250.0                   # GPU time of a form's launches before its timed launches
SECONDARY_STEPS = 40                # least timed launches of the window, long-window and 64-station forms


SETTLE_LOG: dict = {}               # extra warm-up launches per timed form


def time_form(plan, vis, outs, stream, steps, warmup, key):
    """Warm up, then time `steps` screens with HIP events on the launch stream.

    Warm-up is `warmup` launches and then, untimed as well, as many more as it takes for the
    form's launches to have run SETTLE_MS of GPU time: the first 20-30 ms of a form after a
    switch (other kernels, host work, a fresh array) run up to twice as slow while the GPU's
    clocks settle, and a form that follows the generation of a fresh array on the device
    still runs up to 4 % slow after 50 ms (profiles/screen_fp32_baseline.md, launch-to-launch
    spread).  The count of those extra launches is logged in SETTLE_LOG under ``key``."""
    import torch
    stream.wait_stream(torch.cuda.current_stream())              # inputs written on torch's stream
    w0 = torch.cuda.Event(enable_timing=True)
    w1 = torch.cuda.Event(enable_timing=True)
    w0.record(stream)
    for _ in range(warmup):
        plan.screen(vis, outs["avg"], outs["weight"], outs["flags"], None, stream=stream)
    w1.record(stream)
    torch.cuda.synchronize()
    done_ms = w0.elapsed_time(w1)
    extra = 0
    while done_ms < SETTLE_MS:
        n = max(1, int(np.ceil((SETTLE_MS - done_ms) / max(done_ms / max(warmup, 1), 0.05))))
        w0.record(stream)
        for _ in range(n):
            plan.screen(vis, outs["avg"], outs["weight"], outs["flags"], None, stream=stream)
        w1.record(stream)
        torch.cuda.synchronize()
        done_ms += w0.elapsed_time(w1)
        extra += n
    SETTLE_LOG[key] = extra
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t_begin = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_begin.record(stream)
    for a, b in ev:
        a.record(stream)
        plan.screen(vis, outs["avg"], outs["weight"], outs["flags"], None, stream=stream)
        b.record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) for a, b in ev])          # ms per screen
    total_ms = t_begin.elapsed_time(t_end)
    return per, total_ms, wall


def put_baselines(vis_dev, bl, vis_host):
    """Write host visibilities [len(bl), C, T, 4] complex64 over baselines ``bl`` of the device
    array [B, C, T, 4, 2] float32 (so that the GPU screens the oracle's exact input bytes)."""
    import torch
    a = np.ascontiguousarray(vis_host.astype(np.complex64)).view(np.float32).reshape(vis_host.shape + (2,))
    vis_dev[torch.as_tensor(bl, device=vis_dev.device)] = torch.from_numpy(a).to(vis_dev.device)


def sampled_precision(plan, vis, bl, ref):
    """One screen with statistics (outside any timed region); the sampled baselines'
    statistics and flags against the FP64 oracle's ``ref``."""
    import torch
    outs = plan.alloc_outputs(flags=True, stats=True)
    plan.screen(vis, outs["avg"], outs["weight"], outs["flags"], outs["stats"])
    torch.cuda.synchronize()
    idx = torch.as_tensor(bl, device=vis.device)
    st = outs["stats"][idx].cpu().numpy()
    fl = outs["flags"][idx].cpu().numpy()
    return {"statistic_error": stat_errors(st, ref), "flags_vs_oracle": flag_disagreement(fl, ref["flags"])}


def probe_bandwidth(vis_bytes_tensor, nbytes, stream, reps=10):
    import torch
    from paper_2412_14775_amd import rfi
    sink = torch.empty(rfi.rfi_probe_sink_floats(nbytes), dtype=torch.float32, device="cuda:0")
    for _ in range(2):
        rfi.rfi_probe_read(vis_bytes_tensor, nbytes, sink, stream)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        rfi.rfi_probe_read(vis_bytes_tensor, nbytes, sink, stream)
    b.record(stream)
    torch.cuda.synchronize()
    return nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9


COPY_CALIBRATION_BYTES = 1 << 30


def copy_calibration(buf, stream, reps=3):
    """A plain copy of exactly 1 GiB (read 1 GiB, write 1 GiB): the known-traffic kernel
    against which the hardware byte counters of a profiling run are scaled."""
    import torch
    from paper_2412_14775_amd import rfi
    n = COPY_CALIBRATION_BYTES
    flat = buf.view(torch.uint8).view(-1)
    assert flat.numel() >= 2 * n
    for _ in range(reps):
        rfi.rfi_probe_copy(flat[n:2 * n], flat[:n], n, stream)
    torch.cuda.synchronize()


def stored_traffic(digest: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    this exact kernel source; None otherwise."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_digest") != digest:
        return None
    return t.get("cf32_bytes_per_launch")


def tf_window_form(steps: int, warmup: int, refs=None):
    """The paper's own window shape, 10 time samples x 2 channels (W = 20), on a 48-station,
    64-channel integration of 3000 samples (T divisible by 10), complex64 and complex half, and
    the paper's mixed precision (Tables 3-4); then M = 100 on the same array (complex64 and
    complex half), a length with no exact lane layout, and 300 x 2, a window wider than 64 lanes.  With ``refs`` (precision_references) the
    sampled baselines carry the oracle's input bytes, and each form's statistics and flags
    are compared with the FP64 oracle's after its timing."""
    import torch
    from paper_2412_14775_amd import rfi
    dev = torch.device("cuda:0")
    sc = synth.scene_fp32_baseline(SEED, N_STATIONS, N_CHANNELS, 3000)
    e = synth.device_voltages(sc, dev)
    B, C, T = sc.n_baselines, sc.n_channels, sc.n_samples
    vis32 = torch.empty((B, C, T, 4, 2), dtype=torch.float32, device=dev)
    synth.correlate_torch(e, vis32, "cf32")
    del e
    if refs is not None:
        put_baselines(vis32, refs["bl"], refs["vis3000"])
    torch.cuda.synchronize()
    stream = torch.cuda.Stream(device=dev)
    res = {"window": "10 x 2", "samples": T}
    flags = {}
    prec = {}
    for name, fmt, sb, opt in (("cf32", rfi.RFI_VIS_CF32, 32, 0), ("cf16", rfi.RFI_VIS_CF16, 16, 0),
                               ("cf32_paper_mixed", rfi.RFI_VIS_CF32, 32, rfi.RFI_OPT_PAPER_MIXED)):
        vis = vis32 if fmt == rfi.RFI_VIS_CF32 else vis32.to(torch.float16)
        params = rfi.rfi_params_default(n_stations=N_STATIONS, n_baselines=B, n_channels=C,
                                        n_samples=T, block_m=10, block_f=2, vis_format=fmt, options=opt,
                                        **TF_PLAN)
        plan = rfi.Plan(params)
        outs = plan.alloc_outputs(flags=True, stats=False)
        with torch.cuda.stream(stream):
            per, total_ms, _ = time_form(plan, vis, outs, stream, steps, warmup, f"tf_window.{name}")
        if refs is not None:
            prec[name] = sampled_precision(plan, vis, refs["bl"], refs["ref10"])
        plan.close()
        flags[name] = outs["flags"].clone()
        alg = B * C * (T * sb + 36) + B * (C // 2) * (T // 10)
        res[name] = {"samples_per_s": B * C * T * steps / (total_ms * 1e-3),
                     "kernel_ms_mean": float(per.mean()),
                     "achieved_GBs": alg / (per.mean() * 1e-3) / 1e9,
                     "hbm_frac": alg / (per.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del vis
    f32 = flags["cf32"].cpu().numpy()
    res["paper_mixed_flag_disagreement_vs_cf32"] = flag_disagreement(flags["cf32_paper_mixed"].cpu().numpy(), f32)
    res["cf16_flag_disagreement_vs_cf32"] = flag_disagreement(flags["cf16"].cpu().numpy(), f32)
    if refs is not None:
        res["vs_fp64_oracle"] = prec
    # a window length with no exact lane layout on the same array: M = 100 time samples (complex
    # half: 15 runs of 7 samples on 16 lanes, the last run zero-padded; complex64: 25 runs of 4
    # on 32 lanes); and a time x frequency window wider than 64 lanes of runs of 8, 300 x 2 (a
    # window over 2 steps of one channel's 300 samples each: complex half 5 per lane on 60 lanes,
    # complex64 2 chunks of 192)
    for key, M, F, th in (("window_100", 100, 1, dict(sk_d=2.2, sk_low=0.55, sk_high=1.55, ds_gamma=0.16)),
                          ("window_300x2", 300, 2, dict(sk_d=2.2, sk_low=0.8, sk_high=1.25, ds_gamma=0.07))):
        res[key] = {}
        for name, fmt, sb in (("cf32", rfi.RFI_VIS_CF32, 32), ("cf16", rfi.RFI_VIS_CF16, 16)):
            vis = vis32 if fmt == rfi.RFI_VIS_CF32 else vis32.to(torch.float16)
            params = rfi.rfi_params_default(n_stations=N_STATIONS, n_baselines=B, n_channels=C, n_samples=T,
                                            block_m=M, block_f=F, vis_format=fmt, **th)
            plan = rfi.Plan(params)
            outs = plan.alloc_outputs(flags=True, stats=False)
            with torch.cuda.stream(stream):
                per, total_ms, _ = time_form(plan, vis, outs, stream, steps, warmup, f"{key}.{name}")
            plan.close()
            alg = algorithmic_bytes(B * C, T, M, sb, F)
            res[key][name] = {"samples_per_s": B * C * T * steps / (total_ms * 1e-3),
                              "kernel_ms_mean": float(per.mean()),
                              "achieved_GBs": alg / (per.mean() * 1e-3) / 1e9,
                              "hbm_frac": alg / (per.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS}
            del vis
    del vis32
    torch.cuda.empty_cache()
    return res


def long_window_form(steps: int, warmup: int):
    """One window per integration (M = T = 3072, not a power of two times a small factor):
    the long-window kernel on the 48-station, 64-channel array, complex64 and complex half."""
    import torch
    from paper_2412_14775_amd import rfi
    dev = torch.device("cuda:0")
    sc = synth.scene_fp32_baseline(SEED, N_STATIONS, N_CHANNELS, N_SAMPLES)
    e = synth.device_voltages(sc, dev)
    B, C, T = sc.n_baselines, sc.n_channels, sc.n_samples
    vis32 = torch.empty((B, C, T, 4, 2), dtype=torch.float32, device=dev)
    synth.correlate_torch(e, vis32, "cf32")
    del e
    stream = torch.cuda.Stream(device=dev)
    res = {"window": f"{T} x 1", "samples": T}
    for name, fmt, sb in (("cf32", rfi.RFI_VIS_CF32, 32), ("cf16", rfi.RFI_VIS_CF16, 16)):
        vis = vis32 if fmt == rfi.RFI_VIS_CF32 else vis32.to(torch.float16)
        params = rfi.rfi_params_default(n_stations=N_STATIONS, n_baselines=B, n_channels=C, n_samples=T,
                                        block_m=T, vis_format=fmt, sk_d=2.2, sk_low=0.9, sk_high=1.1,
                                        ds_gamma=0.03)
        plan = rfi.Plan(params)
        outs = plan.alloc_outputs(flags=True, stats=False)
        with torch.cuda.stream(stream):
            per, total_ms, _ = time_form(plan, vis, outs, stream, steps, warmup, f"long_window.{name}")
        plan.close()
        alg = algorithmic_bytes(B * C, T, T, sb)
        res[name] = {"samples_per_s": B * C * T * steps / (total_ms * 1e-3),
                     "kernel_ms_mean": float(per.mean()),
                     "achieved_GBs": alg / (per.mean() * 1e-3) / 1e9,
                     "hbm_frac": alg / (per.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del vis
    del vis32
    torch.cuda.empty_cache()
    return res


def mixed_case_form(steps: int, warmup: int):
    """Larger mixed-RFI case: 64 stations (2080 baselines), 256 channels, 3072 samples, complex
    half (26.2 GB per integration), M = 16, 64, 256."""
    import torch
    from paper_2412_14775_amd import rfi
    dev = torch.device("cuda:0")
    sc = synth.scene_mixed(3)
    e = synth.device_voltages(sc, dev)
    B, C, T = sc.n_baselines, sc.n_channels, sc.n_samples
    vis = torch.empty((B, C, T, 4, 2), dtype=torch.float16, device=dev)
    synth.correlate_torch(e, vis, "cf16")
    del e
    stream = torch.cuda.Stream(device=dev)
    res = {"stations": sc.n_stations, "channels": C, "samples": T, "GB": B * C * T * 16 / 1e9}
    for M in (16, 64, 256):
        params = rfi.rfi_params_default(n_stations=sc.n_stations, n_baselines=B, n_channels=C, n_samples=T,
                                        block_m=M, vis_format=rfi.RFI_VIS_CF16, sk_d=2.2, sk_low=0.5,
                                        sk_high=1.6, ds_gamma=float(np.sqrt(7.815 / (3 * M))))
        plan = rfi.Plan(params)
        outs = plan.alloc_outputs(flags=True, stats=False)
        with torch.cuda.stream(stream):
            per, total_ms, _ = time_form(plan, vis, outs, stream, steps, warmup, f"mixed_case_cf16.M{M}")
        plan.close()
        alg = algorithmic_bytes(B * C, T, M, 16)
        res[f"M{M}"] = {"samples_per_s": B * C * T * steps / (total_ms * 1e-3), "kernel_ms_mean": float(per.mean()),
                        "achieved_GBs": alg / (per.mean() * 1e-3) / 1e9,
                        "hbm_frac": alg / (per.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS}
    del vis
    torch.cuda.empty_cache()
    return res


def serving(seconds: float, rate: float):
    """Serving form: 16 arrays (12-64 stations, 16-256 channels, M = 64, complex half,
    adaptive thresholds), inputs pre-staged in HBM; Poisson arrivals at `rate` per second in
    total for `seconds`, then the same requests all at once (saturated)."""
    import torch
    from paper_2412_14775_amd import rfi
    scenes = synth.serving_mix()
    dev = torch.device("cuda:0")
    arrays = []
    for sc in scenes:
        e = synth.device_voltages(sc, dev)
        vis = torch.empty((sc.n_baselines, sc.n_channels, sc.n_samples, 4, 2), dtype=torch.float16, device=dev)
        synth.correlate_torch(e, vis, "cf16")
        del e
        params = rfi.rfi_params_default(n_stations=sc.n_stations, n_baselines=sc.n_baselines,
                                        n_channels=sc.n_channels, n_samples=sc.n_samples, block_m=64,
                                        vis_format=rfi.RFI_VIS_CF16, options=rfi.RFI_OPT_ADAPTIVE,
                                        n_warm=64, **PLAN)
        plan = rfi.Plan(params)
        arrays.append((sc, plan, vis, plan.alloc_outputs(flags=True, stats=False)))
    torch.cuda.synchronize()
    samples = [sc.n_baselines * sc.n_channels * sc.n_samples for sc, *_ in arrays]
    nbytes = [s * 16 for s in samples]
    srv = rfi.Server(n_slots=16, hbm_budget=200 << 30)
    tag = 0
    for i, (sc, plan, vis, out) in enumerate(arrays):                 # capture every graph once
        srv.submit(plan, vis, out, tag=tag)
        tag += 1
    srv.drain(120)
    srv.poll(10000)

    def run(arrivals):
        nonlocal tag
        first = tag
        for t, i in arrivals:
            sc, plan, vis, out = arrays[i]
            srv.submit(plan, vis, out, arrival=t, tag=tag)
            tag += 1
        srv.drain(600)
        done = [c for c in srv.poll(100000) if c["tag"] >= first]
        assert len(done) == len(arrivals) and all(c["status"] == 0 for c in done)
        lat = np.array([c["done"] - c["arrival"] for c in done])
        span = max(c["done"] for c in done) - min(c["arrival"] for c in done)
        idx = [arrivals[c["tag"] - first][1] for c in done]
        return lat, span, sum(samples[i] for i in idx), sum(nbytes[i] for i in idx)

    rng = np.random.default_rng(11)
    t, arr = srv.now() + 0.05, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > srv.now() + 0.05 + seconds:
            break
        arr.append((t, int(rng.integers(0, len(arrays)))))
    lat, span, n_s, n_b = run(arr)
    t0 = srv.now()
    sat = [(t0, i) for i in range(len(arrays)) for _ in range(4)]
    lat_s, span_s, n_s2, n_b2 = run(sat)
    st = srv.stats()
    srv.close()
    for _, plan, *_ in arrays:
        plan.close()
    return {
        "arrays": [[sc.n_stations, sc.n_channels] for sc, *_ in arrays],
        "pool_GB": sum(nbytes) / 1e9,
        "requests": len(arr), "rate_per_s": rate, "deadline_ms": 1000.0,
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "max_ms": float(lat.max() * 1e3), "deadline_misses": int((lat > 1.0).sum()),
        "offered_samples_per_s": n_s / span,
        "saturated": {"requests": len(sat), "makespan_ms": span_s * 1e3,
                      "samples_per_s": n_s2 / span_s, "GBs": n_b2 / span_s / 1e9,
                      "p99_ms": float(np.percentile(lat_s, 99) * 1e3)},
        "peak_inflight": st["peak_inflight"], "graphs": st["graphs"],
    }


def parse_shape(spec: str):
    """'fmt:M[xF][m][@T]' -> (fmt, M, F, mixed, T): storage format cf32 or cf16, window of M time
    samples x F channels, 'm' for the paper's mixed precision, T samples per stream (default 3072
    when M divides it, else 3000)."""
    fmt, rest = spec.split(":")
    T = None
    if "@" in rest:
        rest, t = rest.split("@")
        T = int(t)
    mixed = rest.endswith("m")
    rest = rest.rstrip("m")
    M, F = (int(x) for x in rest.split("x")) if "x" in rest else (int(rest), 1)
    if T is None:
        T = N_SAMPLES if N_SAMPLES % M == 0 else 3000
    if fmt not in ("cf32", "cf16") or T % M or N_CHANNELS % F:
        raise ValueError(f"bad shape {spec!r}")
    return fmt, M, F, mixed, T


def time_shapes(specs, steps: int, warmup: int) -> list:
    """Each listed window shape on the 48-station, 64-channel array (synthetic, as the FP32
    baseline), one screen with flags per launch: `warmup` launches plus the settling launches,
    then `steps` timed with HIP events on the launch stream.  For profiling single kernels
    (rocprofv3 runs over this mode launch nothing else of the screen)."""
    import torch
    from paper_2412_14775_amd import rfi
    dev = torch.device("cuda:0")
    arrays, out = {}, []
    stream = torch.cuda.Stream(device=dev)
    for spec in specs:
        fmt, M, F, mixed, T = parse_shape(spec)
        if (T, "cf32") not in arrays:
            sc = synth.scene_fp32_baseline(SEED, N_STATIONS, N_CHANNELS, T)
            e = synth.device_voltages(sc, dev)
            v = torch.empty((sc.n_baselines, N_CHANNELS, T, 4, 2), dtype=torch.float32, device=dev)
            synth.correlate_torch(e, v, "cf32")
            del e
            arrays[(T, "cf32")] = v
        if (T, fmt) not in arrays:
            arrays[(T, fmt)] = arrays[(T, "cf32")].to(torch.float16)
        vis = arrays[(T, fmt)]
        B = vis.shape[0]
        params = rfi.rfi_params_default(
            n_stations=N_STATIONS, n_baselines=B, n_channels=N_CHANNELS, n_samples=T, block_m=M, block_f=F,
            vis_format=rfi.RFI_VIS_CF16 if fmt == "cf16" else rfi.RFI_VIS_CF32,
            options=rfi.RFI_OPT_PAPER_MIXED if mixed else 0, sk_d=2.2, sk_low=0.5, sk_high=1.6,
            ds_gamma=float(min(0.95, np.sqrt(7.815 / (3 * M * F)))))
        plan = rfi.Plan(params)
        outs = plan.alloc_outputs(flags=True, stats=False)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            per, total_ms, _ = time_form(plan, vis, outs, stream, steps, warmup, spec)
        plan.close()
        sb = 16 if fmt == "cf16" else 32
        alg = B * N_CHANNELS * (T * sb + 36) + B * (N_CHANNELS // F) * (T // M)
        r = {"shape": spec, "samples": T, "kernel_ms_mean": float(per.mean()), "kernel_ms_p50": float(np.median(per)),
             "achieved_GBs": alg / (per.mean() * 1e-3) / 1e9, "hbm_frac": alg / (per.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS}
        out.append(r)
        progress(f"{spec}: {r['kernel_ms_mean'] * 1e3:.1f} us per launch, {r['hbm_frac']:.3f} of the HBM peak")
    return out


def progress(msg: str) -> None:
    """One line per stage on stderr (stdout carries only the JSON result line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-seconds", type=float, default=6.0,
                    help="length of the real-time serving run (0 skips the serving form)")
    ap.add_argument("--shapes", nargs="+", metavar="FMT:M[xF][m][@T]",
                    help="time only these window shapes (e.g. cf16:64 cf16:10x2 cf32:10x2m) on the "
                         "48-station array instead of the benchmark; prints one JSON line of results")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: only --gpus 1 is supported (got {args.gpus}); the screen shards by "
              "baseline with no exchange, and bench.py measures one GPU's share.", file=sys.stderr)
        return 2
    if args.shapes:
        from paper_2412_14775_amd import rfi
        rfi.load_library()
        res = time_shapes(args.shapes, args.steps, args.warmup)
        print(json.dumps({"shapes": res, "steps": args.steps, "warmup": args.warmup,
                          "settle": SETTLE_LOG, "kernel_source_digest": kernel_source_digest()}), flush=True)
        return 0

    scene = synth.scene_fp32_baseline(SEED, N_STATIONS, N_CHANNELS, N_SAMPLES)
    e = synth.make_voltages(scene)                                # [N, C, T, 2] complex64
    cpu = refs = None
    if not args.no_cpu_baseline:                                  # host work, before any GPU use
        cpu = cpu_baseline(e)
        progress(f"cpu baseline: {cpu['value']:.3g} samples/s ({cpu['sample']})")
        e3000 = synth.make_voltages(synth.scene_fp32_baseline(SEED, N_STATIONS, N_CHANNELS, 3000))
        refs = precision_references(e, e3000)
        del e3000
        progress(f"oracle references of {len(refs['bl'])} sampled baselines done")

    import torch
    from paper_2412_14775_amd import rfi
    rfi.load_library()
    B, C, T, M = synth.n_baselines(N_STATIONS), N_CHANNELS, N_SAMPLES, BLOCK_M
    n_streams = B * C
    samples = n_streams * T
    dev = torch.device("cuda:0")
    e_dev = torch.from_numpy(e).to(dev)
    vis32 = torch.empty((B, C, T, 4, 2), dtype=torch.float32, device=dev)
    synth.correlate_torch(e_dev, vis32, "cf32")
    del e_dev
    if refs is not None:
        put_baselines(vis32, refs["bl"], refs["vis"])
    vis16 = vis32.to(torch.float16)
    torch.cuda.synchronize()

    stream = torch.cuda.Stream(device=dev)                       # default priority
    forms, all_flags, prec = {}, {}, {}
    for name, vis, fmt, sb in (("cf32", vis32, rfi.RFI_VIS_CF32, 32), ("cf16", vis16, rfi.RFI_VIS_CF16, 16)):
        params = rfi.rfi_params_default(n_stations=N_STATIONS, n_baselines=B, n_channels=C,
                                        n_samples=T, block_m=M, vis_format=fmt, **PLAN)
        plan = rfi.Plan(params)
        outs = plan.alloc_outputs(flags=True, stats=False)
        with torch.cuda.stream(stream):
            per, total_ms, wall = time_form(plan, vis, outs, stream, args.steps, args.warmup, name)
        flagged = float((outs["flags"] != 0).float().mean().item())
        all_flags[name] = outs["flags"].cpu().numpy()
        if refs is not None:
            prec[name] = sampled_precision(plan, vis, refs["bl"], refs["ref32"])
            if name == "cf16":
                prec["cf16_on_fp16_bytes"] = sampled_precision(plan, vis, refs["bl"], refs["ref16"])
        plan.close()
        alg = algorithmic_bytes(n_streams, T, M, sb)
        avg_s = per.mean() * 1e-3
        forms[name] = {
            "samples_per_s": samples * args.steps / (total_ms * 1e-3),
            "ms_per_step": total_ms / args.steps,
            "kernel_ms_mean": float(per.mean()),
            "p50_ms": float(np.percentile(per, 50)),
            "p99_ms": float(np.percentile(per, 99)),
            "achieved_GBs": alg / avg_s / 1e9,
            "hbm_frac": alg / avg_s / 1e9 / HBM_PEAK_GBS,
            "bytes_per_launch": alg,
            "flagged_frac": flagged,
            "host_wall_s": wall,
        }
        progress(f"{name}: {forms[name]['samples_per_s']:.4g} samples/s, {forms[name]['achieved_GBs']:.0f} GB/s")
    probe = probe_bandwidth(vis32, vis32.numel() * 4, stream)
    copy_calibration(vis32, stream)
    del vis32, vis16
    torch.cuda.empty_cache()
    progress(f"read probe: {probe:.0f} GB/s")
    tf = tf_window_form(max(SECONDARY_STEPS, args.steps), max(2, args.warmup // 4), refs)
    progress("10 x 2 windows done")
    long_w = long_window_form(max(SECONDARY_STEPS, args.steps), max(2, args.warmup // 4))
    progress("one-window-per-integration form done")
    mixed = mixed_case_form(max(SECONDARY_STEPS, args.steps), max(2, args.warmup // 4))
    progress("64-station mixed case done")
    serve = serving(args.serving_seconds, 16.0) if args.serving_seconds > 0 else None
    if serve is not None:
        progress(f"serving: p99 {serve['p99_ms']:.2f} ms")

    f32 = forms["cf32"]
    digest = kernel_source_digest()
    traffic = stored_traffic(digest)
    line = {
        "metric": "visibility samples/s screened (FP16 vs FP32, % HBM peak); p99 latency/integ",
        "value": f32["samples_per_s"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle": {"min_ms_of_launches_before_timing": SETTLE_MS,
                   "timed_launches_other_forms": max(SECONDARY_STEPS, args.steps),
                   "extra_warmup_launches": SETTLE_LOG},
        "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fp32 baseline: 48 stations (1176 baselines incl. autos), 64 channels, "
                               "3072 samples per 1 s integration, M=64, complex64 (7.40 GB)",
                   "stations": N_STATIONS, "baselines": B, "channels": C, "samples": T,
                   "block_m": M, "vis_format": "cf32", "seed": SEED},
        "roofline": {"bound": "hbm", "achieved": f32["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": f32["hbm_frac"], "traffic": traffic,
                     "kernel": "screen_tiled<0, 6, persistent> (complex64, M=64)",
                     "bytes_per_launch": f32["bytes_per_launch"]},
        "cpu_baseline": cpu,
        "latency_ms": {"p50": f32["p50_ms"], "p99": f32["p99_ms"], "deadline": 1000.0},
        "cf16": {k: forms["cf16"][k] for k in ("samples_per_s", "ms_per_step", "p50_ms", "p99_ms",
                                               "achieved_GBs", "hbm_frac")},
        "cf16_over_cf32": forms["cf16"]["samples_per_s"] / f32["samples_per_s"],
        "read_probe_GBs": probe,
        "tf_window": tf,
        "long_window": long_w,
        "mixed_case_cf16": mixed,
        "serving": serve,
        "precision": None if refs is None else {
            "sample": f"{len(refs['bl'])} seeded baselines (one autocorrelation) x 64 channels of the "
                      "FP32-baseline workload and of the 10 x 2 workload; the GPU screens the oracle's "
                      "exact input bytes",
            "statistic_error": "|gpu - oracle| / max(1, |oracle|) over windows (tolerance 1e-5 "
                               "complex64, 3e-3 complex half against the complex64 input)",
            "cf32_vs_fp64": prec["cf32"],
            "cf16_vs_fp64_on_complex64_input": prec["cf16"],
            "cf16_vs_fp64_on_fp16_bytes": prec["cf16_on_fp16_bytes"],
            "cf16_vs_cf32_all_streams": flag_disagreement(all_flags["cf16"], all_flags["cf32"]),
            "tf_window_10x2_vs_fp64": tf.get("vs_fp64_oracle"),
        },
        "flagged_frac": f32["flagged_frac"],
        "kernel_source_digest": digest,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
