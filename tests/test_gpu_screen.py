"""GPU parity of librfi's screen against the FP64 oracle (needs an MI355X)."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.cases import cf16_total_tolerance, scene_vis, thresholds_for
from tests.gpu_helpers import TOL_F32, compare, flags_from_stats32, make_params, run_gpu, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2412_14775_amd import rfi
    rfi.load_library()
    yield


def screen_both(vis, M, fmt="cf32", stats=True, **kw):
    from paper_2412_14775_amd import rfi
    B, C, T, _ = vis.shape
    op, rp = make_params(B, C, T, M, fmt, **kw)
    plan = rfi.Plan(rp)
    try:
        dev = to_device(vis if fmt == "cf32" else synth.to_cf16(vis), fmt)
        gpu = run_gpu(plan, dev, stats=stats)
    finally:
        plan.close()
    return op, gpu


def check_cf16(vis, M, label, **kw):
    """Complex-half storage: arithmetic error against the oracle on the same FP16 bytes
    (1e-5, every M) and total error against the oracle on the original complex64 input
    (3e-3 wherever the storage rounding alone stays within it; at W = 2 it does not, and the
    bound is what the oracle itself shows between the two inputs plus 1e-5:
    tests/test_cf16_storage_cpu.py)."""
    op, gpu = screen_both(vis, M, "cf16", **kw)
    rep_a = compare(gpu, synth.to_cf16(vis), op, TOL_F32, label=label + " (fp16 input)")
    rep_t = compare(gpu, vis, op, cf16_total_tolerance(vis, op), label=label + " (original input)")
    print(f"{label}: arithmetic error " + ", ".join(f"{k} {rep_a['max_err_' + k]:.2e}" for k in ("tau", "r_re", "r_im"))
          + "; total error " + ", ".join(f"{k} {rep_t['max_err_' + k]:.2e}" for k in ("tau", "r_re", "r_im")))
    return rep_a, rep_t


# ----------------------------------------------------------------------------- the plain case

def test_plain_case_cf32():
    vis = synth.correlate(synth.make_voltages(synth.scene_plain(0)))
    op, gpu = screen_both(vis, 16, **thresholds_for(16))
    rep = compare(gpu, vis, op, TOL_F32, label="plain cf32")
    print("plain cf32", rep)
    assert 0.05 < rep["flagged_frac"] < 0.6


def test_plain_case_against_stored_oracle_outputs():
    """GPU results against the committed oracle outputs (tests/golden/plain_case_oracle.npz)."""
    from tests.golden.make_golden import OUT, PARAMS
    g = np.load(OUT)
    vis = synth.correlate(synth.make_voltages(synth.scene_plain(0)))
    kw = {k: v for k, v in PARAMS.items() if k != "M"}
    op, gpu = screen_both(vis, PARAMS["M"], **kw)
    ref = {k: g[k] for k in ("tau", "r_re", "r_im", "flags", "avg", "weight")}
    compare(gpu, vis, op, TOL_F32, ref=ref, label="stored plain case")


def test_plain_case_cf16():
    vis = synth.correlate(synth.make_voltages(synth.scene_plain(0)))
    rep_a, rep_t = check_cf16(vis, 16, "plain cf16", **thresholds_for(16))
    print("plain cf16", rep_a, rep_t)


# ----------------------------------------------------------------------------- window lengths

@pytest.mark.parametrize("fmt", ["cf32", "cf16"])
@pytest.mark.parametrize("M", [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048])
def test_power_of_two_windows(fmt, M):
    T = M * max(3, 1600 // M)         # several steps per stream and a ragged last step
    vis = scene_vis(2, 5, T, seed=M)
    if fmt == "cf32":
        op, gpu = screen_both(vis, M, **thresholds_for(M))
        compare(gpu, vis, op, TOL_F32, label=f"cf32 M={M}")
    else:
        check_cf16(vis, M, f"cf16 M={M}", **thresholds_for(M))


@pytest.mark.parametrize("fmt", ["cf32", "cf16"])
@pytest.mark.parametrize("M,T", [(3, 300), (10, 400), (20, 3060), (48, 960), (100, 500)])
def test_other_window_lengths(fmt, M, T):
    vis = scene_vis(2, 3, T, seed=M + 7, duty=(60, 20))
    if fmt == "cf32":
        op, gpu = screen_both(vis, M, **thresholds_for(M))
        compare(gpu, vis, op, TOL_F32, label=f"cf32 M={M}")
    else:
        check_cf16(vis, M, f"cf16 M={M}", **thresholds_for(M))


@pytest.mark.parametrize("fmt", ["cf32", "cf16"])
@pytest.mark.parametrize("M,T", [(16, 4096), (64, 1088), (64, 3072), (256, 3072)])
def test_few_long_streams_split_over_waves(fmt, M, T):
    """A handful of streams: each is split over several waves whose partial sums are combined."""
    vis = scene_vis(1, 3, T, seed=T + M)
    if fmt == "cf32":
        op, gpu = screen_both(vis, M, **thresholds_for(M))
        compare(gpu, vis, op, TOL_F32, label=f"segmented cf32 M={M} T={T}")
    else:
        check_cf16(vis, M, f"segmented cf16 M={M} T={T}", **thresholds_for(M))


@pytest.mark.parametrize("fmt,M,F,T,adaptive,mixed", [
    ("cf32", 16, 1, 256, False, False), ("cf32", 64, 1, 256, False, False), ("cf32", 16, 1, 256, True, False),
    ("cf16", 16, 1, 256, False, False), ("cf16", 64, 1, 256, True, False),
    ("cf16", 10, 2, 300, False, False), ("cf32", 10, 2, 300, False, False), ("cf16", 10, 2, 300, True, False),
    ("cf32", 10, 2, 300, False, True), ("cf16", 100, 1, 300, False, False), ("cf32", 100, 1, 300, False, False),
    ("cf16", 5, 4, 300, False, False), ("cf16", 10, 2, 3000, False, False), ("cf16", 5, 4, 3000, True, False)])
def test_persistent_and_per_wave_launches_agree(fmt, M, F, T, adaptive, mixed):
    """With a flag array the complex64 tiled kernel and the exact windowed layouts of at most 6
    samples per lane (both formats, the mixed form included) run persistent launches (a block
    screens a range of streams or channel groups, its waves splitting the windowed groups' steps
    evenly, and holds their flags in LDS until it is done); without a flag array the same plan runs
    one wave per stream or group.  Complex half does so only where a group has at least 16 steps
    (10 x 2 and 5 x 4 on 3000 samples: 19 and 38); the other cases run one wave per stream or group
    either way and stay here as a check that the flag array changes nothing else.  48 stations x
    32 channels (37 632 streams: no segments).  Weights, statistics and window counts of the two must agree
    bit for bit, averages and the adaptive moments to float32 rounding (a group split between two
    waves adds two partial sums), and the persistent launch's flags must be the flag rule applied
    to those statistics."""
    import torch
    from paper_2412_14775_amd import rfi
    B, C = 1176, 32
    g = torch.Generator(device="cuda:0").manual_seed(M * F + T)
    vis = torch.randn((B, C, T, 4, 2), generator=g, device="cuda:0", dtype=torch.float32)
    vis[:, 3, 40:48] *= 30.0                                    # some flagged windows
    if fmt == "cf16":
        vis = vis.to(torch.float16)
    th = thresholds_for(M * F)
    op = oracle.Params(M=M, F=F, **th)
    options = (rfi.RFI_OPT_ADAPTIVE if adaptive else 0) | (rfi.RFI_OPT_PAPER_MIXED if mixed else 0)
    rp = rfi.rfi_params_default(n_stations=48, n_baselines=B, n_channels=C, n_samples=T, block_m=M, block_f=F,
                                vis_format=rfi.RFI_VIS_CF16 if fmt == "cf16" else rfi.RFI_VIS_CF32,
                                sk_d=op.d, sk_low=op.s_low, sk_high=op.s_high, ds_gamma=op.gamma, eps=op.eps,
                                options=options)
    plan = rfi.Plan(rp)
    try:
        with_flags = plan.alloc_outputs(flags=True, stats=True)
        without = plan.alloc_outputs(flags=False, stats=True)
        plan.screen(vis, with_flags["avg"], with_flags["weight"], with_flags["flags"], with_flags["stats"])
        torch.cuda.synchronize()
        state_after = plan.state().copy() if adaptive else None
        if adaptive:
            rfi.rfi_state_reset(plan.handle)
        plan.screen(vis, without["avg"], without["weight"], None, without["stats"])
        torch.cuda.synchronize()
        if adaptive:                              # counts exact; moments of a channel group split
            st = plan.state()                     # between two waves merged in another order
            assert np.array_equal(st["n"], state_after["n"]) and state_after["n"].sum() > 0
            np.testing.assert_allclose(st["mean"], state_after["mean"], rtol=1e-5, atol=1e-7)
            np.testing.assert_allclose(st["m2"], state_after["m2"], rtol=1e-5, atol=1e-7)
    finally:
        plan.close()
    for k in ("weight", "stats"):                   # bit patterns: the mixed form has NaN statistics
        assert torch.equal(with_flags[k].view(torch.int32), without[k].view(torch.int32)), k
    # averages: a channel group split between two waves of a persistent block adds its two partial
    # sums, in another association than one wave's lane tree (a few float32 roundings of sums of
    # magnitude <= the kept count x the mean magnitude)
    a0, a1 = with_flags["avg"].double(), without["avg"].double()
    assert torch.isfinite(a0).all() and float((a0 - a1).abs().max()) <= 1e-6, "avg"
    if not mixed:                                   # the mixed form compares in binary16
        p32 = op.f32()
        thb = dict(s_low=p32.s_low, s_high=p32.s_high, gamma=p32.gamma, gamma_im=p32.gamma)
        flags = with_flags["flags"].cpu().numpy()
        assert np.array_equal(flags, flags_from_stats32(with_flags["stats"].cpu().numpy(), thb, 0))
    flags = with_flags["flags"].cpu().numpy()
    assert flags.any() and not flags.all()


def test_half_sums_are_exact():
    """The complex-half kernels' sums and differences of binary16 parts (one v_fma_mix_f32
    each) equal conversion to float32 and a float32 add, bit for bit, for every binary16 value
    against 1024 others (include/rfi.h, rfi_probe_half_sums)."""
    import torch
    from paper_2412_14775_amd import rfi
    bad = torch.full((rfi.HALF_SUMS_VALUES,), -1, dtype=torch.int32, device="cuda:0")
    rfi.rfi_probe_half_sums(bad)
    torch.cuda.synchronize()
    counts = bad.cpu().numpy()
    assert counts.min() >= 0, "not every counter was written"
    assert counts.sum() == 0, f"{int(counts.sum())} differences, first at binary16 0x{int(np.argmax(counts > 0)):04x}"


@pytest.mark.parametrize("fmt", ["cf32", "cf16"])
@pytest.mark.parametrize("M,T,N", [(300, 3000, 2), (600, 3000, 2), (1000, 3000, 2), (3000, 3000, 2),
                                   (3072, 6144, 2), (768, 6144, 1), (8192, 16384, 1),
                                   (513, 5130, 1), (1023, 8184, 1), (257, 2570, 2), (511, 5110, 1),
                                   (500, 5000, 2), (450, 4050, 1), (131, 1310, 2), (193, 3860, 1),
                                   (251, 2510, 1), (127, 1270, 2), (97, 1940, 1), (67, 1340, 2)])
def test_long_windows(fmt, M, T, N):
    """Windows of more than a quarter of a step (64 complex64 / 128 complex-half samples) that
    are not powers of two up to 4096 and take more than 64 runs of 5 (complex64) or 8 (complex
    half) samples (the long-window kernel): edges fall anywhere inside a step, steps are ragged at
    the stream end, and few streams split over waves.  A window one sample longer or shorter
    than a whole number of steps (513, 1023 complex half; 511 complex64) walks the edge through
    every offset of the step; 3072 and 768 (complex64) end every window with a step.  The
    shorter lengths (67-511 complex half, 67-320 complex64, and 300 = 5 x 60) go to the windowed
    kernel with padded runs or partial lane groups instead; they stay here as cross-checks."""
    vis = scene_vis(N, 2, T, seed=M + T, duty=(500, 60))
    if fmt == "cf32":
        op, gpu = screen_both(vis, M, **thresholds_for(M))
        compare(gpu, vis, op, TOL_F32, label=f"long cf32 M={M} T={T}")
    else:
        check_cf16(vis, M, f"long cf16 M={M} T={T}", **thresholds_for(M))


@pytest.mark.parametrize("fmt", ["cf32", "cf16"])
@pytest.mark.parametrize("M,F,C,T", [(300, 2, 4, 1200), (129, 4, 4, 516), (1000, 2, 4, 3000), (600, 2, 2, 1800),
                                     (257, 2, 4, 1028), (200, 4, 4, 800), (300, 2, 2, 300), (513, 4, 4, 1026),
                                     (100, 4, 4, 1000), (81, 4, 4, 810), (256, 4, 4, 512), (129, 4, 8, 129)])
def test_wide_windows(fmt, M, F, C, T):
    """Time x frequency windows wider than 64 lanes of runs of 8 samples: a window over F R steps of
    one chunk (64 C samples) of one channel each.  Runs that fill part of one chunk (300 x 2 on 60
    of 64 lanes, complex64 129 x 4 on 33), several chunks with a partial last one (1000 x 2: 512 +
    488 in complex half; 600 x 2, 257 x 2 in complex64), one window per stream (T = M), and 513 x 4
    (chunks of 320 + 193 complex-half samples, 3 chunks of 192, the last 129, complex64).  Four
    channels whose runs fit 32 lanes take two runs per step: complex half 129 x 4 (runs of 5 on
    26 + 26 lanes), 200 x 4 (7 on 29 + 29), 256 x 4 (8 on 32 + 32), complex64 100 x 4 (4 on 25 + 25)
    and 81 x 4 (3 on 27 + 27; complex half 81 x 4 is a windowed layout)."""
    vis = scene_vis(2, C, T, seed=M * 3 + F, duty=(120, 25))
    if fmt == "cf32":
        op, gpu = screen_both(vis, M, F=F, **thresholds_for(M * F))
        compare(gpu, vis, op, TOL_F32, label=f"wide cf32 {M}x{F}")
    else:
        check_cf16(vis, M, f"wide cf16 {M}x{F}", F=F, **thresholds_for(M * F))


@pytest.mark.parametrize("fmt", ["cf32", "cf16"])
@pytest.mark.parametrize("M,F,C,T", [(100, 1, 2, 1000), (300, 1, 2, 3000), (50, 1, 2, 1000), (15, 2, 4, 600),
                                     (9, 2, 4, 450), (25, 4, 8, 500), (100, 2, 4, 1000),
                                     (100, 1, 2, 1300), (50, 1, 2, 1350), (61, 1, 3, 1281), (67, 1, 2, 1005),
                                     (97, 1, 2, 679), (113, 1, 2, 1017), (127, 1, 2, 1143), (131, 1, 2, 655),
                                     (193, 1, 2, 965), (251, 1, 2, 753), (257, 1, 2, 771), (500, 1, 2, 1500),
                                     (100, 2, 4, 1300), (33, 2, 4, 990)])
def test_windows_on_partial_lane_groups(fmt, M, F, C, T):
    """Windows cut into runs of C samples per lane that do not fill whole power-of-two lane
    groups: the last run of each channel padded with zeros (M = 100 as 15 runs of 7 on 16 lanes
    in complex half, 61 as 8 runs of 8, 500 as 63 runs of 8 on 64, ...) or the left-over lanes of
    a group idle (complex64 M = 100 = 4 x 25 on 32 lanes, 300 = 5 x 60 on 64).  Left-over lanes
    must neither read nor add, padding must add nothing, and the channel sums are masked wave
    sums; the second half of the cases ends on a ragged step (fewer windows than a step holds)."""
    vis = scene_vis(2, C, T, seed=M * 10 + F + T, duty=(120, 25))
    if fmt == "cf32":
        op, gpu = screen_both(vis, M, F=F, **thresholds_for(M * F))
        compare(gpu, vis, op, TOL_F32, label=f"partial groups cf32 {M}x{F} T={T}")
    else:
        check_cf16(vis, M, f"partial groups cf16 {M}x{F} T={T}", F=F, **thresholds_for(M * F))


# ----------------------------------------------------------------------------- time x frequency windows

@pytest.mark.parametrize("fmt", ["cf32", "cf16"])
@pytest.mark.parametrize("M,F,C,T", [(10, 2, 8, 400), (5, 4, 8, 300), (16, 2, 6, 512), (20, 1, 4, 400),
                                     (64, 4, 8, 3072), (10, 2, 8, 3000), (5, 4, 8, 3000)])
def test_time_frequency_windows(fmt, M, F, C, T):
    """Windows of M time samples x F adjacent channels (the paper's 10 x 2 and 5 x 4 shapes).  On
    3000 samples a channel group has 19 (10 x 2) or 38 (5 x 4) steps and the array only 24 or 12
    groups, so the persistent launch (complex half too, at 16 or more steps) gives each block one
    group whose steps its four waves split: four partial records merged per group."""
    vis = scene_vis(3, C, T, seed=31 + M * F, rfi_channels=(1, 2), duty=(50, 12))
    th = thresholds_for(M * F)
    if fmt == "cf32":
        op, gpu = screen_both(vis, M, F=F, **th)
        rep = compare(gpu, vis, op, TOL_F32, label=f"cf32 {M}x{F}")
    else:
        rep, _ = check_cf16(vis, M, f"cf16 {M}x{F}", F=F, **th)
    assert gpu_flag_shape_ok(vis, M, F)
    print(f"{fmt} {M}x{F}", rep)


def gpu_flag_shape_ok(vis, M, F):
    B, C, T, _ = vis.shape
    return C % F == 0 and T % M == 0


# ----------------------------------------------------------------------------- edge cases

@pytest.mark.parametrize("fmt", ["cf32", "cf16"])
def test_degenerate_inputs(fmt):
    M, T = 16, 256
    vis = scene_vis(2, 4, T, seed=3).astype(np.complex64)
    vis[0, 0] = 0                                  # all-zero stream: every window SK_LOW
    vis[1, 1, 20, 2] = np.nan                      # NaN sample: its window flagged
    vis[2, 2, 100, 0] = np.inf                     # Inf sample
    vis[2, 3, 33:48] = 0                           # a partly zero window
    op, gpu = screen_both(vis, M, fmt, **thresholds_for(M))
    ref_vis = vis if fmt == "cf32" else synth.to_cf16(vis)
    compare(gpu, ref_vis, op, TOL_F32, label=f"degenerate {fmt}")
    assert np.all(gpu["flags"][0, 0] == oracle.SK_LOW)
    assert gpu["weight"][0, 0] == 0.0 and np.all(gpu["avg"][0, 0] == 0)
    assert gpu["flags"][1, 1, 1] != 0 and np.isfinite(gpu["avg"]).all()


def test_single_window_and_single_station():
    vis = scene_vis(1, 2, 64, seed=9)              # N = 1: one autocorrelation stream per channel
    op, gpu = screen_both(vis, 64, **thresholds_for(64))
    compare(gpu, vis, op, TOL_F32, label="T = M")
    assert np.all(gpu["r_im"] == 0.0)              # autos are Hermitian


@pytest.mark.parametrize("options", [oracle.OPT_NO_SK, oracle.OPT_NO_DS, oracle.OPT_NO_SK | oracle.OPT_NO_DS])
def test_options_disable_tests(options):
    vis = scene_vis(2, 4, 512, seed=4, inr=15.0)
    op, gpu = screen_both(vis, 16, options=options, **thresholds_for(16))
    compare(gpu, vis, op, TOL_F32, label=f"options {options}")
    if options & oracle.OPT_NO_SK:
        assert not np.any(gpu["flags"] & 3)
    if options & oracle.OPT_NO_DS:
        assert not np.any(gpu["flags"] & 12)


@pytest.mark.parametrize("fmt", ["cf32", "cf16"])
def test_dynamic_range_fuzz(fmt):
    """Circular-Gaussian correlations scaled by 10^U(-2, 3) per window, with random
    rank-one RFI blocks mixed by a random 2x2 complex matrix (the precision-search
    data distribution of Section 4.1)."""
    rng = np.random.default_rng(77)
    B, C, T, M = 6, 4, 640, 16
    z = (rng.standard_normal((B, C, T, 4)) + 1j * rng.standard_normal((B, C, T, 4))) / math.sqrt(2)
    scale = 10.0 ** rng.uniform(-2, 3, (B, C, T // M, 1, 1))
    vis = (z.reshape(B, C, T // M, M, 4) * scale)
    hit = rng.random((B, C, T // M)) < 0.4
    J = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / math.sqrt(2)
    rfi_block = (J @ J.conj().T).reshape(4) * (10.0 ** rng.uniform(-2, 3, (B, C, T // M, 1, 1)))
    vis = vis + hit[..., None, None] * rfi_block
    vis = vis.reshape(B, C, T, 4).astype(np.complex64)
    op, gpu = screen_both(vis, M, fmt, **thresholds_for(M))
    compare(gpu, vis if fmt == "cf32" else synth.to_cf16(vis), op, TOL_F32, label=f"fuzz {fmt}")


def test_repeatable_bitwise():
    from paper_2412_14775_amd import rfi
    vis = scene_vis(3, 8, 1024, seed=5)
    B, C, T, _ = vis.shape
    op, rp = make_params(B, C, T, 64, **thresholds_for(64))
    plan = rfi.Plan(rp)
    dev = to_device(vis, "cf32")
    a = run_gpu(plan, dev)
    b = run_gpu(plan, dev)
    plan.close()
    for k in ("avg", "weight", "flags", "stats32"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_outputs_optional():
    vis = scene_vis(2, 3, 256, seed=6)
    op, gpu = screen_both(vis, 16, stats=False, **thresholds_for(16))
    compare(gpu, vis, op, TOL_F32, label="no stats")


def test_size_checks_in_binding():
    import torch
    from paper_2412_14775_amd import rfi
    op, rp = make_params(3, 2, 64, 16)
    plan = rfi.Plan(rp)
    out = plan.alloc_outputs()
    short = torch.zeros((3, 2, 63, 4, 2), dtype=torch.float32, device="cuda:0")
    with pytest.raises(ValueError):
        plan.screen(short, out["avg"], out["weight"], out["flags"])
    wrong = torch.zeros((3, 2, 64, 4, 2), dtype=torch.float16, device="cuda:0")
    with pytest.raises(ValueError):
        plan.screen(wrong, out["avg"], out["weight"], out["flags"])
    plan.close()


def test_persistent_launch_with_a_ragged_last_block():
    """The persistent complex64 launch gives each block U = ceil(streams / (3 x CUs)) streams,
    rounded up to a multiple of its 4 waves: 48 stations x 33 channels (38 808 streams) x 256
    samples at M = 16 on 256 CUs makes U = 52 and a last block of 16 streams (4 per wave).  Every
    stream, the last block's included, against the oracle; flags against the rule applied to the
    kernel's own statistics."""
    import torch
    from paper_2412_14775_amd import rfi
    N, C, T, M = 48, 33, 256, 16
    vis = scene_vis(N, C, T, seed=4833, rfi_channels=(5, 32), duty=(64, 12))
    B = vis.shape[0]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    G = 3 * n_cu
    U = -(-B * C // G)
    if U > 4:
        U = -(-U // 4) * 4
    last = B * C - (-(-B * C // U) - 1) * U
    print(f"{n_cu} CUs: U = {U} streams per block, last block {last}")
    if n_cu == 256:
        assert (U, last) == (52, 16)
    op, gpu = screen_both(vis, M, **thresholds_for(M))
    rep = compare(gpu, vis, op, TOL_F32, label="persistent ragged")
    assert 0.0 < rep["flagged_frac"] < 0.5
    tail = slice(B * C - last, B * C)                  # the last block's streams, flattened
    assert np.isfinite(gpu["avg"].reshape(B * C, 4)[tail]).all()
    assert (gpu["weight"].reshape(-1)[tail] > 0).all()
