"""GPU parity at the size limits of a plan: the longest tiled window, the first window length past
it, and streams as long as the byte limit of one stream allows (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import TOL_F32, compare, flags_from_stats32, near_threshold, stat_error
from tests.test_gpu_screen import check_cf16, scene_vis, screen_both, thresholds_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2412_14775_amd import rfi
    rfi.load_library()
    yield
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fmt", ["cf32", "cf16"])
@pytest.mark.parametrize("M,F,n_windows", [(4096, 1, 3), (8192, 1, 2), (8192, 2, 2)])
def test_longest_windows(fmt, M, F, n_windows):
    """M = 4096 is the longest window of the tiled kernel (several steps per window, segments);
    M = 8192 of one channel goes to the long-window kernel, and over two channels (16384
    samples per window) to the wide-window kernel (32 steps of 512 or 256 samples per window,
    step sums added into the window sums, so no lane sums more than 40 terms in a row)."""
    T = M * n_windows
    vis = scene_vis(2, 2, T, seed=M + n_windows + F, duty=(300, 40))
    if fmt == "cf32":
        op, gpu = screen_both(vis, M, F=F, **thresholds_for(M * F))
        compare(gpu, vis, op, TOL_F32, label=f"cf32 M={M} F={F}")
    else:
        check_cf16(vis, M, f"cf16 M={M} F={F}", F=F, **thresholds_for(M * F))


def _oracle_stream_average(vis_stream, flags_stream, M, chunk_windows=256):
    """The oracle's masked average and weight of one whole stream, taken over chunks of
    ``chunk_windows`` windows (a stream of 2 GiB does not fit the oracle's complex128 copy at
    once): each chunk's oracle sum (average x kept count) is added up in float64 and divided by
    the stream's kept count.  Also returns the mean magnitude of the kept samples per
    correlation, the scale the average's error is measured against."""
    nW = flags_stream.shape[-1]
    total = np.zeros(4, np.complex128)
    mags = np.zeros(4)
    kept = 0
    for w0 in range(0, nW, chunk_windows):
        w1 = min(nW, w0 + chunk_windows)
        v = vis_stream[w0 * M:w1 * M].float().cpu().numpy()[None]        # [1, Tc, 4, 2]
        f = flags_stream[w0:w1][None]                                      # [1, nWc]
        avg_c, w_c = oracle.masked_average(v, f, M)
        n_c = int(round(w_c[0] * (w1 - w0) * M))
        total += avg_c[0] * n_c
        kept += n_c
        keep = np.repeat(f[0] == 0, M)
        vc = oracle.as_complex128(v[0])
        mags += np.abs(vc[keep]).sum(axis=0)
    n = max(kept, 1)
    T = nW * M
    return (total / n if kept else np.zeros(4, np.complex128)), mags / n, kept / T


@pytest.mark.parametrize("fmt,n_windows", [("cf16", 32767), ("cf16", 32764), ("cf32", 16383)])
def test_longest_streams(fmt, n_windows):
    """Streams of just under 2 GiB, the largest a plan accepts (T x bytes per sample < 2^31):
    32767 windows of 4096 samples of complex half (one wave per stream), 32764 (each stream
    split over 4 waves) and 16383 of complex64.  Three baselines of a two-station array.
    Statistics and flags are checked against the oracle on sampled windows (first, last and
    in between); average and weight of one whole stream against the oracle's masked
    average."""
    import torch
    from paper_2412_14775_amd import rfi
    M = 4096
    T = M * n_windows
    sb = 16 if fmt == "cf16" else 32
    assert T * sb < 2 ** 31
    dev = torch.device("cuda:0")
    sc = synth.Scene(2, 1, T, seed=n_windows, rho=0.1)
    e = synth.device_voltages(sc, dev)
    vis = torch.empty((3, 1, T, 4, 2), dtype=torch.float16 if fmt == "cf16" else torch.float32, device=dev)
    synth.correlate_torch(e, vis, fmt, chunk=1)
    del e
    torch.cuda.empty_cache()
    last = n_windows - 1
    vis[1, 0, 7 * M:8 * M] = 0                                       # an empty window (SK low)
    vis[2, 0, last * M:last * M + 8] *= 40                          # a burst in the very last window
    vis[0, 0, (last - 1) * M + 100:(last - 1) * M + 104] *= 40
    th = thresholds_for(M, d=2.2)
    op = oracle.Params(M=M, **th)
    rp = rfi.rfi_params_default(n_stations=2, n_baselines=3, n_channels=1, n_samples=T, block_m=M,
                                vis_format=rfi.RFI_VIS_CF16 if fmt == "cf16" else rfi.RFI_VIS_CF32,
                                sk_d=op.d, sk_low=op.s_low, sk_high=op.s_high, ds_gamma=op.gamma, eps=op.eps)
    plan = rfi.Plan(rp)
    try:
        out = plan.alloc_outputs(flags=True, stats=True)
        plan.screen(vis, out["avg"], out["weight"], out["flags"], out["stats"])
        torch.cuda.synchronize()
    finally:
        plan.close()
    flags = out["flags"].cpu().numpy()
    st32 = out["stats"].cpu().numpy()
    assert flags.shape == (3, 1, n_windows)
    assert flags[1, 0, 7] & 1 and flags[2, 0, last] & 2 and flags[0, 0, last - 1] & 2
    p32 = op.f32()
    thb = dict(s_low=p32.s_low, s_high=p32.s_high, gamma=p32.gamma, gamma_im=p32.gamma)
    assert np.array_equal(flags_from_stats32(st32, thb, 0), flags)

    # oracle on sampled windows, each screened as a one-window stream of its own exact bytes
    rng = np.random.default_rng(n_windows)
    picks = sorted({0, 1, 7, n_windows // 2, last - 1, last, *rng.integers(0, n_windows, 4).tolist()})
    for b in range(3):
        for w in picks:
            win = vis[b, 0, w * M:(w + 1) * M].float().cpu().numpy()
            win = win[..., 0].astype(np.float64) + 1j * win[..., 1]
            ref = oracle.screen(win[None, None], op)
            for k, j in (("tau", 0), ("r_re", 1), ("r_im", 2)):
                err = stat_error(st32[b, 0, w, j], ref[k][0, 0, 0])
                assert err <= TOL_F32, f"{fmt} b={b} window {w}: {k} rel err {err:.3g}"
            if flags[b, 0, w] != ref["flags"][0, 0, 0]:
                assert near_threshold({k: ref[k][0, 0, 0] for k in ("tau", "r_re", "r_im")}, thb, TOL_F32), \
                    f"{fmt} b={b} window {w}: flags {flags[b, 0, w]} vs oracle {ref['flags'][0, 0, 0]}"

    # average and weight of one whole stream (a different one per case) against the oracle's
    # masked average with the kernel's flags
    b = {32767: 2, 32764: 0, 16383: 1}[n_windows]
    avg_ref, scale, w_ref = _oracle_stream_average(vis[b, 0], flags[b, 0], M)
    a = out["avg"][b, 0].cpu().numpy()
    avg = a[..., 0].astype(np.float64) + 1j * a[..., 1]
    err = np.abs(avg - avg_ref) / np.maximum(scale, 1e-30)
    assert err.max() <= TOL_F32, f"{fmt} stream {b}: average rel err {err.max():.3g}"
    np.testing.assert_allclose(float(out["weight"][b, 0]), w_ref, rtol=1e-6, atol=0)
    del vis
    torch.cuda.empty_cache()
