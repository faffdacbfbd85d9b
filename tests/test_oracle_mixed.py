"""Pins of the paper's mixed-precision emulation (Tables 3-4) against binary16 error bounds
of the float64 oracle (CPU only).  Parity of this form is pinned by error bounds only."""
import math

import numpy as np
import pytest

import oracle
from oracle import Params

U16 = 2.0 ** -11                                 # unit roundoff of binary16


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * math.sqrt(0.5)


def tau_bound(ref_tau, W, d):
    """Group 7 is five binary16 roundings of O(1) quantities plus two input conversions:
    |tau16 - tau64| <= 12 u max(1, pre * ratio) (a loose first-order bound)."""
    pre = (W * d + 1) / (W - 1)
    ratio = ref_tau / pre + 1
    return 12 * U16 * np.maximum(1.0, pre * np.abs(ratio))


def r_bound(W):
    """Sequential binary16 sums of W unit-vector components: |partial_i| <= i, so the sum
    errs by at most u (W(W+1)/2 + W); r = |sum| / W adds a few roundings."""
    return math.sqrt(3) * U16 * (W * (W + 1) / 2 + W) / W + 6 * U16


@pytest.mark.parametrize("W", [10, 20, 64])
def test_mixed_statistics_within_binary16_bounds_of_float64(W):
    rng = np.random.default_rng(80 + W)
    win = (_cn(rng, (4000, W, 4)) * np.exp(rng.normal(0, 0.5, (4000, 1, 1)))).astype(np.complex64)
    d = 1.7
    t16, re16, im16 = oracle.mixed_window_stats(win, d, 2.0 ** -23)
    I, Q, U, V = oracle.stokes(win.astype(np.complex128))
    t64 = oracle.sk_tau(I, float(np.float32(d)), 2.0 ** -23)
    re64 = oracle.ds_r(Q.real, U.real, V.real, 2.0 ** -23)
    im64 = oracle.ds_r(Q.imag, U.imag, V.imag, 2.0 ** -23)
    y = I.real ** 2 + I.imag ** 2
    fits = W * y.sum(-1) < 65504 * (1 - 4 * U16)             # W S2 representable in binary16
    assert np.isfinite(t16[fits]).all()
    assert not np.isfinite(t16[W * y.sum(-1) > 65520]).any()   # overflow -> inf / NaN tau
    ok = fits
    assert np.all(np.abs(t16[ok].astype(float) - t64[ok]) <= tau_bound(t64[ok], W, d))
    assert np.all(np.abs(re16.astype(float) - re64) <= r_bound(W))
    assert np.all(np.abs(im16.astype(float) - im64) <= r_bound(W))
    assert t16.dtype == np.float16 and re16.dtype == np.float16
    # the emulation is not the float64 result: binary16 rounding is visible
    assert np.abs(t16[ok].astype(float) - t64[ok]).max() > 1e-5


def test_binary16_overflow_of_s2_flags_the_window():
    """|I| of 300 in a 20-sample window: W S2 = 20 * 20 * 9e4 exceeds the binary16 range, the
    ratio is inf / inf = NaN, and the negated low test flags the window (the overflow the
    paper's reward penalises)."""
    win = np.zeros((1, 1, 20, 4), np.complex64)
    win[..., 0] = 300.0
    out = oracle.screen_mixed(win, Params(M=20, s_low=0.1, s_high=5.0, gamma=1.0))
    assert np.isnan(out["tau"][0, 0, 0]) or np.isinf(out["tau"][0, 0, 0])
    assert out["flags"][0, 0, 0] & oracle.SK_LOW


def test_mixed_flags_agree_with_float64_on_null_data():
    """The paper reports under 1 % flag difference between 32-bit and the trained mixed form."""
    rng = np.random.default_rng(90)
    vis = _cn(rng, (6, 8, 2000, 4)).astype(np.complex64)
    p = Params(M=10, F=2, d=1.0, s_low=0.45, s_high=2.0, gamma=0.43)
    a = oracle.screen(vis, p)
    b = oracle.screen_mixed(vis, p)
    assert (a["flags"] != b["flags"]).mean() < 0.01


def test_binary16_unit_vector_sums_by_hand():
    """Table 4 group 4 sums the unit vectors in 16 bit, sequentially.  Window of W = 16: first
    (xx, xy, yx, yy) = (1, 0, 0, 0), Re(Q, U, V) = (1, 0, 0); then 15 samples
    ((1 + 2^-12)/2, s/2, s/2, (1 - 2^-12)/2) with s = +1, -1, ..., +1, i.e. Re(Q, U, V) =
    (2^-12, s, 0) (float32 exactly; |.| rounds to 1 in float32, p = 1 + eps).  In binary16 each
    q/p rounds to 2^-12 and 1 + 2^-12 rounds back to 1, so sum q^ = 1; sum u^ = 1 (each u/p rounds
    to 1); then r_re = sqrt(1^2 + 1^2) / 16 = 1.4140625 / 16 = 0.08837890625 in binary16
    (sqrt(2) rounds to 1448 / 1024).  Summed in float32 instead, sum q^ = 1.0036621...
    (1.00390625 in binary16) and r_re = 0.08856201171875; the float64 value is 0.0885503...
    All parts are real: r_im = 0; |I| = 1 throughout, so tau = 0 exactly."""
    q = 2.0 ** -12
    samples = [(1, 0, 0, 0)] + [((1 + q) / 2, s * 0.5, s * 0.5, (1 - q) / 2) for s in [1, -1] * 7 + [1]]
    win = np.array(samples, np.complex64)[None]
    tau, r_re, r_im = oracle.mixed_window_stats(win, 1.0, 2.0 ** -23)
    assert float(r_re[0]) == 0.08837890625
    assert float(r_im[0]) == 0.0 and float(tau[0]) == 0.0
    I, Q, U, V = oracle.stokes(win)
    assert abs(oracle.ds_r(Q.real, U.real, V.real, 2.0 ** -23)[0] - 0.0885503) < 1e-6


def test_mixed_flags_on_the_48_station_10x2_workload():
    """The paper's mixed form against the FP64 oracle on 24 seeded baselines of the 48-station,
    64-channel, 10 x 2 workload (pulsed RFI of random polarisation, 0-20 dB, in 5 % of the
    channels).  Flag masks (flagged or not: the measure of Section 4.3's comparison) differ in
    well under 1 % of windows.  Flag bits differ in about 1 %: where W S2 passes the binary16
    range (strong RFI) the ratio of group 7 is inf / inf or inf, so tau is NaN or infinite and
    the window carries SK_LOW where the FP64 oracle sets SK_HIGH -- flagged either way."""
    import synth
    e = synth.make_voltages(synth.scene_fp32_baseline(1, 48, 64, 3000))
    bl = np.sort(np.random.default_rng(5).choice(1176, 24, replace=False))
    vis = synth.correlate(e, bl)
    p = Params(M=10, F=2, d=2.2, s_low=0.42, s_high=2.0, gamma=0.40)
    a = oracle.screen(vis, p)
    b = oracle.screen_mixed(vis, p)
    mask = float(np.mean((a["flags"] != 0) != (b["flags"] != 0)))
    bits = a["flags"] != b["flags"]
    overflow = ~np.isfinite(b["tau"])
    print(f"masks differ {mask:.5f}, bits differ {bits.mean():.5f}, non-finite mixed tau {overflow.mean():.5f}")
    assert mask < 0.002
    assert np.mean(a["flags"][overflow] != 0) > 0.99         # overflowing windows are RFI the FP64 oracle flags
    # bit differences outside those windows are near-threshold statistics only
    assert np.mean(bits & ~overflow) < 0.002
