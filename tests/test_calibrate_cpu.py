"""Hyperparameter helpers (Section 2.3) against the oracle's Monte Carlo (CPU only)."""
import math

import numpy as np
import pytest
from scipy.special import gammaln

import oracle
from paper_2412_14775_amd import rfi


def _gamma_windows(rng, k, W, n):
    """Windows whose |I| are i.i.d. Gamma(k): k = 1 single-pol autos, k = 2 dual-pol autos."""
    vis = np.zeros((n, W, 4), complex)
    vis[..., 0] = rng.gamma(k, size=(n, W))
    return vis


def _oracle_tau(vis, d):
    I, *_ = oracle.stokes(vis)
    return oracle.sk_tau(I, d, 0.0)


@pytest.mark.parametrize("W,d", [(4, 1.0), (16, 1.0), (20, 2.0), (64, 2.2), (256, 0.7)])
def test_null_moments_match_the_closed_form_variance(W, d):
    """Mean 1 and the Nita & Gary variance 2d(d+1)W^2 Gamma(Wd+2)/((W-1) Gamma(Wd+4)),
    derived independently of the Dirichlet-moment route the helper takes."""
    mean, var, _ = rfi.rfi_sk_null_moments(W, d)
    d = float(np.float32(d))                     # the helper takes d as a float32 plan value
    ng = 2 * d * (d + 1) * W * W * math.exp(gammaln(W * d + 2) - gammaln(W * d + 4)) / (W - 1)
    assert mean == pytest.approx(1.0, abs=1e-9)
    assert var == pytest.approx(ng, rel=1e-9)


@pytest.mark.parametrize("k,W", [(1, 16), (2, 20), (1, 64)])
def test_null_skewness_matches_monte_carlo(k, W):
    rng = np.random.default_rng(40 + W)
    tau = _oracle_tau(_gamma_windows(rng, k, W, 200_000), float(k))
    mc = ((tau - tau.mean()) ** 3).mean() / tau.std() ** 3
    _, _, skew = rfi.rfi_sk_null_moments(W, float(k))
    assert skew == pytest.approx(mc, rel=0.06)


@pytest.mark.parametrize("W", [16, 64, 256])
def test_ds_threshold_matches_isotropic_null_quantile(W):
    rng = np.random.default_rng(50 + W)
    n = 40_000 if W < 256 else 10_000
    z = (rng.standard_normal((n, W, 4)) + 1j * rng.standard_normal((n, W, 4))) / math.sqrt(2)
    _, Q, U, V = oracle.stokes(z)
    r = oracle.ds_r(Q.real, U.real, V.real, 0.0)
    g = rfi.rfi_thresholds_from_pfa(W, 1.0, 0.05, 0.05)["ds_gamma"]
    assert g == pytest.approx(np.quantile(r, 0.95), rel=0.03)
    assert (r > g).mean() == pytest.approx(0.05, abs=0.01)


@pytest.mark.parametrize("W,tol", [(64, 0.4), (256, 0.25), (16, 0.7)])
def test_sk_thresholds_reach_the_requested_false_alarm_rate(W, tol):
    """Achieved two-sided false-alarm rate of the theory thresholds on Gamma(1) null windows.
    The Cornish-Fisher tails get better with W; at W = 16 the paper's fine-tuning is needed."""
    rng = np.random.default_rng(60 + W)
    tau = _oracle_tau(_gamma_windows(rng, 1, W, 100_000), 1.0)
    th = rfi.rfi_thresholds_from_pfa(W, 1.0, 0.05, 0.05)
    pfa = ((tau < th["sk_low"]) | (tau > th["sk_high"])).mean()
    assert abs(pfa / 0.05 - 1) < tol, pfa


@pytest.mark.parametrize("k,W", [(1, 16), (2, 64)])
def test_calibration_recovers_d_and_the_false_alarm_rate(k, W):
    """Calibrate on one null sample (statistics written with d = 1), check on another."""
    rng = np.random.default_rng(70 + W)
    train = _gamma_windows(rng, k, W, 100_000)
    st = np.zeros((len(train), 3), np.float32)
    st[:, 0] = _oracle_tau(train, 1.0)
    _, Q, U, V = oracle.stokes(train + 0.3 * rng.standard_normal(train.shape))
    st[:, 1] = oracle.ds_r(Q.real, U.real, V.real, 0.0)
    cal = rfi.rfi_calibrate_from_stats(st, W, 1.0, 0.05, 0.05)
    assert cal["sk_d"] == pytest.approx(k, rel=0.03)
    test = _gamma_windows(rng, k, W, 100_000)
    tau = _oracle_tau(test, cal["sk_d"])
    pfa = ((tau < cal["sk_low"]) | (tau > cal["sk_high"])).mean()
    assert pfa == pytest.approx(0.05, abs=0.005)
    assert (st[:, 1] > cal["ds_gamma"]).mean() == pytest.approx(0.05, abs=0.002)


def test_helper_argument_checks():
    with pytest.raises(rfi.RfiError):
        rfi.rfi_sk_null_moments(1, 1.0)
    with pytest.raises(rfi.RfiError):
        rfi.rfi_thresholds_from_pfa(16, 1.0, 0.0, 0.05)
    with pytest.raises(rfi.RfiError):
        rfi.rfi_calibrate_from_stats(np.zeros((10, 3), np.float32), 16, 1.0)
