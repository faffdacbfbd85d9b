"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against something other than itself: a closed form
from the SK literature the paper cites (Nita & Gary 2010, Section 2.1), a
hand-derived worked window, an invariance of the mathematics, a brute-force
table, or a library routine.  A plausible mistake in the oracle (a dropped j
in Stokes V, SK on |I|^2, the Table-1 one-line bracket, epsilon misplaced, a
wrong comparison direction, flags applied to the wrong samples) fails at least
one of them.
"""
import math

import numpy as np
import pytest
from scipy.special import gammaln

import oracle
from oracle import Params, SK_LOW, SK_HIGH, DS_RE, DS_IM
import synth

EPS = 2.0 ** -23


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * math.sqrt(0.5)


def _stats(win, d=1.0, eps=EPS):
    I, Q, U, V = oracle.stokes(win)
    return (oracle.sk_tau(I, d, eps), oracle.ds_r(Q.real, U.real, V.real, eps),
            oracle.ds_r(Q.imag, U.imag, V.imag, eps))


# ----------------------------------------------------------------------------- Stokes

def test_stokes_are_pauli_traces():
    """I, Q, U, V = tr(V s0), tr(V s3), tr(V s1), tr(V s2) (Section 2, eq. IQUV), via numpy.trace."""
    rng = np.random.default_rng(11)
    v = _cn(rng, (50, 4))
    mats = v.reshape(50, 2, 2)
    s0 = np.eye(2)
    s1 = np.array([[0, 1], [1, 0]], complex)
    s2 = np.array([[0, -1j], [1j, 0]])
    s3 = np.array([[1, 0], [0, -1]], complex)
    I, Q, U, V = oracle.stokes(v)
    for got, s in ((I, s0), (Q, s3), (U, s1), (V, s2)):
        ref = np.trace(mats @ s, axis1=1, axis2=2)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def test_float_pair_input_equals_complex_input():
    rng = np.random.default_rng(12)
    v = _cn(rng, (3, 5, 4)).astype(np.complex64)
    pairs = v.view(np.float32).reshape(3, 5, 4, 2)
    for a, b in zip(oracle.stokes(v), oracle.stokes(pairs)):
        np.testing.assert_array_equal(a, b)


# ----------------------------------------------------------------------------- SK closed forms

def _sk_var_gamma(k, M):
    """Var of the generalised SK estimator for i.i.d. Gamma(k) inputs with d = k
    (Nita & Gary 2010): 2 k (k+1) M^2 Gamma(Mk+2) / ((M-1) Gamma(Mk+4))."""
    return 2 * k * (k + 1) * M * M * math.exp(gammaln(M * k + 2) - gammaln(M * k + 4)) / (M - 1)


@pytest.mark.parametrize("k,M,n", [(1, 16, 200_000), (1, 64, 60_000), (2, 16, 200_000), (2, 64, 60_000)])
def test_sk_unit_mean_and_variance_on_gamma_inputs(k, M, n):
    """P1: |I| ~ Gamma(k) i.i.d. and d = k give E[tau] = 1 and the closed-form variance.

    k = 1: single-pol autocorrelation xx = |x|^2 of circular Gaussian voltage.
    k = 2: dual-pol autocorrelation, I = |x|^2 + |y|^2.
    """
    rng = np.random.default_rng(100 + 10 * k + M)
    x = _cn(rng, (n, M))
    vis = np.zeros((n, M, 4), complex)
    vis[..., 0] = np.abs(x) ** 2
    if k == 2:
        vis[..., 3] = np.abs(_cn(rng, (n, M))) ** 2
    I, _, _, _ = oracle.stokes(vis)
    tau = oracle.sk_tau(I, float(k), 0.0)
    var = _sk_var_gamma(k, M)
    se = math.sqrt(var / n)
    assert abs(tau.mean() - 1.0) < 4 * se, (tau.mean(), se)
    assert abs(tau.var() / var - 1.0) < 0.05, (tau.var(), var)


def test_sk_variance_formula_limit():
    """The closed form tends to 4/M for exponential power (k = 1) as M grows."""
    for M in (1024, 4096):
        assert abs(_sk_var_gamma(1, M) * M / 4.0 - 1.0) < 5.0 / M


@pytest.mark.parametrize("M,d", [(4, 1.0), (16, 2.2), (64, 0.5)])
def test_sk_constant_window(M, d):
    """|I| constant = a: M S2 = M^2 a^2 = S1^2, so tau = -(Md+1)/(M-1) * eps / (M^2 a^2 + eps)."""
    a = 0.37
    vis = np.zeros((M, 4), complex)
    vis[:, 0] = a * np.exp(1j * np.linspace(0, 3, M))      # |I| = a, phase varies
    I, *_ = oracle.stokes(vis)
    tau = oracle.sk_tau(I, d, EPS)
    want = -(M * d + 1) / (M - 1) * EPS / (M * M * a * a + EPS)
    assert tau == pytest.approx(want, rel=1e-9)
    assert oracle.sk_tau(I, d, 0.0) == pytest.approx(0.0, abs=1e-14)


@pytest.mark.parametrize("M,d", [(4, 1.0), (16, 2.2), (64, 0.5)])
def test_sk_one_hot_is_maximum(M, d):
    """One nonzero sample: S1 = a, S2 = a^2, so tau = M d + 1 at eps = 0 (the upper bound)."""
    vis = np.zeros((M, 4), complex)
    vis[M // 2, 3] = 2.5 - 1j
    I, *_ = oracle.stokes(vis)
    assert oracle.sk_tau(I, d, 0.0) == pytest.approx(M * d + 1, rel=1e-12)


def test_sk_bounds_and_scale_invariance():
    """Cauchy-Schwarz: 0 <= tau <= Md + 1 (eps = 0); tau(cV) = tau(V)."""
    rng = np.random.default_rng(13)
    M, d = 16, 1.3
    vis = _cn(rng, (5000, M, 4)) * np.exp(rng.normal(0, 2, (5000, M, 1)))
    I, *_ = oracle.stokes(vis)
    tau = oracle.sk_tau(I, d, 0.0)
    assert tau.min() >= -1e-12 and tau.max() <= M * d + 1 + 1e-9
    I2, *_ = oracle.stokes(vis * (3.7 - 8j))
    np.testing.assert_allclose(oracle.sk_tau(I2, d, 0.0), tau, rtol=1e-10, atol=1e-12)


# ----------------------------------------------------------------------------- DS closed forms

def test_ds_identical_directions():
    """All (q, u, v) along one unit direction with magnitudes m_i: r = (1/M) sum m_i / (m_i + eps)."""
    rng = np.random.default_rng(14)
    M = 32
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    m = rng.uniform(1e-6, 10, M)
    q, u, v = (m[:, None] * n[None]).T
    r = oracle.ds_r(q, u, v, EPS)
    assert r == pytest.approx((m / (m + EPS)).sum() / M, rel=1e-12)
    assert r < 1.0


def test_ds_antipodal_pairs_cancel():
    rng = np.random.default_rng(15)
    vec = rng.standard_normal((8, 3))
    vec = np.concatenate([vec, -vec])
    assert oracle.ds_r(vec[:, 0], vec[:, 1], vec[:, 2], EPS) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("M", [16, 64])
def test_ds_isotropic_null_second_moment(M):
    """i.i.d. symmetric directions: E|sum of unit vectors|^2 = M, so E[M r^2] = 1 (eps = 0)."""
    rng = np.random.default_rng(16 + M)
    n = 100_000 if M == 16 else 30_000
    vis = _cn(rng, (n, M, 4))
    _, Q, U, V = oracle.stokes(vis)
    for part in (np.real, np.imag):
        r = oracle.ds_r(part(Q), part(U), part(V), 0.0)
        x = M * r * r
        se = x.std() / math.sqrt(n)
        assert abs(x.mean() - 1.0) < 4 * se, (x.mean(), se)
        assert r.max() < 1.0


def test_ds_chi2_quantile_approximation():
    """3 M r^2 -> chi^2_3 for large M under the isotropic null (CLT): check the 95th percentile."""
    from scipy.stats import chi2
    rng = np.random.default_rng(17)
    M, n = 256, 20_000
    _, Q, U, V = oracle.stokes(_cn(rng, (n, M, 4)))
    r = oracle.ds_r(Q.real, U.real, V.real, 0.0)
    q95 = np.quantile(r, 0.95)
    assert q95 == pytest.approx(math.sqrt(chi2.ppf(0.95, 3) / (3 * M)), rel=0.02)


# ----------------------------------------------------------------------------- invariances

def _random_su2(rng):
    a = _cn(rng, 2)
    a /= np.linalg.norm(a)
    return np.array([[a[0], -np.conj(a[1])], [a[1], np.conj(a[0])]])


def test_su2_invariance_of_all_statistics():
    """V -> U V U^H leaves I = tr V unchanged and rotates the complex (Q, U, V) by a real SO(3)
    matrix, so tau, r_re and r_im are unchanged.  A missing j in Stokes V breaks this."""
    rng = np.random.default_rng(18)
    M = 16
    vis = _cn(rng, (200, M, 4)) + 0.8 * np.array([1, 0.3j, -0.3j, 0.5])
    U = _random_su2(rng)
    mats = vis.reshape(200, M, 2, 2)
    rot = (U @ mats @ U.conj().T).reshape(200, M, 4)
    for a, b in zip(_stats(vis, 1.7), _stats(rot, 1.7)):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12)


def test_multiplying_by_j_swaps_real_and_imaginary_statistics():
    rng = np.random.default_rng(19)
    vis = _cn(rng, (100, 16, 4))
    t0, re0, im0 = _stats(vis)
    t1, re1, im1 = _stats(1j * vis)
    np.testing.assert_allclose(t1, t0, rtol=1e-12)
    np.testing.assert_allclose(re1, im0, rtol=1e-12)
    np.testing.assert_allclose(im1, re0, rtol=1e-12)


def test_autocorrelations_have_zero_imaginary_alignment():
    """Autos are Hermitian (xx, yy real, yx = conj(xy)): Im(Q, U, V) = 0, p = eps, r_im = 0."""
    e = synth.make_voltages(synth.scene_null(3, 2, 64, seed=5))
    p, q = synth.baseline_pairs(3)
    autos = np.where(p == q)[0]
    vis = synth.correlate(e, autos)
    out = oracle.screen(vis, Params(M=16))
    assert np.all(out["r_im"] == 0.0)
    assert np.all(out["r_re"] > 0.0)


def test_noise_free_polarized_tone():
    """A noise-free, fully polarised tone injected at voltage level: every sample has the
    same direction, so r_re = r_im = 1 - O(eps), and |I| is constant, so tau = 0 - O(eps)."""
    sc = synth.Scene(2, 1, 64, seed=0, rho=0.0, noise_free=True,
                     rfi=[synth.Rfi([0], 20.0, 0.4, 0.3, None, f0=0.13)])
    vis = synth.correlate(synth.make_voltages(sc))
    out = oracle.screen(vis, Params(M=16, d=1.0))
    np.testing.assert_allclose(out["r_re"], 1.0, atol=1e-6)
    np.testing.assert_allclose(out["r_im"][1], 1.0, atol=1e-6)     # the cross baseline
    np.testing.assert_allclose(out["tau"], 0.0, atol=1e-6)


# ----------------------------------------------------------------------------- worked windows

def _w(*samples):
    return np.array(samples, complex)[None]


WIN_A = _w(*[(1, 0, 0, 0)] * 4)
WIN_B = _w((1, 0, 0, 0), (0, 0, 0, 0), (0, 0, 0, 0), (0, 0, 0, 0))
WIN_D = _w((1, 0, 0, 0), (0, 0, 0, 1), (0, 1, 1, 0), (0, 1j, -1j, 0))


@pytest.mark.parametrize("d", [1.0, 0.5])
def test_worked_window_A_constant(d):
    """A = 4 x (1,0,0,0): I = 1 each, S1 = 4, S2 = 4 -> tau = pre (16/(16+eps) - 1);
    Re(Q,U,V) = (1,0,0) each, p = 1 + eps -> r_re = 1/(1+eps); Im parts 0 -> r_im = 0."""
    tau, rre, rim = _stats(WIN_A, d)
    pre = (4 * d + 1) / 3
    assert tau[0] == pytest.approx(pre * (16 / (16 + EPS) - 1), rel=1e-9)
    assert rre[0] == pytest.approx(1 / (1 + EPS), rel=1e-15)
    assert rim[0] == 0.0


@pytest.mark.parametrize("d", [1.0, 0.5])
def test_worked_window_B_one_hot(d):
    """B: one sample (1,0,0,0), three zeros: S1 = S2 = 1 -> tau = pre (4/(1+eps) - 1) (= 4d+1 at eps=0);
    r_re = (1/(1+eps))/4."""
    tau, rre, rim = _stats(WIN_B, d)
    pre = (4 * d + 1) / 3
    assert tau[0] == pytest.approx(pre * (4 / (1 + EPS) - 1), rel=1e-12)
    assert rre[0] == pytest.approx(0.25 / (1 + EPS), rel=1e-12)
    assert rim[0] == 0.0


def test_worked_window_D_by_hand():
    """D = (1,0,0,0), (0,0,0,1), (0,1,1,0), (0,j,-j,0):
    |I| = 1, 1, 0, 0 -> S1 = S2 = 2 -> tau = (5/3)(8/(4+eps) - 1)  (= 5/3 at eps = 0, d = 1).
    Re(Q,U,V) = (1,0,0), (-1,0,0), (0,2,0), (0,0,-2) -> normalised sum (0, 2/(2+eps), -2/(2+eps))
    -> r_re = sqrt(2) * 2/(2+eps) / 4  (= sqrt(2)/4 at eps = 0).  Im parts all 0 -> r_im = 0."""
    tau, rre, rim = _stats(WIN_D, 1.0)
    assert tau[0] == pytest.approx(5 / 3 * (8 / (4 + EPS) - 1), rel=1e-12)
    assert rre[0] == pytest.approx(math.sqrt(2) * 2 / (2 + EPS) / 4, rel=1e-12)
    assert rim[0] == 0.0


# Window C: four samples with every correlation nonzero, complex and unequal in size, so that
# each convention of Section 2 eq. (IQUV) and Section 2.1 shows in the statistics.  The values
# were computed from the definitions in 50-digit decimal arithmetic (eps = 2^-23, W = 4).
WIN_C = _w((1 + 2j, 2 - 1j, -1 + 1j, 3), (-2 + 1j, 1j, 2 + 2j, -1 - 1j),
           (0.5 - 1j, -1 + 0.5j, 1 - 2j, 2 + 1j), (1 + 1j, 3 - 2j, -2, -0.5 + 0.5j))
C_TAU = {1.0: 0.21878537824648759078730028155504581, 0.5: 0.13127122694789255447238016893302749}
C_R_RE = 0.51851931750774140389812422056026663
C_R_IM = 0.20739014015070117673008540179000159
# the same window under readings the paper does not make (they must not be produced):
C_WRONG = {
    "V without j (r_re, r_im)": (0.413889574309308, 0.330967786415696),
    "SK of |I|^2 (tau, d = 1)": 0.795506044850538,
    "Table 1 one-line bracket (tau, d = 1)": 0.885452044913154,
}


@pytest.mark.parametrize("d", [1.0, 0.5])
def test_worked_window_C_high_precision(d):
    """Window C against its 50-digit values: tau (Section 2.1 eq., Table 1 eps), r_re, r_im
    (Section 2.2, Table 2 eps), flags SK_LOW | DS_RE at (s_low, s_high, gamma) = (0.5, 2, 0.4)."""
    tau, rre, rim = _stats(WIN_C, d)
    assert tau[0] == pytest.approx(C_TAU[d], rel=1e-13)
    assert rre[0] == pytest.approx(C_R_RE, rel=1e-13)
    assert rim[0] == pytest.approx(C_R_IM, rel=1e-13)
    out = oracle.screen(WIN_C[None], Params(M=4, d=d, s_low=0.5, s_high=2.0, gamma=0.4))
    assert out["flags"].tolist() == [[[SK_LOW | DS_RE]]]


def test_worked_window_C_is_not_a_wrong_convention():
    tau, rre, rim = _stats(WIN_C, 1.0)
    no_j = C_WRONG["V without j (r_re, r_im)"]
    assert abs(rre[0] - no_j[0]) > 0.05 and abs(rim[0] - no_j[1]) > 0.05
    assert abs(tau[0] - C_WRONG["SK of |I|^2 (tau, d = 1)"]) > 0.1
    assert abs(tau[0] - C_WRONG["Table 1 one-line bracket (tau, d = 1)"]) > 0.1
    # V = -j (xy - yx) is a reflection of (Q, U, V): the same r
    I, Q, U, V = oracle.stokes(WIN_C)
    assert oracle.ds_r(Q.real, U.real, -V.real, EPS)[0] == pytest.approx(C_R_RE, rel=1e-13)


def _w20():
    """A 10 x 2 time x frequency window (W = 20, Sections 3.2 and 4.1), then a second one.
    Window 0: channel 0 holds 10 x (1, 0, 0, 0) (I = 1, Re(Q, U, V) = (1, 0, 0)); channel 1
    holds 10 x (1, 1, 1, 1) (I = 2, Re(Q, U, V) = (0, 2, 0)).
    Window 1, both channels: (1, 0, 0, 0) and (1, 0, 0, 2) alternating (I = 1, 3; Re(Q, U, V) =
    (1, 0, 0), (-1, 0, 0)), so the directions cancel."""
    vis = np.zeros((2, 20, 4), complex)
    vis[0, :10] = (1, 0, 0, 0)
    vis[1, :10] = (1, 1, 1, 1)
    vis[:, 10::2] = (1, 0, 0, 0)
    vis[:, 11::2] = (1, 0, 0, 2)
    return vis


def test_time_frequency_window_W20_by_hand():
    """W = 20 over two channels.  Window 0: S1 = 10 + 20 = 30, S2 = 10 + 40 = 50, so
    tau = (20d+1)/19 (20 * 50 / (900 + eps) - 1); the unit vectors sum to (10/(1+eps), 20/(2+eps), 0),
    r_re = |sum| / 20 (= sqrt(2)/2 at eps = 0), r_im = 0.  Window 1: S1 = 40, S2 = 100,
    tau = (20d+1)/19 (2000 / (1600 + eps) - 1), r_re = 0.  With d = 3 and (0.5, 2, 0.4), window 0
    is flagged SK_LOW | DS_RE, window 1 is kept; the flag removes window 0 from both channels'
    averages, which are then the mean of window 1's samples, (1, 0, 0, 1), with weight 1/2.
    Had the window been 20 samples of one channel, tau would be 0 - O(eps) and r_re 1 - O(eps)."""
    d = 3.0
    out = oracle.screen(_w20()[None], Params(M=10, F=2, d=d, s_low=0.5, s_high=2.0, gamma=0.4))
    pre = (20 * d + 1) / 19
    assert out["tau"][0, 0, 0] == pytest.approx(pre * (1000 / (900 + EPS) - 1), rel=1e-13)
    assert out["tau"][0, 0, 1] == pytest.approx(pre * (2000 / (1600 + EPS) - 1), rel=1e-13)
    r0 = math.hypot(10 / (1 + EPS), 20 / (2 + EPS)) / 20
    assert out["r_re"][0, 0, 0] == pytest.approx(r0, rel=1e-14)
    assert out["r_re"][0, 0, 1] == 0.0 and np.all(out["r_im"] == 0.0)
    assert out["flags"].tolist() == [[[SK_LOW | DS_RE, 0]]]
    np.testing.assert_array_equal(out["avg"][0], [[1, 0, 0, 1], [1, 0, 0, 1]])
    np.testing.assert_array_equal(out["weight"][0], [0.5, 0.5])


def test_masked_average_worked_example():
    """T = 8, M = 4, windows [D, B], (s_low, s_high, gamma) = (0.5, 2, 0.4), d = 1:
    D: tau = 5/3, r_re = 0.354, r_im = 0 -> kept;  B: tau = 5 > 2 -> SK_HIGH.
    avg = mean of D = (1/4, (1+j)/4, (1-j)/4, 1/4), weight = 4/8."""
    vis = np.concatenate([WIN_D, WIN_B], axis=1)           # [1, 8, 4]: one stream
    out = oracle.screen(vis[None], Params(M=4, d=1.0, s_low=0.5, s_high=2.0, gamma=0.4))
    assert out["flags"].tolist() == [[[0, SK_HIGH]]]
    np.testing.assert_allclose(out["avg"][0, 0], [0.25, 0.25 + 0.25j, 0.25 - 0.25j, 0.25], atol=1e-15)
    assert out["weight"][0, 0] == 0.5
    everything = oracle.screen(vis[None], Params(M=4, s_low=0.5, s_high=0.6, gamma=0.4))
    assert np.all(everything["flags"] != 0)
    assert np.all(everything["avg"] == 0) and everything["weight"][0, 0] == 0.0


# ----------------------------------------------------------------------------- flags

@pytest.mark.parametrize("tau,rre,rim,bits", [
    (1.0, 0.1, 0.1, 0),
    (0.5, 0.4, 0.4, 0),                           # equality is not a flag (strict tests)
    (2.0, 0.0, 0.0, 0),
    (0.4999, 0.1, 0.1, SK_LOW),
    (2.0001, 0.1, 0.1, SK_HIGH),
    (1.0, 0.4001, 0.1, DS_RE),
    (1.0, 0.1, 0.41, DS_IM),
    (0.1, 0.9, 0.9, SK_LOW | DS_RE | DS_IM),
    (float("nan"), 0.1, 0.1, SK_LOW),             # NaN fails the in-range test
    (1.0, float("nan"), float("nan"), DS_RE | DS_IM),
    (float("inf"), 0.1, 0.1, SK_HIGH),
])
def test_flag_bits_brute_force(tau, rre, rim, bits):
    assert int(oracle.flag_bits(tau, rre, rim, 0.5, 2.0, 0.4)) == bits


def test_flag_options_clear_tests():
    b = oracle.flag_bits(0.1, 0.9, 0.9, 0.5, 2.0, 0.4, options=oracle.OPT_NO_SK)
    assert int(b) == DS_RE | DS_IM
    b = oracle.flag_bits(0.1, 0.9, 0.9, 0.5, 2.0, 0.4, options=oracle.OPT_NO_DS)
    assert int(b) == SK_LOW


def test_nonfinite_input_flags_window():
    """A NaN / Inf sample flags its window, and the excluded window leaves the average
    equal to the plain mean of the other window (numpy.mean)."""
    rng = np.random.default_rng(20)
    for bad in (np.nan, np.inf):
        vis = _cn(rng, (1, 1, 32, 4))
        vis[0, 0, 5, 1] = bad
        out = oracle.screen(vis, Params(M=16, s_low=-1e30, s_high=1e30, gamma=1.0))
        assert out["flags"][0, 0, 0] != 0 and out["flags"][0, 0, 1] == 0
        np.testing.assert_allclose(out["avg"][0, 0], vis[0, 0, 16:].mean(axis=0), rtol=1e-13)
        assert out["weight"][0, 0] == 0.5


def test_all_zero_window_is_flagged_low():
    vis = np.zeros((1, 1, 16, 4), complex)
    out = oracle.screen(vis, Params(M=16, d=2.0))
    assert out["tau"][0, 0, 0] == pytest.approx(-(16 * 2 + 1) / 15)
    assert out["flags"][0, 0, 0] == SK_LOW


# ----------------------------------------------------------------------------- averaging

def test_masked_average_library_cross_check():
    rng = np.random.default_rng(21)
    vis = _cn(rng, (3, 2, 64, 4))
    flags = (rng.random((3, 2, 8)) < 0.3).astype(np.uint8)
    avg, w = oracle.masked_average(vis, flags, 8)
    for b in range(3):
        for c in range(2):
            keep = np.repeat(flags[b, c] == 0, 8)
            ref = vis[b, c][keep].mean(axis=0) if keep.any() else np.zeros(4)
            np.testing.assert_allclose(avg[b, c], ref, rtol=1e-13, atol=1e-15)
            assert w[b, c] == keep.mean()


# ----------------------------------------------------------------------------- time x frequency windows

def test_time_frequency_window_brute_force():
    """A T x F window holds M time samples of F adjacent channels (Sections 3.2, 4.1)."""
    rng = np.random.default_rng(22)
    C, T, M, F = 4, 20, 10, 2
    vis = _cn(rng, (C, T, 4))
    out = oracle.screen(vis, Params(M=M, F=F))
    assert out["tau"].shape == (C // F, T // M)
    for cg in range(C // F):
        for k in range(T // M):
            win = vis[cg * F:(cg + 1) * F, k * M:(k + 1) * M].reshape(1, F * M, 4)
            tau, rre, rim = _stats(win, 1.0)
            assert out["tau"][cg, k] == pytest.approx(tau[0], rel=1e-12)
            assert out["r_re"][cg, k] == pytest.approx(rre[0], rel=1e-12)
            assert out["r_im"][cg, k] == pytest.approx(rim[0], rel=1e-12)


def test_time_frequency_window_with_F1_is_time_window():
    rng = np.random.default_rng(23)
    vis = _cn(rng, (3, 48, 4))
    a = oracle.screen(vis, Params(M=16, F=1))
    win = vis.reshape(3, 3, 16, 4)
    tau, rre, rim = _stats(win, 1.0)
    np.testing.assert_array_equal(a["tau"], tau)
    np.testing.assert_array_equal(a["r_re"], rre)


# ----------------------------------------------------------------------------- adaptive state

def test_adaptive_state_matches_numpy_moments():
    """After several integrations the running (n, mean, M2) equals numpy's mean / var
    over every unflagged window seen so far; thresholds are mean -/+ kappa sigma."""
    rng = np.random.default_rng(24)
    params = Params(M=16, d=1.0, s_low=0.2, s_high=3.0, gamma=0.6, kappa_sk=2.5,
                    kappa_ds=2.0, n_warm=20, options=oracle.OPT_ADAPTIVE)
    state = oracle.AdaptiveState((2, 3))
    seen = [[[] for _ in range(3)] for _ in range(2)]
    for it in range(4):
        vis = _cn(rng, (2, 3, 128, 4))
        vis[0, 1, 32:48] *= 8.0                      # some RFI-like windows
        out = oracle.screen_adaptive(vis, params, state)
        st = np.stack([out["tau"], out["r_re"], out["r_im"]], -1)
        for b in range(2):
            for c in range(3):
                seen[b][c].append(st[b, c][out["flags"][b, c] == 0])
    for b in range(2):
        for c in range(3):
            allw = np.concatenate(seen[b][c])
            assert state.n[b, c] == len(allw)
            np.testing.assert_allclose(state.mean[b, c], allw.mean(axis=0), rtol=1e-12)
            np.testing.assert_allclose(state.m2[b, c], allw.var(axis=0) * len(allw), rtol=1e-10)
    th = state.thresholds(params)
    sd = np.sqrt(state.m2 / (state.n - 1)[..., None])
    np.testing.assert_allclose(th["s_high"], state.mean[..., 0] + np.float32(2.5) * sd[..., 0])
    np.testing.assert_allclose(th["gamma_im"], state.mean[..., 2] + np.float32(2.0) * sd[..., 2])


@pytest.mark.parametrize("M", [16, 64])
def test_adaptive_state_converges_to_null_moments(M):
    """The running state against closed forms rather than numpy: unpolarized dual-pol voltages
    (xx = |x|^2, xy = x y*, yx = y x*, yy = |y|^2 with x, y circular Gaussian) give |I| ~ Gamma(2),
    so with d = 2 the state's tau mean tends to 1 and its variance to the Nita & Gary closed form;
    each sample's Re(Q, U, V) has length |I| and a direction uniform on the sphere, so
    E[r_re^2] = E|sum of M unit vectors|^2 / M^2 = 1/M exactly (mean^2 + variance of the state).
    Five integrations, nothing flagged (loose plan thresholds, adaptive ones never engaged)."""
    rng = np.random.default_rng(700 + M)
    n_int, n_win = 5, 8000
    params = Params(M=M, d=2.0, s_low=-10.0, s_high=100.0, gamma=1.5,
                    n_warm=10 ** 9, options=oracle.OPT_ADAPTIVE)
    state = oracle.AdaptiveState((1,))
    for _ in range(n_int):
        x, y = _cn(rng, (1, n_win * M)), _cn(rng, (1, n_win * M))
        xy = x * np.conj(y)
        vis = np.stack([np.abs(x) ** 2, xy, np.conj(xy), np.abs(y) ** 2], axis=-1)
        out = oracle.screen_adaptive(vis, params, state)
        assert not out["flags"].any()
    n = n_int * n_win
    assert state.n[0] == n
    var_tau = _sk_var_gamma(2, M)
    mean, var = state.mean[0], state.m2[0] / (n - 1)
    assert abs(mean[0] - 1.0) < 4 * math.sqrt(var_tau / n), mean[0]
    assert abs(var[0] / var_tau - 1.0) < 0.06, (var[0], var_tau)
    r2 = mean[1] ** 2 + var[1] * (n - 1) / n                # sample mean of r_re^2
    se_r2 = math.sqrt(2.0 / 3.0 / n) / M                    # |S|^2 ~ (M/3) chi2_3 for large M
    assert abs(r2 - 1.0 / M) < 4 * se_r2, (r2, 1.0 / M)
    assert state.mean[0, 2] == 0.0 and state.m2[0, 2] == 0.0   # autocorrelation-like: Im parts vanish


def test_adaptive_state_cold_uses_plan_thresholds():
    params = Params(M=16, s_low=0.25, s_high=2.5, gamma=0.5, n_warm=1000)
    state = oracle.AdaptiveState((4,))
    th = state.thresholds(params)
    assert np.all(th["s_low"] == np.float32(0.25)) and np.all(th["gamma"] == np.float32(0.5))
