"""Plain FP64 definition of the online SK + DS screen (test infrastructure only).

Section references are to arXiv 2412.14775.  Notation follows the paper:
window W = M time samples (times F channels for a time x frequency window),
statistic tau (SK), r (DS), thresholds s_low, s_high, gamma, constant d.

Readings taken where the paper is silent or ambiguous:

R1  SK input: x_i = |I_i| with S1 = sum x_i, S2 = sum x_i^2 (Section 2.1,
    Table 1 groups 1-4), computed as y_i = Re(I)^2 + Im(I)^2, z_i = sqrt(y_i).
R2  SK bracket: tau = (W d + 1)/(W - 1) * (W S2 / (S1^2 + eps) - 1), i.e. the
    bracket of the Section 2.1 equation (Nita & Gary's estimator, mean 1) with
    the epsilon of Table 1 group 7 added to S1^2.  Table 1's one-line form puts
    the "-1" outside the product, which has no unit mean; it is not used.
R3  epsilon is one plan constant (default 2^-23), used in both places:
    S1^2 + eps (Table 1) and p_i = sqrt(q^2 + u^2 + v^2) + eps (Table 2).
R4  comparisons are strict as printed (Sections 2.1, 2.2), written as negated
    in-range tests for the low and DS thresholds, so that a NaN statistic
    (non-finite input) flags the window:
      SK_LOW  = not (tau >= s_low)     SK_HIGH = tau > s_high
      DS_RE   = not (r_re <= gamma)    DS_IM   = not (r_im <= gamma)
R5  a window is flagged if any bit is set; a flag covers all four correlations
    of every sample of the window (end of Section 2.2).
R6  flagged windows are left out of the time average (Section 2.1); the
    average is over the unflagged samples, weight = unflagged fraction n / T,
    and an integration with every window flagged gives average 0, weight 0.
R7  option bits NO_SK / NO_DS clear the corresponding flag bits, so the test
    is not applied.
R8  Stokes V = j (xy - yx) exactly as printed (Section 2, eq. IQUV).
R9  the window is M consecutive time samples of one channel (F = 1) unless a
    time x frequency window (Section 3.2, Section 4.1: T x F = 10 x 2, 5 x 4)
    is requested; then it is M time samples of F adjacent channels.
R10 thresholds, d and eps are single-precision plan values; the oracle uses
    exactly those values (rounded to float32) in float64 arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

SK_LOW, SK_HIGH, DS_RE, DS_IM = 1, 2, 4, 8
OPT_NO_SK, OPT_NO_DS, OPT_ADAPTIVE, OPT_PAPER_MIXED = 1, 2, 4, 8

EPS_DEFAULT = 2.0 ** -23


def _f32(x) -> float:
    return float(np.float32(x))


@dataclass
class Params:
    """Screen parameters (Section 2.3): window, d, thresholds, epsilon, options."""
    M: int
    d: float = 1.0
    s_low: float = 0.5
    s_high: float = 2.0
    gamma: float = 0.4
    eps: float = EPS_DEFAULT
    options: int = 0
    F: int = 1
    kappa_sk: float = 3.0
    kappa_ds: float = 3.0
    n_warm: int = 0

    def f32(self) -> "Params":
        """The same parameters with every real value rounded to float32 (R10)."""
        return Params(self.M, _f32(self.d), _f32(self.s_low), _f32(self.s_high),
                      _f32(self.gamma), _f32(self.eps), self.options, self.F,
                      _f32(self.kappa_sk), _f32(self.kappa_ds), self.n_warm)


def as_complex128(vis) -> np.ndarray:
    """Visibilities as complex128 [..., 4]: accepts complex arrays or (re, im) float pairs [..., 4, 2]."""
    a = np.asarray(vis)
    if np.iscomplexobj(a):
        return a.astype(np.complex128)
    a = a.astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def stokes(vis):
    """Complex Stokes parameters of V = [[xx, xy], [yx, yy]] (Section 2, eq. IQUV).

    I = xx + yy,  Q = xx - yy,  U = xy + yx,  V = j (xy - yx).
    """
    v = as_complex128(vis)
    xx, xy, yx, yy = v[..., 0], v[..., 1], v[..., 2], v[..., 3]
    return xx + yy, xx - yy, xy + yx, 1j * (xy - yx)


def sk_tau(I, d: float, eps: float):
    """Spectral-kurtosis statistic over the last axis (the window), Section 2.1 with Table 1.

    y_i = Re(I_i)^2 + Im(I_i)^2 (= |I_i|^2),  z_i = sqrt(y_i) (= |I_i|),
    S1 = sum z_i,  S2 = sum y_i,
    tau = (W d + 1)/(W - 1) * (W S2 / (S1^2 + eps) - 1)          (readings R1-R3)
    """
    W = I.shape[-1]
    y = I.real ** 2 + I.imag ** 2
    z = np.sqrt(y)
    S1 = z.sum(axis=-1)
    S2 = y.sum(axis=-1)
    pre = (W * d + 1.0) / (W - 1.0)
    return pre * (W * S2 / (S1 * S1 + eps) - 1.0)


def ds_r(q, u, v, eps: float):
    """Directional statistic over the last axis, Section 2.2 with Table 2.

    p_i = sqrt(q_i^2 + u_i^2 + v_i^2) + eps,  (q^, u^, v^)_i = (q, u, v)_i / p_i,
    r = sqrt((sum q^)^2 + (sum u^)^2 + (sum v^)^2) / W.
    """
    W = q.shape[-1]
    p = np.sqrt(q * q + u * u + v * v) + eps
    Qs = (q / p).sum(axis=-1)
    Us = (u / p).sum(axis=-1)
    Vs = (v / p).sum(axis=-1)
    return np.sqrt(Qs * Qs + Us * Us + Vs * Vs) / W


def flag_bits(tau, r_re, r_im, s_low, s_high, gamma, options: int = 0,
              gamma_im=None) -> np.ndarray:
    """Flag bits per window (Sections 2.1 and 2.2, combined by OR; readings R4, R7).

    Thresholds may be scalars or arrays broadcastable to the statistics.
    ``gamma_im`` (default: ``gamma``) is the DS threshold of the imaginary part.
    """
    tau = np.asarray(tau, np.float64)
    r_re = np.asarray(r_re, np.float64)
    r_im = np.asarray(r_im, np.float64)
    g_im = gamma if gamma_im is None else gamma_im
    with np.errstate(invalid="ignore"):
        bits = (np.where(~(tau >= s_low), SK_LOW, 0)
                | np.where(tau > s_high, SK_HIGH, 0)
                | np.where(~(r_re <= gamma), DS_RE, 0)
                | np.where(~(r_im <= g_im), DS_IM, 0))
    if options & OPT_NO_SK:
        bits &= ~(SK_LOW | SK_HIGH)
    if options & OPT_NO_DS:
        bits &= ~(DS_RE | DS_IM)
    return bits.astype(np.uint8)


def window_view(vis, M: int, F: int = 1):
    """Group visibilities [..., C, T, 4] into windows [..., C/F, T/M, F*M, 4] (reading R9)."""
    v = as_complex128(vis)
    *lead, C, T, four = v.shape
    assert four == 4 and T % M == 0 and C % F == 0
    v = v.reshape(*lead, C // F, F, T // M, M, 4)
    v = np.moveaxis(v, -4, -3)                      # [..., C/F, T/M, F, M, 4]
    return v.reshape(*lead, C // F, T // M, F * M, 4)


def _window_stats(win, d, eps):
    I, Q, U, V = stokes(win)
    tau = sk_tau(I, d, eps)
    r_re = ds_r(Q.real, U.real, V.real, eps)
    r_im = ds_r(Q.imag, U.imag, V.imag, eps)
    return tau, r_re, r_im


def masked_average(vis, flags, M: int, F: int = 1):
    """Flag-masked time average and weight (Section 2.1; readings R5, R6).

    vis [..., C, T, 4], flags [..., C/F, T/M] -> avg [..., C, 4] complex128, weight [..., C].
    """
    v = as_complex128(vis)
    *lead, C, T, _ = v.shape
    keep = (np.asarray(flags) == 0)                          # [..., C/F, T/M]
    keep = np.repeat(np.repeat(keep, F, axis=-2), M, axis=-1)  # [..., C, T]
    n = keep.sum(axis=-1)
    # flagged samples are left out of the sum (not multiplied by zero: a NaN or
    # Inf in a flagged window must not reach the average)
    total = np.where(keep[..., None], v, 0.0).sum(axis=-2)
    with np.errstate(invalid="ignore", divide="ignore"):
        avg = np.where(n[..., None] > 0, total / np.maximum(n, 1)[..., None], 0.0)
    return avg, n / T


def screen(vis, params: Params, thresholds: Optional[dict] = None):
    """One integration of the screen on visibilities [..., C, T, 4].

    Returns a dict with tau, r_re, r_im [..., C/F, T/M] (float64), flags (uint8),
    avg [..., C, 4] (complex128) and weight [..., C] (float64).
    ``thresholds`` may override s_low, s_high, gamma, gamma_im with per-window
    arrays (used by the adaptive extension); otherwise the plan values apply.
    """
    p = params.f32()
    win = window_view(vis, p.M, p.F)
    tau, r_re, r_im = _window_stats(win, p.d, p.eps)
    th = dict(s_low=p.s_low, s_high=p.s_high, gamma=p.gamma, gamma_im=p.gamma)
    if thresholds:
        th.update(thresholds)
    flags = flag_bits(tau, r_re, r_im, th["s_low"], th["s_high"], th["gamma"],
                      p.options, th["gamma_im"])
    avg, weight = masked_average(vis, flags, p.M, p.F)
    return dict(tau=tau, r_re=r_re, r_im=r_im, flags=flags, avg=avg, weight=weight)


# --------------------------------------------------------------------------- adaptive thresholds

class AdaptiveState:
    """Per-stream running (n, mean, M2) of tau, r_re, r_im over unflagged windows.

    An extension the paper lists as future work (Section 5: thresholds adapted
    online, per data stream).  Each integration's batch moments are computed
    two-pass in float64 and merged with the pairwise update of Chan, Golub &
    LeVeque (1979):  n' = n + n_b,  delta = mean_b - mean,
    mean' = mean + delta n_b / n',  M2' = M2 + M2_b + delta^2 n n_b / n'.
    Once n >= n_warm (and n >= 2), with sigma = sqrt(M2 / (n - 1)):
    s_low = mean_tau - kappa_sk sigma_tau, s_high = mean_tau + kappa_sk sigma_tau,
    gamma_re = mean_re + kappa_ds sigma_re, gamma_im = mean_im + kappa_ds sigma_im.
    Before that the plan thresholds apply.
    """

    def __init__(self, stream_shape):
        self.n = np.zeros(stream_shape, np.int64)
        self.mean = np.zeros(tuple(stream_shape) + (3,), np.float64)
        self.m2 = np.zeros(tuple(stream_shape) + (3,), np.float64)

    def thresholds(self, params: Params):
        p = params.f32()
        warm = (self.n >= max(p.n_warm, 2))
        with np.errstate(invalid="ignore", divide="ignore"):
            sd = np.sqrt(self.m2 / np.maximum(self.n - 1, 1)[..., None])
        s_low = np.where(warm, self.mean[..., 0] - p.kappa_sk * sd[..., 0], p.s_low)
        s_high = np.where(warm, self.mean[..., 0] + p.kappa_sk * sd[..., 0], p.s_high)
        g_re = np.where(warm, self.mean[..., 1] + p.kappa_ds * sd[..., 1], p.gamma)
        g_im = np.where(warm, self.mean[..., 2] + p.kappa_ds * sd[..., 2], p.gamma)
        return dict(s_low=s_low, s_high=s_high, gamma=g_re, gamma_im=g_im)

    def update(self, stats, keep):
        """Merge one integration: stats [..., nW, 3], keep [..., nW] (unflagged windows)."""
        kb = keep.astype(np.float64)
        nb = kb.sum(axis=-1)
        with np.errstate(invalid="ignore", divide="ignore"):
            mb = (stats * kb[..., None]).sum(axis=-2) / np.maximum(nb, 1)[..., None]
            dev = (stats - mb[..., None, :]) * kb[..., None]
        m2b = (dev * dev).sum(axis=-2)
        n0 = self.n.astype(np.float64)
        n1 = n0 + nb
        has = nb > 0
        delta = mb - self.mean
        frac = np.where(has, nb / np.maximum(n1, 1), 0.0)[..., None]
        cross = np.where(has, n0 * nb / np.maximum(n1, 1), 0.0)[..., None]
        self.mean = np.where(has[..., None], self.mean + delta * frac, self.mean)
        self.m2 = np.where(has[..., None], self.m2 + m2b + delta * delta * cross, self.m2)
        self.n = self.n + nb.astype(np.int64)


def screen_adaptive(vis, params: Params, state: AdaptiveState):
    """One integration with per-stream thresholds taken from ``state``, then a state update.

    vis [..., C, T, 4] with F = 1; the state has one entry per (..., C) stream.
    """
    th = state.thresholds(params)
    th = {k: np.asarray(v)[..., None] for k, v in th.items()}   # broadcast over windows
    out = screen(vis, params, th)
    stats = np.stack([out["tau"], out["r_re"], out["r_im"]], axis=-1)
    state.update(stats, out["flags"] == 0)
    out["thresholds"] = {k: v[..., 0] for k, v in th.items()}
    return out
