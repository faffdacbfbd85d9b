"""The paper's mixed-precision form of the screen (test infrastructure only).

Section 3 splits the two statistics into 14 groups of operations (Tables 1
and 2) and Section 4.1 (Tables 3 and 4) gives the precision a trained agent
chose per group, by the rule "action < 0.5: 32 bit, else 16 bit":

  SK  g1 y = xr^2 + xi^2 ....... 32     DS  g1 q^2, u^2, v^2 ......... 32
      g2 z = sqrt(y) ........... 32         g2 p = sqrt(.) + eps ...... 32
      g3 s1 = sum z ............ 32         g3 q/p, u/p, v/p ......... 32
      g4 s2 = sum y ............ 32         g4 sums of q^, u^, v^ .... 16
      g5 (Wd+1)/(W-1) .......... 32 (*)     g5 squares of the sums ... 16
      g6 s12 = s1^2 ............ 32         g6 r = sqrt(.)/W ......... 16
      g7 ratio, -1, x, compare . 16         g7 r > gamma ............. 16

(*) Table 3 labels g5 (action 0.497) as 16 bit although the stated rule gives
32 bit; the rule is followed here.

Emulation: every operation of a 16-bit group rounds its result to IEEE
binary16 (round to nearest even); its 32-bit inputs are converted to binary16
first (the conversions the paper's cost model counts).  32-bit groups compute
in float32.  Sums run sequentially in sample order, as written.  The 16-bit
epsilon of group 7 is the binary16 machine epsilon 2^-10 (Table 1: epsilon
depends on the number of bits).  The bracket of the SK statistic is that of
the Section 2.1 equation (reading R2 of ``oracle.screen``).

Parity pins: the emulated statistics stay within binary16 error bounds of the
float64 oracle, and an S2 beyond the binary16 range overflows to a NaN
statistic, which flags the window.
"""
from __future__ import annotations

import numpy as np

from .screen import Params, as_complex128, flag_bits, masked_average, window_view

EPS16 = float(np.finfo(np.float16).eps)      # 2^-10
f16 = np.float16
f32 = np.float32


def _seq_sum16(x):
    """Sequential binary16 sum over the last axis (each addition rounded to binary16)."""
    acc = np.zeros(x.shape[:-1], f16)
    with np.errstate(over="ignore", invalid="ignore"):
        for i in range(x.shape[-1]):
            acc = (acc + x[..., i].astype(f16)).astype(f16)
    return acc


def mixed_window_stats(win, d: float, eps32: float):
    """tau, r_re, r_im of windows [..., W, 4] in the paper's mixed precision."""
    v = as_complex128(win).astype(np.complex64)                  # float32 data stream
    xx, xy, yx, yy = v[..., 0], v[..., 1], v[..., 2], v[..., 3]
    I = xx + yy
    Q = xx - yy
    U = xy + yx
    V = (np.complex64(1j) * (xy - yx)).astype(np.complex64)
    W = win.shape[-2]
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        # SK groups 1-6 in float32, summed in order
        y = (I.real * I.real + I.imag * I.imag).astype(f32)
        z = np.sqrt(y).astype(f32)
        s1 = np.zeros(y.shape[:-1], f32)
        s2 = np.zeros(y.shape[:-1], f32)
        for i in range(W):
            s1 = (s1 + z[..., i]).astype(f32)
            s2 = (s2 + y[..., i]).astype(f32)
        pre = f32((W * float(d) + 1.0) / (W - 1.0))               # group 5: a 32-bit value (rule)
        s12 = (s1 * s1).astype(f32)                               # group 6
        # group 7 in binary16
        num = (f16(W) * s2.astype(f16)).astype(f16)
        den = (s12.astype(f16) + f16(EPS16)).astype(f16)
        ratio = (num / den).astype(f16)
        tau = (f16(pre) * (ratio - f16(1)).astype(f16)).astype(f16)

        def ds(q, u, w):
            q, u, w = q.astype(f32), u.astype(f32), w.astype(f32)
            p = (np.sqrt((q * q + u * u + w * w).astype(f32)) + f32(eps32)).astype(f32)   # groups 1-2
            qs = _seq_sum16((q / p).astype(f32))                                          # groups 3-4
            us = _seq_sum16((u / p).astype(f32))
            ws = _seq_sum16((w / p).astype(f32))
            sq = ((qs * qs).astype(f16) + (us * us).astype(f16)).astype(f16)               # group 5
            sq = (sq + (ws * ws).astype(f16)).astype(f16)
            return (np.sqrt(sq).astype(f16) / f16(W)).astype(f16)                          # group 6

        r_re = ds(Q.real, U.real, V.real)
        r_im = ds(Q.imag, U.imag, V.imag)
    return tau, r_re, r_im


def screen_mixed(vis, params: Params):
    """One integration in the paper's mixed precision; thresholds compared in binary16 (g7)."""
    p = params.f32()
    win = window_view(vis, p.M, p.F)
    tau, r_re, r_im = mixed_window_stats(win, p.d, p.eps)
    s_low, s_high, g = (float(f16(x)) for x in (p.s_low, p.s_high, p.gamma))
    flags = flag_bits(tau.astype(np.float64), r_re.astype(np.float64), r_im.astype(np.float64),
                      s_low, s_high, g, p.options)
    avg, weight = masked_average(vis, flags, p.M, p.F)
    return dict(tau=tau.astype(np.float64), r_re=r_re.astype(np.float64), r_im=r_im.astype(np.float64),
                flags=flags, avg=avg, weight=weight)
