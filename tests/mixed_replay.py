"""The GPU kernel's summation order for the paper's mixed-precision form, replayed in NumPy.

Test infrastructure: a second, independent statement of what RFI_OPT_PAPER_MIXED computes,
used to check the kernel closely (the oracle, ``oracle.mixed``, sums in the paper's sample
order; the kernel sums K samples per lane and then a butterfly over the L lanes of a window,
so the two differ by binary16 rounding order only).  Per sample (Tables 3-4, groups 1-3 of
both statistics) float32; the unit-vector sums, their squares, r, and the SK ratio in
binary16; S1, S2 in float32 in the same tree order.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

F16, F32 = np.float16, np.float32
U16 = 2.0 ** -11                                   # unit roundoff of binary16


def lanes_for(M: int, F: int):
    """(K, S, L) of the windowed kernel: K samples per lane (2..8, dividing M, F S <= 64 with
    F S a power of two for this form; the largest such K), S = M / K lanes per channel,
    L = F S lanes per window."""
    for K in range(8, 1, -1):
        if M % K == 0:
            FS = F * (M // K)
            if FS <= 64 and FS & (FS - 1) == 0:
                return K, M // K, FS
    raise ValueError(f"no whole lane group for M={M}, F={F}")


def _tree(x, K, L, r16):
    """Sum over the last axis (W = K L terms, lane-major): K terms per lane in order, then a
    pairwise butterfly over the L lane sums; each addition rounded to binary16 if r16."""
    rnd = (lambda v: v.astype(F16).astype(F32)) if r16 else (lambda v: v.astype(F32))
    x = x.astype(F32).reshape(*x.shape[:-1], L, K)
    acc = rnd(x[..., 0])
    for k in range(1, K):
        acc = rnd(acc + x[..., k])
    while acc.shape[-1] > 1:
        acc = rnd(acc[..., 0::2] + acc[..., 1::2])
    return acc[..., 0]


def mixed_stats_tree(vis, M: int, F: int, d: float, eps: float):
    """tau, r_re, r_im [..., C/F, T/M] as the kernel orders the sums (float32 arrays)."""
    K, S, L = lanes_for(M, F)
    W = M * F
    win = oracle.window_view(vis, M, F).astype(np.complex64)     # [..., C/F, nW, F M, 4]
    xx, xy, yx, yy = (win[..., i] for i in range(4))
    f = lambda z: (z.real.astype(F32), z.imag.astype(F32))  # noqa: E731
    Ir, Ii = f(xx + yy)
    Qr, Qi = f(xx - yy)
    Ur, Ui = f(xy + yx)
    Vr = (yx.imag - xy.imag).astype(F32)               # V = j (xy - yx)
    Vi = (xy.real - yx.real).astype(F32)
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        y = (Ir * Ir + Ii * Ii).astype(F32)
        s1 = _tree(np.sqrt(y), K, L, False)
        s2 = _tree(y, K, L, False)
        r16 = lambda v: v.astype(F16).astype(F32)  # noqa: E731
        num = r16(r16(F32(W)) * r16(s2))
        den = r16(r16((s1 * s1).astype(F32)) + F32(2.0 ** -10))
        ratio = r16(num / den)
        pre = F32((W * float(d) + 1.0) / (W - 1.0))
        tau = r16(r16(pre) * r16(ratio - F32(1.0)))

        def ds(q, u, v):
            p = (np.sqrt((q * q + u * u + v * v).astype(F32)) + F32(eps)).astype(F32)
            qs, us, vs = (_tree(r16((c / p).astype(F32)), K, L, True) for c in (q, u, v))
            sq = r16(r16(qs * qs) + r16(us * us))
            sq = r16(sq + r16(vs * vs))
            return r16(r16(np.sqrt(sq)) / r16(F32(W)))

        return tau, ds(Qr, Ur, Vr), ds(Qi, Ui, Vi)


def sum_error_bound(W: int, K: int, L: int) -> float:
    """|binary16 tree sum - binary16 sequential sum| of W terms |t_i| <= 1: the sequential
    sum's rounding errors (partial i <= i in magnitude: u sum_{i=2}^{W} i), the tree's (K
    terms per lane, then log2 L levels whose sums stay below K 2^level), and one binary16
    ulp per term where the float32 terms of the two sides round to different binary16
    values."""
    seq = U16 * (W * (W + 1) / 2 - 1)
    tree = U16 * (L * (K * (K + 1) / 2 - 1) + W * math.log2(L))
    return seq + tree + 2 * U16 * W


def r_order_bound(W: int, K: int, L: int) -> float:
    """|r_tree - r_sequential|: r = |sums| / W is 1-Lipschitz in the 3-vector of sums over W,
    plus the binary16 roundings of groups 5-6 on each side (at most 8 u r <= 8 u each)."""
    return math.sqrt(3) * sum_error_bound(W, K, L) / W + 16 * U16
