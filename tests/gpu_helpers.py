"""Helpers for the GPU parity tests: run librfi through the binding, compare with the oracle.

Tolerances (relative error as |gpu - oracle| / max(1, |oracle|) for statistics; r lies in
[0, 1], so for r this is an absolute bound, and r is also held to the same tolerance as a true
relative error |gpu - oracle| / |oracle| wherever |oracle| >= R_FLOOR = 0.05: below that the
FP32 sum of W unit-vector components, whose error is about sqrt(W) 2^-24 per unit, cancels to
a total too small for a relative bound):
  complex64 storage, FP32 arithmetic ............ 1e-5
  complex-half storage vs oracle on the same
    (FP16-rounded) input: arithmetic error ....... 1e-5
  complex-half storage vs oracle on the original
    complex64 input: total error ................ 3e-3
Flags must be identical except for windows where an oracle statistic lies
within tol * max(1, |threshold|) of a threshold it is compared with; and they
must be bit-exact against the kernel's own statistics compared in float32.
Masked averages: error relative to the mean magnitude of the kept samples,
checked against the oracle average recomputed with the GPU's flags.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2412_14775_amd import rfi

TOL_F32 = 1e-5
TOL_F16_TOTAL = 3e-3
R_FLOOR = 0.05


def make_params(B, C, T, M, fmt="cf32", **kw):
    """Matching (oracle.Params, rfi_params) for one configuration."""
    N = int(round((np.sqrt(8 * B + 1) - 1) / 2))
    assert N * (N + 1) // 2 == B
    op = oracle.Params(M=M, **{k: v for k, v in kw.items() if k in oracle.Params.__dataclass_fields__})
    rp = rfi.rfi_params_default(
        n_stations=N, n_baselines=B, n_channels=C, n_samples=T, block_m=M,
        vis_format=rfi.RFI_VIS_CF16 if fmt == "cf16" else rfi.RFI_VIS_CF32,
        sk_d=op.d, sk_low=op.s_low, sk_high=op.s_high, ds_gamma=op.gamma, eps=op.eps,
        options=op.options, kappa_sk=op.kappa_sk, kappa_ds=op.kappa_ds, n_warm=op.n_warm,
        block_f=op.F)
    return op, rp


def to_device(vis, fmt):
    """complex64 [B,C,T,4] (or float16 pairs) -> torch tensor [B,C,T,4,2] on cuda:0."""
    import torch
    a = np.asarray(vis)
    if np.iscomplexobj(a):
        a = np.ascontiguousarray(a.astype(np.complex64)).view(np.float32).reshape(a.shape + (2,))
    a = a.astype(np.float16 if fmt == "cf16" else np.float32)
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def run_gpu(plan: "rfi.Plan", vis_dev, stats=True, flags=True):
    import torch
    out = plan.alloc_outputs(flags=flags, stats=stats)
    plan.screen(vis_dev, out["avg"], out["weight"], out["flags"], out["stats"])
    torch.cuda.synchronize()
    res = {}
    avg = out["avg"].cpu().numpy()
    res["avg"] = avg[..., 0].astype(np.float64) + 1j * avg[..., 1]
    res["weight"] = out["weight"].cpu().numpy()
    if flags:
        res["flags"] = out["flags"].cpu().numpy()
    if stats:
        st = out["stats"].cpu().numpy()
        res["stats32"] = st
        res["tau"], res["r_re"], res["r_im"] = (st[..., k].astype(np.float64) for k in range(3))
    return res


def stat_error(g, o):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    both_nan = np.isnan(g) & np.isnan(o)
    err = np.abs(g - o) / np.maximum(1.0, np.abs(o))
    return np.where(both_nan, 0.0, err)


def near_threshold(ref, th, tol):
    """Windows where any oracle statistic is within tol*max(1,|thr|) of its threshold."""
    def close(x, t):
        t = np.asarray(t, np.float64)
        return np.abs(x - t) <= tol * np.maximum(1.0, np.abs(t))
    return (close(ref["tau"], th["s_low"]) | close(ref["tau"], th["s_high"])
            | close(ref["r_re"], th["gamma"]) | close(ref["r_im"], th["gamma_im"]))


def flags_from_stats32(st32, th, options):
    """The flag rule evaluated in float32 on the kernel's own statistics."""
    tau, rre, rim = st32[..., 0], st32[..., 1], st32[..., 2]
    f = lambda v: np.asarray(v, np.float32)  # noqa: E731
    with np.errstate(invalid="ignore"):
        bits = (np.where(~(tau >= f(th["s_low"])), 1, 0) | np.where(tau > f(th["s_high"]), 2, 0)
                | np.where(~(rre <= f(th["gamma"])), 4, 0) | np.where(~(rim <= f(th["gamma_im"])), 8, 0))
    if options & oracle.OPT_NO_SK:
        bits &= ~3
    if options & oracle.OPT_NO_DS:
        bits &= ~12
    return bits.astype(np.uint8)


def avg_scale(vis, flags, M, F=1):
    """Mean magnitude of each correlation over the kept samples (the condition of the sum)."""
    v = oracle.as_complex128(vis)
    keep = np.repeat(np.repeat(np.asarray(flags) == 0, F, axis=-2), M, axis=-1)
    n = np.maximum(keep.sum(-1), 1)
    return np.where(keep[..., None], np.abs(v), 0.0).sum(-2) / n[..., None]


def compare(gpu, vis_for_oracle, op: "oracle.Params", tol, thresholds=None, ref=None, label=""):
    """Assert GPU results match the oracle on ``vis_for_oracle``; returns a report dict."""
    if ref is None:
        ref = oracle.screen(vis_for_oracle, op, thresholds)
    p32 = op.f32()
    th = dict(s_low=p32.s_low, s_high=p32.s_high, gamma=p32.gamma, gamma_im=p32.gamma)
    if thresholds:
        th.update(thresholds)
    rep = {}
    if "tau" in gpu:
        for k in ("tau", "r_re", "r_im"):
            e = stat_error(gpu[k], ref[k])
            rep[f"max_err_{k}"] = float(e.max()) if e.size else 0.0
            assert e.max(initial=0.0) <= tol, f"{label}: {k} max rel err {e.max():.3g} > {tol} at {np.unravel_index(np.argmax(e), e.shape)}"
            if k != "tau":
                o = np.asarray(ref[k], np.float64)
                big = np.abs(o) >= R_FLOOR
                rel = np.abs(np.asarray(gpu[k], np.float64)[big] - o[big]) / np.abs(o[big])
                rep[f"max_relerr_{k}"] = float(rel.max()) if rel.size else 0.0
                assert rel.max(initial=0.0) <= tol, f"{label}: {k} true relative error {rel.max():.3g} > {tol} (|r| >= {R_FLOOR})"
    if "flags" in gpu:
        thb = {k: (np.asarray(v)[..., None] if np.ndim(v) else v) for k, v in th.items()}
        near = near_threshold(ref, thb, tol)
        mism = (gpu["flags"] != ref["flags"])
        bad = mism & ~near
        rep["flag_mismatch"] = int(mism.sum())
        rep["flag_excused_frac"] = float(near.mean()) if near.size else 0.0
        rep["flagged_frac"] = float((ref["flags"] != 0).mean()) if near.size else 0.0
        assert not bad.any(), f"{label}: {int(bad.sum())} flag mismatches outside the excusal band, first at {np.argwhere(bad)[0]}"
        if "stats32" in gpu and not thresholds:
            own = flags_from_stats32(gpu["stats32"], thb, op.options)
            assert np.array_equal(own, gpu["flags"]), f"{label}: flags differ from the rule applied to the kernel's own statistics"
        # conditional parity of the average: the oracle average with the GPU's flags
        avg_c, w_c = oracle.masked_average(vis_for_oracle, gpu["flags"], op.M, op.F)
        scale = avg_scale(vis_for_oracle, gpu["flags"], op.M, op.F)
        e = np.abs(gpu["avg"] - avg_c) / np.maximum(scale, 1e-30)
        rep["max_err_avg"] = float(e.max()) if e.size else 0.0
        assert e.max(initial=0.0) <= tol, f"{label}: avg max rel err {e.max():.3g} > {tol}"
        np.testing.assert_allclose(gpu["weight"], w_c, rtol=1e-6, atol=0, err_msg=label)
    return rep
