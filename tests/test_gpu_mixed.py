"""The paper's mixed-precision form (RFI_OPT_PAPER_MIXED) on the GPU.

Three references, from the closest to the paper's own statement:
* tests/mixed_replay.py replays the kernel's order of the binary16 sums (K samples per lane,
  then a butterfly over the L lanes of a window): the kernel must give the same binary16
  values, up to one binary16 rounding of a per-sample term where the hardware reciprocal /
  square root and fused multiply-adds move a float32 term across a binary16 boundary
  (r within 2 binary16 ulps; tau within 1 ulp of its ratio, times the prefactor);
* the oracle (oracle/mixed.py) sums in the paper's sample order: r within the derived order
  bound r_order_bound(W, K, L) (test_mixed_replay_cpu.py pins it on the CPU); tau within the
  first-order binary16 bound of group 7 (tau_bound);
* every statistic the kernel writes is a binary16 value (an FP32 kernel would fail here).
Flags may differ from the oracle's only where a statistic is within those tolerances of a
threshold.  Masked averages are FP32 (conditional parity at 1e-5).  Against the FP64 oracle
the flag masks (flagged or not, the paper's measure) must differ in under 1 % of windows."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import avg_scale, make_params, run_gpu, to_device
from tests.mixed_replay import lanes_for, mixed_stats_tree, r_order_bound
from tests.test_oracle_mixed import tau_bound

pytestmark = pytest.mark.gpu


def _ulp16(x):
    """binary16 ulp at |x| (normal range; 2^-24 below it)."""
    x = np.abs(np.asarray(x, np.float64))
    e = np.floor(np.log2(np.maximum(x, 2.0 ** -14)))
    return 2.0 ** (e - 10)


@pytest.mark.parametrize("M,F,T", [(10, 2, 400), (5, 4, 400), (20, 1, 400), (16, 1, 512), (16, 2, 512)])
def test_mixed_form_matches_its_emulation(M, F, T):
    from paper_2412_14775_amd import rfi
    env = synth.pulse_train(T, 60, 15, 5)
    sc = synth.Scene(3, 8, T, seed=M * F, rho=0.1, rfi=[synth.Rfi([1, 2, 5], 6.0, 0.4, 0.2, env, f0=0.1)])
    vis = synth.correlate(synth.make_voltages(sc))
    B, C = vis.shape[:2]
    W = M * F
    K, S, L = lanes_for(M, F)
    op, rp = make_params(B, C, T, M, "cf32", d=2.1, s_low=0.45, s_high=2.0, gamma=0.43, F=F,
                         options=oracle.OPT_PAPER_MIXED)
    plan = rfi.Plan(rp)
    gpu = run_gpu(plan, to_device(vis, "cf32"))
    plan.close()
    st = gpu["stats32"]
    fin_all = np.isfinite(st)
    # binary16 values only
    assert np.array_equal(st[fin_all].astype(np.float16).astype(np.float32), st[fin_all])
    # the kernel's own order, replayed
    p32 = op.f32()
    t_tau, t_re, t_im = mixed_stats_tree(vis, M, F, p32.d, p32.eps)
    fin = np.isfinite(t_tau)
    assert np.array_equal(np.isfinite(gpu["tau"]), fin)
    for name, tr in (("r_re", t_re), ("r_im", t_im)):
        diff = np.abs(gpu[name] - tr.astype(np.float64))
        assert np.all(diff <= 2 * _ulp16(tr)), (name, diff.max())
        same = float(np.mean(diff == 0))
        print(f"{M}x{F} {name}: identical to the kernel-order replay in {same:.4f} of windows")
        assert same >= 0.8
    pre = (W * p32.d + 1) / (W - 1)
    ratio = t_tau[fin].astype(np.float64) / pre + 1
    assert np.all(np.abs(gpu["tau"][fin] - t_tau[fin]) <= pre * _ulp16(ratio) + _ulp16(t_tau[fin]))
    # the oracle's sequential order
    ref = oracle.screen_mixed(vis, op)
    fin = np.isfinite(ref["tau"])
    assert np.array_equal(np.isfinite(gpu["tau"]), fin)
    tol_tau = tau_bound(np.where(fin, ref["tau"], 0.0), W, op.d)
    tol_r = r_order_bound(W, K, L)
    assert np.all(np.abs(gpu["tau"][fin] - ref["tau"][fin]) <= tol_tau[fin])
    assert np.all(np.abs(gpu["r_re"] - ref["r_re"]) <= tol_r)
    assert np.all(np.abs(gpu["r_im"] - ref["r_im"]) <= tol_r)
    th = [float(np.float16(x)) for x in (p32.s_low, p32.s_high, p32.gamma)]
    near = ((np.abs(ref["tau"] - th[0]) <= tol_tau) | (np.abs(ref["tau"] - th[1]) <= tol_tau)
            | (np.abs(ref["r_re"] - th[2]) <= tol_r) | (np.abs(ref["r_im"] - th[2]) <= tol_r))
    bad = (gpu["flags"] != ref["flags"]) & ~near
    assert not bad.any(), np.argwhere(bad)[:5]
    avg_c, w_c = oracle.masked_average(vis, gpu["flags"], M, F)
    err = np.abs(gpu["avg"] - avg_c) / np.maximum(avg_scale(vis, gpu["flags"], M, F), 1e-30)
    assert err.max() <= 1e-5
    np.testing.assert_allclose(gpu["weight"], w_c, rtol=1e-6)
    # the paper: flags of the trained mixed form differ from 32-bit ones by under 1 %
    ref64 = oracle.screen(vis, op)
    mask = float(((gpu["flags"] != 0) != (ref64["flags"] != 0)).mean())
    bits = float((gpu["flags"] != ref64["flags"]).mean())
    print(f"{M}x{F}: mixed vs FP64 flag masks differ in {mask:.4f} of windows (flag bits {bits:.4f}), "
          f"max |dtau| {np.abs(gpu['tau'][fin] - ref64['tau'][fin]).max():.2e}, "
          f"max |dr| {np.abs(gpu['r_re'] - ref64['r_re']).max():.2e}")
    assert mask < 0.01


def test_mixed_form_rejected_where_not_built():
    from paper_2412_14775_amd import rfi
    for kw in (dict(fmt="cf16", M=10, F=2), dict(fmt="cf32", M=100, F=1)):
        op, rp = make_params(3, 4, 400 if kw["M"] != 100 else 500, kw["M"], kw["fmt"], F=kw["F"],
                             options=oracle.OPT_PAPER_MIXED)
        with pytest.raises(rfi.RfiError) as ei:
            rfi.Plan(rp)
        assert ei.value.code == rfi.RFI_ERR_UNSUPPORTED
