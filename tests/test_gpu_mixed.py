"""The paper's mixed-precision form (RFI_OPT_PAPER_MIXED) on the GPU against its emulation.

Tolerances: tau passes through identical binary16 operations on both sides, fed by FP32
sums S1, S2 that differ only in summation order; a one-ulp difference of their binary16
conversions is covered by the first-order binary16 bound of group 7 (tau_bound); the unit-vector sums are binary16 sums in a different order on the GPU (per lane,
then a butterfly) than in the emulation (sequential), bounded by the sequential-sum error
bound on both sides (r_bound); flags may differ only where a statistic is within those
tolerances of a threshold.  Masked averages are FP32 (conditional parity at 1e-5)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import avg_scale, make_params, run_gpu, to_device
from tests.test_oracle_mixed import U16, r_bound, tau_bound

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,F,T", [(10, 2, 400), (5, 4, 400), (20, 1, 400), (16, 1, 512), (16, 2, 512)])
def test_mixed_form_matches_its_emulation(M, F, T):
    from paper_2412_14775_amd import rfi
    env = synth.pulse_train(T, 60, 15, 5)
    sc = synth.Scene(3, 8, T, seed=M * F, rho=0.1, rfi=[synth.Rfi([1, 2, 5], 6.0, 0.4, 0.2, env, f0=0.1)])
    vis = synth.correlate(synth.make_voltages(sc))
    B, C = vis.shape[:2]
    W = M * F
    op, rp = make_params(B, C, T, M, "cf32", d=2.1, s_low=0.45, s_high=2.0, gamma=0.43, F=F,
                         options=oracle.OPT_PAPER_MIXED)
    plan = rfi.Plan(rp)
    gpu = run_gpu(plan, to_device(vis, "cf32"))
    plan.close()
    ref = oracle.screen_mixed(vis, op)
    # S1 and S2 are FP32 sums in different orders; their binary16 conversions can differ by
    # one ulp each, which moves tau by up to about pre * ratio * 2^-10: the first-order
    # binary16 bound of group 7 covers that
    tol_tau = tau_bound(np.where(np.isfinite(ref["tau"]), ref["tau"], 0.0), W, op.d)
    tol_r = 2 * r_bound(W)
    fin = np.isfinite(ref["tau"])
    assert np.array_equal(np.isfinite(gpu["tau"]), fin)
    assert np.all(np.abs(gpu["tau"][fin] - ref["tau"][fin]) <= tol_tau[fin])
    assert np.all(np.abs(gpu["r_re"] - ref["r_re"]) <= tol_r)
    assert np.all(np.abs(gpu["r_im"] - ref["r_im"]) <= tol_r)
    p32 = op.f32()
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
    print(f"{M}x{F}: mixed vs FP64 flag disagreement {(gpu['flags'] != ref64['flags']).mean():.4f}, "
          f"max |dtau| {np.abs(gpu['tau'][fin] - ref64['tau'][fin]).max():.2e}, "
          f"max |dr| {np.abs(gpu['r_re'] - ref64['r_re']).max():.2e}")
    assert (gpu["flags"] != ref64["flags"]).mean() < 0.01


def test_mixed_form_rejected_where_not_built():
    from paper_2412_14775_amd import rfi
    for kw in (dict(fmt="cf16", M=10, F=2), dict(fmt="cf32", M=100, F=1)):
        op, rp = make_params(3, 4, 400 if kw["M"] != 100 else 500, kw["M"], kw["fmt"], F=kw["F"],
                             options=oracle.OPT_PAPER_MIXED)
        with pytest.raises(rfi.RfiError) as ei:
            rfi.Plan(rp)
        assert ei.value.code == rfi.RFI_ERR_UNSUPPORTED
