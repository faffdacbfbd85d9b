"""FP64 CPU oracle for the online energy + polarisation RFI screen.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU product path
never calls it and shares no code with it (no kernels, helpers, tables or
constants); the two meet only in the seeded input generator ``synth``, which
holds none of the method's arithmetic.

What it computes is the plain definition of the method in Section 2 of
Yatawatta, Boonstra & Broekema, "Energy and polarization based online
interference mitigation in radio interferometry" (arXiv 2412.14775):

* complex Stokes parameters of every 2x2 correlation (Section 2, eq. IQUV);
* the spectral-kurtosis statistic of |I| over a window (Section 2.1), with the
  epsilon guard of Table 1 (group 7);
* the directional statistic of the real and, separately, imaginary parts of
  (Q, U, V) (Section 2.2), with the epsilon of Table 2 (group 2);
* threshold tests combined by OR (end of Section 2.2), and the flag-masked
  time average with its weight (Section 2.1: flagged data are left out of the
  sum and the weight is updated);
* an extension the paper names as future work (Section 5): per-stream running
  estimates of each statistic's null mean and variance, merged after every
  integration with the pairwise update of Chan, Golub & LeVeque (1979), that
  set the next integration's thresholds.

Every function works in float64 on the exact input values.  Readings of the
paper where it is silent or ambiguous are listed in ``oracle.screen``.

Pins (checked in ``tests/test_oracle_pins.py``, marked "not gpu"): closed
forms of the SK estimator's mean and variance for Gamma-distributed inputs
(Nita & Gary 2010, cited in Section 2.1), hand-derived worked windows,
isotropic-null moments of the directional statistic, SU(2) invariance,
brute-force flag tables, library cross-checks of the averaging and of the
running mean/variance.  The adaptive-threshold extension's running state is
pinned against NumPy's mean/variance of the same windows and against the
closed-form null moments it must converge to (tau: mean 1 and the Nita & Gary
variance; r: E r^2 = 1/M for isotropic directions); its threshold rule
(mean -/+ kappa sigma) is a reading of the paper's future-work remark, which
gives no formula.
"""
from .mixed import mixed_window_stats, screen_mixed  # noqa: F401
from .screen import (  # noqa: F401
    SK_LOW, SK_HIGH, DS_RE, DS_IM, OPT_NO_SK, OPT_NO_DS, OPT_ADAPTIVE, OPT_PAPER_MIXED,
    Params, as_complex128, stokes, sk_tau, ds_r, flag_bits, window_view,
    screen, masked_average, AdaptiveState, screen_adaptive,
)
