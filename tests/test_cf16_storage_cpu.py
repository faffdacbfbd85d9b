"""Complex-half storage error of the oracle itself at short windows (CPU, no GPU).

The workload states 3e-3 for complex-half storage against the FP64 oracle on the complex64
input.  That error is a property of the storage format: a kernel within 1e-5 of the oracle on
the same FP16 bytes (the arithmetic check every complex-half GPU test makes) has a total
error within 1e-5 of what the oracle itself shows between the FP16-rounded and the original
input.  For W = 2 the prefactor (W d + 1) / (W - 1) = 2 d + 1 amplifies the rounding of
|I| in tau past 3e-3, so no kernel can meet the bound there; for the other short windows of
the GPU tests (W = 3, 4, 8, 10) the oracle stays within it and the GPU tests assert 3e-3.
"""
from tests.cases import cf16_total_tolerance, exempt_shapes, storage_error
from tests.gpu_helpers import TOL_F16_TOTAL


def test_short_window_storage_error():
    errs = {}
    for label, vis, op in exempt_shapes():
        errs[label] = storage_error(vis, op)
        print(f"{label}: oracle on FP16-rounded vs complex64 input, max statistic error {errs[label]:.2e}")
    assert errs["M=2"] > TOL_F16_TOTAL                     # storage alone exceeds the bound
    for label in ("M=3", "M=4", "M=8", "M=10"):
        assert errs[label] < TOL_F16_TOTAL, label          # here the GPU must meet 3e-3


def test_total_tolerance_rule():
    for label, vis, op in exempt_shapes():
        tol = cf16_total_tolerance(vis, op)
        if label == "M=2":
            assert TOL_F16_TOTAL < tol < 1e-2
        else:
            assert tol == TOL_F16_TOTAL
