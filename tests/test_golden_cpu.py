"""The stored oracle outputs of the plain case (tests/golden/plain_case_oracle.npz, written by
tests/golden/make_golden.py from the oracle alone) still match the oracle: a change to the
oracle's arithmetic or to the generator shows up here."""
import numpy as np

from tests.golden.make_golden import OUT, PARAMS, compute


def test_oracle_reproduces_the_stored_plain_case():
    g = np.load(OUT)
    assert [float(x) for x in g["params"]] == [PARAMS[k] for k in ("M", "d", "s_low", "s_high", "gamma")]
    _, out = compute()
    for k in ("tau", "r_re", "r_im", "avg", "weight"):
        np.testing.assert_array_equal(out[k], g[k], err_msg=k)
    np.testing.assert_array_equal(out["flags"], g["flags"])
    assert 0.05 < (g["flags"] != 0).mean() < 0.5
