"""Detection quality on synthetic RFI (Section 4.2): the paper's qualitative claims."""
import pytest

pytestmark = pytest.mark.gpu


def test_energy_and_polarisation_statistics_complement_each_other():
    from paper_2412_14775_amd.detection import detection_study, format_table
    study = detection_study(inrs_db=(-5, 0, 10, 20), realizations=3)
    print("\n" + format_table(study))
    print("calibration", study["calibration"])
    r = {(x["polarized"], x["inr_db"], x["method"]): x for x in study["rows"]}
    # polarised RFI: the directional statistic detects at lower INR than spectral kurtosis
    assert r[True, 0.0, "DS"]["pmd"] < r[True, 0.0, "SK"]["pmd"]
    # unpolarised RFI: the directional statistic is blind, spectral kurtosis is not
    assert r[False, 20.0, "DS"]["pmd"] > 0.5
    assert r[False, 20.0, "SK"]["pmd"] < r[False, 20.0, "DS"]["pmd"]
    for x in study["rows"]:
        assert x["pfa"] < 0.06
    for pol in (True, False):
        for inr in (-5.0, 0.0, 10.0, 20.0):
            both = r[pol, inr, "BOTH"]["pmd"]
            assert both <= min(r[pol, inr, "SK"]["pmd"], r[pol, inr, "DS"]["pmd"]) + 1e-12
        assert r[pol, 20.0, "BOTH"]["pmd"] < r[pol, -5.0, "BOTH"]["pmd"]


def test_post_correlation_rfi_model():
    """RFI added after correlation with a fixed coherency (the paper's simulation): polarised
    RFI is caught by the directional statistic better than by SK, unpolarised RFI only by SK."""
    from paper_2412_14775_amd.detection import detection_study, format_table
    study = detection_study(inrs_db=(-5, 0, 10, 20), realizations=3, model="post")
    print("\n" + format_table(study))
    r = {(x["polarized"], x["inr_db"], x["method"]): x for x in study["rows"]}
    for inr in (0.0, 10.0, 20.0):      # polarised RFI: DS misses less than SK (Fig. 3a)
        assert r[True, inr, "DS"]["pmd"] < r[True, inr, "SK"]["pmd"]
    assert r[False, 20.0, "DS"]["pmd"] > 0.5     # unpolarised RFI: DS is blind (Fig. 3b)
    assert r[False, 20.0, "SK"]["pmd"] < r[False, 20.0, "DS"]["pmd"]
    for pol in (True, False):
        for inr in (-5.0, 0.0, 10.0, 20.0):
            assert r[pol, inr, "BOTH"]["pmd"] <= min(r[pol, inr, "SK"]["pmd"], r[pol, inr, "DS"]["pmd"]) + 1e-12
    for x in study["rows"]:
        assert x["pfa"] < 0.06
