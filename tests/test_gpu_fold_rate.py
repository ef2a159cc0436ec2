"""Issue-rate calibration of the min-plus folds (apsp_measure_fold_rate),
the measured ceiling the bench reports beside the nominal VALU peak."""
import pytest

pytestmark = pytest.mark.gpu


def test_fold_rate_calibration(native, dev):
    """apsp_measure_fold_rate: the spin kernel's issue rate of each fold is
    positive and no faster than the device can issue (at most two 32-bit
    VALU lane-instructions per lane and cycle at 2.5 GHz), and the fold's
    terms follow from its instruction count (2 per 2 terms, 3 per 2 terms,
    2 per 4 terms)."""
    lanes_cap = 256 * 64 * 2.5e9 * 2
    per = {"int32": 1.0, "float32": 1.5, "packed16": 0.5}
    for fold, instr_per_term in per.items():
        r = native.apsp_measure_fold_rate(fold)
        assert 0 < r["lane_instr_per_s"] < lanes_cap, (fold, r)
        assert abs(r["lane_instr_per_s"] / r["terms_per_s"] - instr_per_term) < 1e-9, (fold, r)
    with pytest.raises(KeyError):
        native.apsp_measure_fold_rate("int8")
