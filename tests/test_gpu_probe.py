"""The machine-balance probes that bench.py reports beside the datasheet
peaks (HBM 8 TB/s, FP64 78.6 TFLOP/s) return rates of the right order: a
plain copy and independent FP64 chains cannot beat the hardware's peaks by
more than timing noise, and on an MI355X they reach well above a tenth of
them."""
import pytest

import paper_2301_04869_amd as R

pytestmark = pytest.mark.gpu


def test_probe_peaks_are_plausible():
    pk = R.rkkt_probe_peaks()
    print(pk, flush=True)
    assert 800.0 < pk["hbm_gbs"] < 1.1 * 8000.0
    assert 7.86 < pk["fp64_vec_tfs"] < 1.1 * 78.6
    assert 7.86 < pk["fp64_mfma_tfs"] < 1.1 * 78.6
