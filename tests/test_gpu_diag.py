"""Device micro-benchmarks behind the roofline figures: they run, return
finite positive rates, and order the instruction kinds as the shooting
kernel's design assumes (the reciprocal is the costly instruction)."""
import math

import pytest

import paper_2308_14278_amd.lensmap as lm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    lm.load()


def test_valu_peak_and_issue_rates():
    fma_tflops, pair_gpairs = lm.lm_measure_valu_peak()
    rates = lm.lm_measure_issue_rates()
    print("FMA %.1f TFLOP/s, pair mix %.3g pairs/s, %s" %
          (fma_tflops, pair_gpairs * 1e9, {k: "%.3g" % v for k, v in rates.items()}))
    assert 1.0 < fma_tflops < 400.0
    for v in rates.values():
        assert math.isfinite(v) and v > 0
    assert rates["v_rcp_f32"] < rates["v_mul_f32"]


def test_issue_rates_rejects_null():
    assert lm.load().lm_measure_issue_rates(None, 5) == lm.LM_EINVAL
