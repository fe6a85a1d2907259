"""The LDS bandwidth probe (the measured denominator of an LDS roofline) runs and reports a
bandwidth between the chip's CU count times a small per-CU rate and ten times its nominal peak."""
import pytest

from paper_2102_11089_amd import ldpc


@pytest.mark.gpu
@pytest.mark.parametrize("width", [4, 8, 16])
def test_lds_probe_reports_plausible_bandwidth(width):
    import torch
    print(f"lds probe width {width}", flush=True)
    gbs = ldpc.probe_lds(width, iters=256)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    nominal = cus * 128 * 2.4  # GB/s at 128 bytes per clock per CU
    assert 0.02 * nominal < gbs < 10 * nominal, gbs
