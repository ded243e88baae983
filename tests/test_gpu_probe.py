"""The integer VALU throughput probe: it runs, reports the lane operations it
launched, and its rate is a plausible fraction of the chip's VALU peak."""
import pytest

from tests.test_gpu_parity import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_12976_amd as sz
    assert torch.cuda.is_available()
    c = sz.Context(0)
    yield c
    c.close()


def test_valu_probe_rate(ctx):
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    wg, trips = 8 * cus, 2000
    log(f"[case] valu probe {wg} workgroups x {trips} trips")
    assert ctx.valu_probe(wg, trips) == wg * 256 * trips * 160  # warm-up; the count is exact
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    ops = ctx.valu_probe(wg, trips)
    end.record()
    torch.cuda.synchronize()
    rate = ops / (start.elapsed_time(end) * 1e-3)
    peak = cus * 64 * 2.4e9  # lane operations per second at 2.4 GHz (a wave64 instruction per 4 cycles per SIMD)
    log(f"[probe] {rate / 1e12:.2f} T lane-ops/s = {rate / peak:.3f} of {peak / 1e12:.2f} T")
    assert 0.5 * peak < rate < 1.2 * peak
    assert ctx.device_error() == 0
