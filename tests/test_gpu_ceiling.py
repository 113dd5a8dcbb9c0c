"""GPU check of the copy-ceiling probe the benchmark reports beside the
roofline: it runs at the benchmark's size and at a small one, and returns a
rate below the published HBM peak (for sizes beyond the last-level cache)."""
import pytest

pytestmark = pytest.mark.gpu

esb = pytest.importorskip("paper_1611_02409_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def test_ceiling_probe_runs_and_is_below_peak():
    big = esb.stream_ceiling(4096 * 4096, 2)
    assert 1000.0 < big < 8000.0
    small = esb.stream_ceiling(1 << 16, 2)
    assert small > 0.0


@pytest.mark.parametrize("planes,sets", [(78, 2), (66, 2), (37, 1), (39, 1), (33, 1)])
def test_ceiling_probe_other_patterns(planes, sets):
    rate = esb.stream_ceiling(1 << 22, 2, planes=planes, sets=sets)
    assert 100.0 < rate < 20000.0
