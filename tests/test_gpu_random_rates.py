"""The device's random-access rates (sssp_device_random_rates), the reference
of the engine's random-access roofline in bench.py."""
import pytest

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2506_19349_amd as sssp  # noqa: E402

pytestmark = pytest.mark.gpu


def test_random_rates_are_measured():
    torch.cuda.set_device(0)
    r = sssp.device_random_rates()
    assert r["accesses"] == 1 << 24
    for k in ("rows64_per_s", "words8_small_per_s", "words8_large_per_s", "atomics8_small_per_s"):
        # anything real is above 10^8 random accesses per second and below the
        # HBM peak in 8-byte words (8 TB/s / 8 B)
        assert 1e8 < r[k] < 1e12, (k, r[k])
    # a 64-byte row moves eight times the bytes of an 8-byte word
    assert r["rows64_per_s"] <= r["words8_large_per_s"] * 1.5
