"""The streaming read probe (a measurement aid) on the device: a 1 GiB buffer,
larger than the on-package cache, is read at a positive rate no higher than
the published 8 TB/s peak, and repeated calls agree to within a factor."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_read_probe_rate_is_plausible():
    import torch

    import paper_2512_13133_amd as ca
    buf = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
    rates = []
    for _ in range(3):
        ms = ca.probe_read_bandwidth(buf, reps=5)
        assert ms > 0.0
        rates.append(buf.numel() * 4 / (ms * 1e-3) / 1e9)
    print(f"[probe] 1 GiB streaming read: {', '.join(f'{r:.0f}' for r in rates)} GB/s", flush=True)
    sys.stdout.flush()
    assert all(500.0 < r <= 8000.0 for r in rates)
    assert max(rates) < 2.0 * min(rates)
