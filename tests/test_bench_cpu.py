"""Host-side logic of bench.py (no GPU): the issue-bound model's closed form,
the recorded-traffic lookup and the one-GPU guard."""
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))
import bench  # noqa: E402


def _cycles(ms, n):
    return ms * 1e-3 * bench.SIMDS * bench.CLOCK_HZ / (n * n / 512.0)


@pytest.mark.parametrize("prec,k,valu,mfma", [
    ("f16x3", 17, 16, 4 + 3 + 2),    # merged last tile: 17 = 16 + 1 columns
    ("f16x3", 16, 16, 4 + 3),        # one full tile
    ("f16x3", 33, 16, 4 + 3 + 3 + 2),
    ("bf16x3", 17, 24, 4 + 3 + 3),   # BF16 split: no merged tile
    ("bf16x1", 17, 4, 4 + 1 + 1),
])
def test_issue_model_counts_per_512_entries(prec, k, valu, mfma):
    """d = 8: 6 d + 6 = 54 exponent slots, two 32-slot MFMAs per 16 x 16 tile,
    two j-tiles per 512 entries; 8 exp2 per lane."""
    n = 4096
    want = 8 * bench.ISSUE_EXP + valu * bench.ISSUE_VALU + mfma * bench.ISSUE_MFMA_HALF
    assert _cycles(bench.bf16_issue_model_ms(n, 8, k, prec), n) == pytest.approx(want, rel=1e-12)


def test_recorded_traffic_only_for_the_measured_configuration():
    class P:
        name, n = "block_fp32", 65536

        class B:
            shape = (65536, 17)
    assert bench._recorded_traffic(P, "f16x3") == pytest.approx((41858.1 * 2.0 + 34816.0) * 1024)
    assert bench._recorded_traffic(P, "bf16x3") is None
    P.n = 4096
    assert bench._recorded_traffic(P, "f16x3") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
