"""Host logic of bench.py (CPU): the counted-traffic record is reported only
for the kernel source it was measured on, the oracle sample is spread over
the subdomain numbering, and more than one GPU is refused before any GPU
work."""
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def test_traffic_record_matches_current_source():
    key = ("k_solve<float, false>", "layered3d")
    assert key in bench.TRAFFIC
    v = bench.measured_traffic(*key)
    assert v == bench.TRAFFIC[key]["bytes_per_launch"] and v > 0


def test_traffic_record_dropped_when_source_changes(monkeypatch):
    key = ("k_solve<float, false>", "layered3d")
    rec = dict(bench.TRAFFIC[key])
    rec["src"] = "0" * 16
    monkeypatch.setitem(bench.TRAFFIC, key, rec)
    assert bench.measured_traffic(*key) is None
    assert bench.measured_traffic("k_unknown", "layered3d") is None


@pytest.mark.parametrize("n,k", [(1188, 12), (64, 8), (5, 12), (1, 1)])
def test_oracle_sample_spread(n, k):
    s = bench.sample_subdomains(n, k)
    assert s == sorted(set(s)) and len(s) == min(k, n)
    assert s[0] == 0 and s[-1] == n - 1 and all(0 <= v < n for v in s)
    assert bench.sample_subdomains(n, k) == s


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=str(ROOT))
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
