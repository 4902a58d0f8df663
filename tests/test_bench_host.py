"""Host logic of bench.py, on the CPU: the traffic figures it takes from the
committed counter profiles (used only while the kernels' sources hash to
the recorded value, and only for a k that was profiled), and the refusal of
more than one GPU before anything touches a device."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _recorded_sha(path):
    m = re.search(r"sources_sha256:\s*([0-9a-f]{64})", open(path).read())
    assert m, path
    return m.group(1)


@pytest.mark.parametrize("k", [64, 256, 1024])
def test_scatter_traffic_is_read_for_the_recorded_sources(k):
    sha = _recorded_sha(bench.SCATTER_COUNTERS)
    v = bench.measured_traffic_per_element(bench.SCATTER_COUNTERS, sha, k)
    # one 128-byte line per lookup and the records: well above the 40
    # algorithmic bytes per entry, below ten lines
    assert v is not None and 40.0 < v < 1280.0


def test_traffic_is_withheld_for_other_sources_or_an_unprofiled_k():
    sha = _recorded_sha(bench.SCATTER_COUNTERS)
    other = ("0" if sha[0] != "0" else "1") + sha[1:]
    assert bench.measured_traffic_per_element(bench.SCATTER_COUNTERS, other, 64) is None
    assert bench.measured_traffic_per_element(bench.SCATTER_COUNTERS, sha, 128) is None
    assert bench.measured_traffic_per_element(os.path.join(ROOT, "profiles", "missing.md"), sha, 64) is None


def test_cd1_traffic_is_read_for_the_recorded_sources():
    sha = _recorded_sha(bench.CD1_COUNTERS)
    v = bench.measured_traffic_per_element(bench.CD1_COUNTERS, sha)
    assert v is not None and 40.0 < v < 1280.0


def test_sources_hash_is_stable_and_hex():
    a, b = bench.scatter_sources_sha256(), bench.scatter_sources_sha256()
    assert a == b and re.fullmatch(r"[0-9a-f]{64}", a)
    assert re.fullmatch(r"[0-9a-f]{64}", bench.cd1_sources_sha256())


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
