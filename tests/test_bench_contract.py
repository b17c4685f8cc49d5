"""Host-side parts of the benchmark contract (no GPU needed): more than one
GPU is refused with a message, and the HBM traffic figure is reported only
while the committed counter record matches the kernel sources and the
launch variant the run uses."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1606_06508_amd import fh  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode != 0
    assert "one GPU" in p.stderr


def test_committed_traffic_record_is_current():
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    assert rec["src_sha256_16"] == bench._src_hash(bench.EVAL_SRC)
    # one launch: nine degrees of 10^6 points
    assert rec["variant"] == fh.tune_get("fp64", 1001, 9 * 10 ** 6)
    assert bench.measured_traffic(1001, 9 * 10 ** 6) == pytest.approx(rec["hbm_bytes_per_launch"])
    # algorithmic bytes per launch (nine degrees): per degree 8 B in, 16 B
    # out per point; the counters may add a little
    # per point and degree 8 B in and 16 B out; the octet variants also read
    # the sorted point's original position (4 B)
    per = 24e6 + (4e6 if fh.variant_octets("fp64", rec["variant"]) else 0)
    assert 9 * per <= rec["hbm_bytes_per_launch"] <= 1.1 * 9 * per


@pytest.mark.parametrize("change", ["variant", "source"])
def test_stale_traffic_record_gives_none(tmp_path, monkeypatch, change):
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    if change == "variant":
        rec["variant"] = rec["variant"] + 1
    else:
        rec["src_sha256_16"] = "0" * 16
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic(1001, 9 * 10 ** 6) is None


def test_host_cpu_fields():
    h = bench.host_cpu()
    assert set(h) == {"cpu_model", "host_logical_cpus", "host_physical_cores"}
    assert h["host_logical_cpus"] >= 1
