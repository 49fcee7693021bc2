"""bench.py on the host: the one-GPU contract and the counter-record lookup
behind roofline.traffic (no GPU needed)."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_lookup(tmp_path, monkeypatch):
    # no record for other workloads or kernels: traffic is null
    assert bench.measured_traffic("grid4k", "atomic") is None
    assert bench.measured_traffic("rmat24", "plain") is None
    # a record is used only while the sources it names still hash to its value
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    h = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    rec = {"sources": ["k.hip"], "sources_sha256_16": h, "traffic_bytes_per_solve": 123.0}
    (prof / "toy_ahook_counters.md").write_text("text\n```json\n%s\n```\n" % json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("toy", "atomic") == 123.0
    src.write_text("kernel source, changed\n")
    assert bench.measured_traffic("toy", "atomic") is None
