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
    # no record for other kernels: traffic is null
    assert bench.measured_traffic("rmat24", "plain") is None
    # a record is used only while the kernel and engine sources still hash to
    # its value, and only if it names exactly those sources
    for f in bench.COUNTER_SOURCES:
        p = tmp_path / f
        p.parent.mkdir(parents=True, exist_ok=True)
        p.write_text("source of %s\n" % f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"sources": list(bench.COUNTER_SOURCES), "sources_sha256_16": bench.sources_hash(),
           "traffic_bytes_per_solve": 123.0}
    (prof / "toy_ahook_counters.md").write_text("text\n```json\n%s\n```\n" % json.dumps(rec))
    assert bench.measured_traffic("toy", "atomic") == 123.0
    assert bench.measured_traffic("other", "atomic") is None
    # an edit to comments or blank lines keeps it
    eng = tmp_path / "paper_1612_01178_amd/csrc/engine.cpp"
    eng.write_text("source of %s  // a comment\n\n/* another\n one */\n" % bench.COUNTER_SOURCES[-1])
    assert bench.measured_traffic("toy", "atomic") == 123.0
    # a plan change in the engine makes the record stale
    eng.write_text("engine, changed\n")
    assert bench.measured_traffic("toy", "atomic") is None
    # a record that leaves the engine out is never used
    rec2 = dict(rec, sources=list(bench.COUNTER_SOURCES[:-1]), sources_sha256_16=bench.sources_hash())
    (prof / "toy_ahook_counters.md").write_text("text\n```json\n%s\n```\n" % json.dumps(rec2))
    assert bench.measured_traffic("toy", "atomic") is None
