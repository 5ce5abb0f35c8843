"""Host-side logic of bench.py (CPU only): a profile's traffic record is
reported only while the hop's sources are the ones it was measured on and
only for the workload it was measured on, the multi-GPU request is refused
before any device work, and the D-slash case tags are unique."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADLINE = (32, 32, 32, 64)


def _record(tmp_path, monkeypatch, traffic):
    h = hashlib.sha256()
    for rel_path in bench.HOP_SOURCES:
        h.update(open(os.path.join(ROOT, rel_path), "rb").read())
    prof = tmp_path / "profile.md"
    prof.write_text("# profile\n\ntraffic_record: " + json.dumps(
        {"kernel": "k_hop", "traffic_bytes": traffic, "sources_sha256": h.hexdigest()}) + "\n")
    monkeypatch.setattr(bench, "PROFILE", str(prof))


def test_traffic_record_read_while_sources_match(tmp_path, monkeypatch):
    _record(tmp_path, monkeypatch, 386149790)
    assert bench.measured_traffic("f16", 12, HEADLINE) == 386149790


def test_traffic_record_dropped_when_sources_change(tmp_path, monkeypatch):
    _record(tmp_path, monkeypatch, 386149790)
    changed = []
    for rel_path in bench.HOP_SOURCES:
        data = open(os.path.join(ROOT, rel_path), "rb").read()
        p = tmp_path / os.path.basename(rel_path)
        p.write_bytes(data + (b"\n" if not changed else b""))
        changed.append(str(p))
    monkeypatch.setattr(bench, "HOP_SOURCES", tuple(changed))
    assert bench.measured_traffic("f16", 12, HEADLINE) is None


def test_traffic_record_only_for_its_workload(tmp_path, monkeypatch):
    _record(tmp_path, monkeypatch, 386149790)
    assert bench.measured_traffic("bf16", 12, HEADLINE) is None
    assert bench.measured_traffic("f16", 12, (24, 24, 24, 48)) is None


def test_multi_gpu_request_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr, (r.returncode, r.stderr)


def test_dslash_case_tags_unique():
    tags = [bench.dslash_tag(*c) for c in bench.DSLASH_CASES]
    assert len(tags) == len(set(tags))
    assert "32c64_f16_r12" in tags and "24c48_f32_r12_12rhs" in tags
