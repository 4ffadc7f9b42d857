"""bench.py's contract on a host without a GPU: one GPU only, and the counter record is used
only when it was taken on the sources the kernel is built from now."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_source_hash_covers_every_kernel_source(tmp_path, monkeypatch):
    assert all(os.path.exists(os.path.join(ROOT, p)) for p in bench.KERNEL_SOURCES)
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()
    # a copy of the tree with one source changed gives another hash
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(ROOT, rel), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h
    with open(tmp_path / bench.KERNEL_SOURCES[2], "ab") as f:
        f.write(b"\n")
    assert bench.kernel_source_hash() != h


def test_traffic_record_needs_the_current_sources(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    rec = {"w": {"kernel_sources_sha256_16": bench.kernel_source_hash(), "traffic_bytes_per_launch": 123},
           "old": {"kernel_sources_sha256_16": "0" * 16, "traffic_bytes_per_launch": 456}}
    (tmp_path / "profiles" / "pjds_spmv_traffic.json").write_text(json.dumps(rec))
    h = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.load_traffic("w") == 123
    assert bench.load_traffic("old") is None
    assert bench.load_traffic("absent") is None
