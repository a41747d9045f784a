"""Host logic of the benchmark driver: the recorded HBM traffic is reported
only while the kernel sources hash as they did when the counters were taken,
and a request for more than one GPU is refused before any device work."""
import os
import subprocess
import sys

import bench


def _write(path, sha, nbytes):
    with open(path, "w") as fh:
        fh.write("# summary\n\nsome text: not a key\n")
        fh.write(f"traffic_bytes_per_launch: {nbytes}\n")
        fh.write(f"kernel_sources_sha256: {sha}\n")


def test_traffic_reported_while_sources_match(tmp_path, monkeypatch):
    f = tmp_path / "traffic.md"
    _write(f, bench.kernel_source_hash(), 123456789.0)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic() == 123456789.0


def test_traffic_dropped_when_sources_changed(tmp_path, monkeypatch):
    f = tmp_path / "traffic.md"
    _write(f, "0" * 16, 123456789.0)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic() is None


def test_traffic_missing_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.md"))
    assert bench.recorded_traffic() is None


def test_source_hash_covers_every_kernel_source(tmp_path, monkeypatch):
    srcs = []
    for i in range(2):
        p = tmp_path / f"k{i}.hip"
        p.write_text(f"// source {i}\n")
        srcs.append(str(p))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", srcs)
    h0 = bench.kernel_source_hash()
    with open(srcs[1], "a") as fh:
        fh.write("// edited\n")
    assert bench.kernel_source_hash() != h0


def test_committed_summary_parses():
    # the committed summary carries both keys; the hash is 16 hex digits
    with open(bench.TRAFFIC_FILE) as fh:
        kv = dict(line.split(":", 1) for line in fh.read().splitlines()
                  if line.startswith(("traffic_bytes_per_launch:", "kernel_sources_sha256:")))
    assert float(kv["traffic_bytes_per_launch"]) > 0
    sha = kv["kernel_sources_sha256"].strip()
    assert len(sha) == 16 and int(sha, 16) >= 0


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
