"""bench.py host logic (no GPU): the --gpus guard and the counter-summary
gating, so a stored HBM-traffic figure is reported only for the kernel
sources, workload and tile order it was measured on."""
import argparse
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _args(**kw):
    a = argparse.Namespace(n_mol=256, tile_order="round-robin")
    for k, v in kw.items():
        setattr(a, k, v)
    return a


def _summary_hash():
    for line in open(bench.TRAFFIC_FILE):
        if line.strip().startswith("source_hash:"):
            return line.split(":", 1)[1].strip()
    raise AssertionError("no source_hash in the counter summary")


def test_stored_traffic_read_from_the_summary(monkeypatch):
    """the committed summary parses to a byte count for the sources it names"""
    monkeypatch.setattr(bench, "kernel_source_hash", _summary_hash)
    got = bench.stored_traffic(_args())
    assert got is not None and got > 0


def test_stored_traffic_only_for_its_workload_and_order():
    assert bench.stored_traffic(_args(n_mol=32)) is None
    assert bench.stored_traffic(_args(tile_order="alternating")) is None
    assert bench.stored_traffic(_args(tile_order="auto")) is None


def test_stored_traffic_ignored_after_a_source_change(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.stored_traffic(_args()) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env={**os.environ, "WORLD_SIZE": "1"})
    line = [x for x in r.stdout.splitlines() if x.startswith("{")][-1]
    d = json.loads(line)
    assert "error" in d and d["n_gpus"] == 2
