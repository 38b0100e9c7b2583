"""Host logic of bench.py (CPU): the one-GPU refusal, the code hash that keys
the committed traffic counters, the percentile used for the latency, and the
pre-warm loop."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_code_only_ignores_comments_and_layout():
    a = "int f(int x) {  // first\n  return x + 1; /* block\n comment */ }\n"
    b = "int f(int x) { return x + 1; }"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(b.replace("1", "2"))


def test_source_hash_covers_every_part():
    # every marker of the hashed source parts is present, in order
    for name, start, end in bench.TRAFFIC_SOURCE_PARTS:
        with open(os.path.join(os.path.dirname(bench.KERNEL_SRC), name)) as f:
            text = f.read()
        i = text.index(start) if start else 0
        assert text.index(end, i) > i
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0


def test_traffic_is_null_once_the_source_changes(monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        recorded = json.load(f)
    monkeypatch.setattr(bench, "kernel_source_hash",
                        lambda: recorded["kernel_source_sha256_16"])
    assert bench.measured_traffic() == recorded["bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic() is None


@pytest.mark.parametrize("q,expected", [(0, 1.0), (50, 3.0), (100, 5.0), (99, 5.0)])
def test_percentile(q, expected):
    assert bench.percentile([5.0, 1.0, 4.0, 2.0, 3.0], q) == expected


def test_prewarm_repeats_the_work_for_its_duration(monkeypatch):
    """The pre-warm runs the work in groups of sync_every calls, one device
    synchronisation after each group, until its time has passed; 0 ms runs
    nothing."""
    torch = pytest.importorskip("torch")
    syncs = []
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: syncs.append(1))
    calls = []
    bench.prewarm(lambda: calls.append(1), 0.0, 4)
    assert calls == [] and syncs == []
    bench.prewarm(lambda: calls.append(1), 20.0, 4)
    assert len(calls) >= 4 and len(calls) == 4 * len(syncs)
