"""Host-side checks of bench.py (no GPU): the one-GPU contract, the row
repetition defaults and the link between the committed traffic counters and
the X-scan's source text."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""                   # no JSON line for a run that did not happen


def test_row_repetitions_default_and_floor(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert (a.rows_reps, a.rows_warmup) == (20, 5)
    assert (a.steps, a.warmup) == (3, 1)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--steps", "30", "--rows-reps", "4"])
    a = bench.parse()
    assert max(a.steps, a.rows_reps) == 30     # the rows never time fewer passes than --steps


def test_traffic_counters_follow_the_scan_source():
    sha = bench.kernel_sources_sha256()
    assert sha is not None, "an X-scan source marker moved: update XSCAN_SOURCES"
    rec = json.load(open(bench.TRAFFIC_FILE))
    if rec.get("source_sha256") == sha:
        for key in rec["kernels"]:
            assert bench.measured_traffic(key, 1 << 20, 4096) == round(rec["kernels"][key]["traffic_bytes"])
    else:
        # the scan changed since the counters were taken: the bench line must then carry no traffic figure
        assert bench.measured_traffic("f32", 1 << 20, 4096) is None
    assert bench.measured_traffic("f32", 1 << 19, 4096) is None     # other shapes never reuse the counters
