"""Host-side logic of bench.py (no GPU): the measured-counter record is reported only
for the workload it was taken on and only while the kernel sources are unchanged."""
import json
import os
import shutil

import bench


def test_counters_only_for_their_workload():
    assert bench.measured_counters("uneven", 4096) is None
    assert bench.measured_counters("uniform", 1024) is None


def test_counters_follow_the_kernel_sources(tmp_path, monkeypatch):
    root = tmp_path
    for f in bench.KERNEL_SOURCES:
        os.makedirs(root / os.path.dirname(f), exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, f), root / f)
    rec = json.load(open(bench.COUNTERS))
    rec_path = root / "counters.json"
    json.dump(rec, open(rec_path, "w"))
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "COUNTERS", str(rec_path))
    got = bench.measured_counters("uniform", 4096)
    if got is not None:  # the committed record matches the committed sources
        assert got["hbm_bytes_per_launch"] > 0
    with open(root / bench.KERNEL_SOURCES[0], "a") as fh:
        fh.write("\n// changed\n")
    assert bench.measured_counters("uniform", 4096) is None
