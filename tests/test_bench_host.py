"""Host-side logic of bench.py (no GPU): the measured-counter record is reported only for
the workload it was taken on and only while the kernel sources are unchanged; the
accuracy summary compares the right things."""
import json
import os
import shutil

import numpy as np

import bench


def test_counters_follow_the_kernel_sources(tmp_path, monkeypatch):
    root = tmp_path
    for f in bench.KERNEL_SOURCES:
        os.makedirs(root / os.path.dirname(f), exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, f), root / f)
    monkeypatch.setattr(bench, "ROOT", str(root))
    os.makedirs(root / "profiles")
    rec = {"kernel_source_sha256": bench.kernel_hash(), "hbm_bytes_per_launch": 123.0,
           "fp64_flop_per_launch_from_counters": 1.0}
    json.dump(rec, open(root / "profiles" / "rollout_kernel_uneven_counters.json", "w"))
    assert bench.measured_counters("uneven")["hbm_bytes_per_launch"] == 123.0
    assert bench.measured_counters("uniform") is None  # taken on another workload
    with open(root / bench.KERNEL_SOURCES[0], "a") as fh:
        fh.write("\n// changed\n")
    assert bench.measured_counters("uneven") is None


def test_compare_counts_misses_and_tolerances():
    rng = np.random.default_rng(0)
    ref = {"theta": rng.normal(size=(5, 8)), "tip": rng.normal(size=(5, 8, 3)),
           "chash": rng.integers(0, 2**63, size=(5, 8), dtype=np.uint64)}
    got = {k: v.copy() for k, v in ref.items()}
    got["theta"][1, 3] += 2e-5          # out of the angle tolerance
    got["chash"][2, 7] ^= np.uint64(1)  # another contact set at the last step
    got["tip"][3, 0, 0] += 5e-5         # within the tip tolerance
    r = bench.compare(got, ref, 8)
    assert r["robots"] == 5 and r["identical_contact_sets"] == 4 and r["within_tolerance"] == 3
    assert abs(r["max_abs_dtheta_rad"] - 2e-5) < 1e-12


def test_quality_counts_converged_contact_states_only():
    status = np.array([[0, 0, 0, 2, -1]])
    out = {"ncont": np.array([[0, 3, 1, 4, 0]]),
           "maxpen": np.array([[0.0, 2e-3, 5e-4, 9e-3, 0.0]])}
    q = bench.quality(status, out)
    assert q["converged_steps"] == 3 and q["other_steps"] == 1
    assert q["converged_contact_states"] == 2 and q["fraction_within_1mm"] == 0.5
    assert q["max_penetration_m"] == 9e-3 and q["p50_penetration_m"] == 1.25e-3


def test_golden_hash_is_the_writers():
    import sys
    sys.path.insert(0, os.path.join(bench.ROOT, "tests", "golden"))
    import make_oracle_outputs as MK
    assert bench.golden_source_hash() == MK.source_hash()
