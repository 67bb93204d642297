"""Actuator synthesis (Sec. 4.2) on the GPU: for many wanted joint angles, the sPAM
(pressure, unit length) to build, by libvinesim's vine_spam_synth.

Run ``python -m paper_2509_15180_amd.synthesis`` for one measurement as a JSON line: the
paper's body (25 mm segments, 33.35 mm vine radius, 1.5 psi), pressures 2-20 kPa in 2 kPa
steps, unit lengths 20-80 mm on the 1 mm fabrication grid, a tolerance of 0.05 degrees,
and uniformly drawn targets of 0.2-4 degrees per joint.
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--targets", type=int, default=1 << 20)
    ap.add_argument("--tol-deg", type=float, default=0.05)
    ap.add_argument("--repeat", type=int, default=5)
    args = ap.parse_args(argv)
    import torch

    from . import vinesim as V
    torch.cuda.set_device(0)
    P = np.arange(2.0, 20.5, 2.0) * 1e3
    Lu = np.arange(20, 81) * 1e-3
    rng = np.random.default_rng(0)
    t = rng.uniform(math.radians(0.2), math.radians(4.0), args.targets)
    geo = (0.025, 0.03335, 10342.0)
    tol = math.radians(args.tol_deg)
    V.spam_synth(P, Lu, t[:16], tol, *geo)  # load and warm the kernels
    grid_s, all_s = [], []
    for _ in range(args.repeat):
        a = time.perf_counter()
        V.spam_synth(P, Lu, [], tol, *geo, want_angles=False)
        b = time.perf_counter()
        des, _ = V.spam_synth(P, Lu, t, tol, *geo, want_angles=False)
        c = time.perf_counter()
        grid_s.append(b - a)
        all_s.append(c - b)
    found = des[:, 0] > 0
    rec = {"study": "actuator synthesis", "targets": args.targets, "pressures": len(P),
           "unit_lengths": len(Lu), "tol_deg": args.tol_deg,
           "s_grid": float(np.median(grid_s)), "s_total": float(np.median(all_s)),
           "targets_per_s": args.targets / float(np.median(all_s)),
           "found": int(found.sum()),
           "pressure_histogram_kPa": {str(int(p / 1e3)): int((des[found, 0] == p).sum()) for p in P}}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
