"""Robustness and funnelling studies of one design (Sec. 6 of the paper), on top of the
batched rollout: every trial is one robot of a batch, rolled out on the GPU by
libvinesim in one launch per chain-length class.  This module only builds the batches
(through the seeded generators of ``workloads``) and reduces the tip positions the
library returns.

* Robustness: the success rate of reaching a goal region over many trials, as the
  Gaussian perturbation of the obstacles (positions and sizes) or of the actuation
  (sPAM pressures and lengths) grows.
* Funnelling: rollouts from evenly spread start headings; the dispersion of their
  end points is measured by the k-nearest-neighbour density concentration ratio the
  paper defines: with r_k(i) the mean distance from end point i to its k nearest
  neighbours, the density estimate is p_i = k / (pi r_k(i)^2), and the ratio is the
  mean of the p_i at or above their 90th percentile divided by the mean of all p_i
  (1 for evenly spread points; larger when the end points bunch up).

Run ``python -m paper_2509_15180_amd.robustness`` for one study as a JSON line.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

from . import workloads as W


def knn_density_ratio(points, k: int = 5, top: float = 0.10) -> float:
    """Density concentration ratio of 2-D points (see the module docstring); points
    at zero distance from their k neighbours are given the largest finite density of
    the set times 10 (an exact cluster), and the ratio is 1 when all distances vanish."""
    P = np.asarray(points, np.float64).reshape(-1, 2)
    m = len(P)
    if m <= k:
        raise ValueError(f"need more than k = {k} points, got {m}")
    d = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    rk = np.sort(d, axis=1)[:, :k].mean(axis=1)
    with np.errstate(divide="ignore"):
        p = k / (np.pi * rk * rk)
    finite = np.isfinite(p)
    if not finite.any():
        return 1.0
    p[~finite] = 10.0 * p[finite].max()
    cut = np.quantile(p, 1.0 - top)
    return float(p[p >= cut].mean() / p.mean())


def success_rate(tips, goal, radius: float) -> float:
    """Fraction of final tip positions within ``radius`` of ``goal``."""
    tips = np.asarray(tips, np.float64).reshape(-1, 2)
    return float((np.hypot(tips[:, 0] - goal[0], tips[:, 1] - goal[1]) <= radius).mean())


def final_tips(work, stream=None):
    """Roll every robot of ``work`` out to full length; final tip (x, y) per robot and
    the per-step statuses."""
    import torch

    from . import vinesim as V
    with V.VineSim(work) as sim:
        s = stream or torch.cuda.current_stream()
        sim.rollout(-1, stream=s)
        s.synchronize()
        tip = sim.read("tip")
        status = sim.read("status")
        n = work.inst_i[:, 0]
    return tip[np.arange(len(n)), n - 1, :2], status


def robustness_curve(work, i: int, levels, trials: int, which: str, radius: float,
                     goal=None):
    """Success rate per perturbation level (``which`` = 'env' or 'act'); the goal is the
    unperturbed design's final tip unless given."""
    if goal is None:
        goal = final_tips(work.subset([i]))[0][0]
    rates = []
    for li, lev in enumerate(levels):
        kw = dict(sigma_env=lev) if which == "env" else dict(sigma_act=lev)
        batch = W.perturbed(work, i, trials, tag=1000 * (which == "act") + li, **kw)
        tips, _ = final_tips(batch)
        rates.append(success_rate(tips, goal, radius))
    return np.asarray(goal), rates


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--instance", type=int, default=0, help="design of the uniform batch")
    ap.add_argument("--trials", type=int, default=1000)
    ap.add_argument("--radius", type=float, default=0.1, help="goal region radius (m)")
    ap.add_argument("--count", type=int, default=50, help="funnelling rollouts")
    ap.add_argument("--spread", type=float, default=np.deg2rad(20.0), help="start headings (rad)")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    work = W.config2(args.instance + 1)
    levels = [0.0, 0.02, 0.05, 0.1, 0.15, 0.2]
    t0 = time.perf_counter()
    goal, env = robustness_curve(work, args.instance, levels, args.trials, "env", args.radius)
    _, act = robustness_curve(work, args.instance, levels, args.trials, "act", args.radius, goal)
    t_rob = time.perf_counter() - t0
    fun = W.start_angles(work, args.instance, args.count, args.spread)
    ends, _ = final_tips(fun)
    free = W.start_angles(W.pack([dict(work.instance(args.instance), kind=np.zeros(0, np.int32),
                                       obs=np.zeros((0, 4)))], "free"), 0, args.count, args.spread)
    ends_free, _ = final_tips(free)
    rec = {"study": "robustness and funnelling of one design",
           "design": f"uniform batch instance {args.instance}", "trials_per_level": args.trials,
           "goal": goal.tolist(), "radius_m": args.radius, "levels": levels,
           "success_env": env, "success_act": act, "seconds_robustness": t_rob,
           "funnel_count": args.count, "funnel_spread_rad": args.spread,
           "density_ratio_obstacles": knn_density_ratio(ends),
           "density_ratio_free": knn_density_ratio(ends_free)}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
