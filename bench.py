"""Benchmark of the batched growth step on one MI355X.

Default workload (the headline line): one bench step = one rollout of the whole batch
to full length, 4096 robots of 64 links (2 cm links, 5 cm tube, 0-4 sPAMs, 10 circles +
10 rectangles), i.e. 64 growth steps per robot and 4096 * 2080 = 8.52e6 joint-updates
(a joint brought to the converged equilibrium of one growth step).

Other workloads (``--workload``), same JSON fields:
  uneven  16384 robots of 16-256 links with 0-64 obstacles in one rollout call
  grad    4096 robots of 96 links: rollout with the trajectory recorded, then the
          adjoint of every step's equilibrium (vine_sim_grad, all steps weighted)
  serve   a Poisson stream of requests (one design of 16-512 links and 0-128 obstacles on
          1-64 environment samples each) through the continuous-batching server at
          ``--rate`` requests/s for ``--duration`` s after a warm-up; reports the
          sustained joint-updates/s and the p50/p99 request latency

Prints one JSON line with the driver's fields plus:
  roofline      the rollout kernel against the FP64 VALU peak (per-joint-evaluation
                FLOP count below), timed with HIP events on the stream the kernel is
                launched on; traffic (HBM bytes per launch) and the executed FP64 VALU
                work from the committed rocprofv3 counter summary, while the kernel
                sources are unchanged since it was taken (else null);
  per_instance  the same kernel launched once per robot (batch of one), serial on one
                stream, on a sample of the robots;
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload on the host
                cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "joint-updates/sec batched vs plain per-instance at 1e-5 rad; p99 rollout latency"
PEAK_FP64_TFLOPS = 78.6          # MI355X vector FP64 (256 CUs x 128 FLOP/clk x 2.4 GHz)


def flops_per_joint_eval(K: float) -> float:
    """Algorithmic FP64 operations of one joint's share of one residual+energy
    evaluation: pose scan 7, joint moment 150, joint energy 150, residual 18, and
    two body disks against K obstacles at 8.5 each (transcendentals count 1)."""
    return 325.0 + 17.0 * K


COUNTERS = os.path.join(ROOT, "profiles", "rollout_kernel_uniform_4096_counters.json")
KERNEL_SOURCES = ("paper_2509_15180_amd/csrc/vs_rollout.hip", "paper_2509_15180_amd/csrc/vs_device.h")


def measured_counters(workload: str, robots: int):
    """HBM bytes and FP64 instruction counts of one rollout launch, taken with rocprofv3
    PMC runs (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size; SQ_INSTS_*)
    and committed under profiles/.  Returned only for the workload they were taken on and
    while the kernel sources hash to what they were then; else None."""
    if workload != "uniform" or robots != 4096 or not os.path.exists(COUNTERS):
        return None
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    with open(COUNTERS) as fh:
        rec = json.load(fh)
    return rec if rec.get("kernel_source_sha256") == h.hexdigest() else None


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("uniform", "uneven", "grad", "serve"),
                    default="uniform")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=30.0, help="serve: measured seconds")
    ap.add_argument("--warm", type=float, default=5.0, help="serve: warm-up seconds")
    ap.add_argument("--slots", type=int, default=4096, help="serve: resident robots")
    ap.add_argument("--tick-steps", type=int, default=8, help="serve: growth steps per round")
    ap.add_argument("--batch", type=int, default=0, help="robots (default: the workload's)")
    ap.add_argument("--per-instance", type=int, default=8, help="robots in the per-instance sample")
    ap.add_argument("--cpu-robots", type=int, default=320, help="robots in the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="time the captured reset + rollout (vine_sim_rollout_graph)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the create-time launch order (no vine_sim_tune_order after the warm-up)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): robots are "
              f"independent, so several GPUs would each run their own share; not measured here.",
              flush=True)
        sys.exit(2)

    import torch

    from paper_2509_15180_amd import vinesim as V
    from paper_2509_15180_amd import workloads as W

    torch.cuda.set_device(0)
    wl = args.workload
    if wl == "serve":
        return serve(args, torch, V, W)
    if wl == "uniform":
        B = args.batch or 4096
        work = W.config2(B)
        desc = (f"uniform batch: {B} robots x 64 links (2 cm), 10 circles + 10 rectangles, "
                f"0-4 sPAMs; rollout to full length")
    elif wl == "uneven":
        B = args.batch or 16384
        work = W.config3(B)
        desc = (f"uneven batch: {B} robots x 16-256 links (2 cm), 0-64 obstacles, 0-6 sPAMs; "
                f"rollout to full length in one call")
    else:
        B = args.batch or 4096
        work = W.config4(B)
        desc = (f"differentiation batch: {B} robots x 96 links, 12 circles + 12 rectangles, "
                f"1-4 sPAMs, a goal each; rollout with trajectory + adjoint of every step")
    n = work.inst_i[:, 0].astype(np.float64)
    K_mean = float((work.inst_i[:, 4] * n * n).sum() / (n * n).sum())  # work-weighted obstacles
    ju = work.joint_updates()
    sim = V.VineSim(work)
    stream = torch.cuda.current_stream()
    T = sim.T
    weights = torch.ones(T, dtype=torch.float64, device="cuda") if wl == "grad" else None
    goal = torch.as_tensor(work.goal, dtype=torch.float64).cuda()

    def one_step():
        if args.graph:
            sim.rollout_graph(ckpt_every=32 if wl == "grad" else 0, stream=stream)
        else:
            sim.reset(stream=stream)
            sim.rollout(-1, ckpt_every=32 if wl == "grad" else 0, stream=stream)
        if wl == "grad":
            sim.grad(goal, weights, stream=stream)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    tuned = bool(args.warmup > 0 and not args.no_tune)
    if tuned:  # launch order from the cycles the warm-up rollout measured per robot
        sim.tune_order(stream=stream)
    ev0, ev1 = _events(torch)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        one_step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    out = sim.read_all()
    jevals = float(out["jevals"].sum())
    nsolves = float(out["nsolves"].sum())
    status = out["status"]
    # time of the rollout call alone (no reset), same stream
    sim.reset(stream=stream)
    k0, k1 = _events(torch)
    k0.record(stream)
    sim.rollout(-1, ckpt_every=32 if wl == "grad" else 0, stream=stream)
    k1.record(stream)
    torch.cuda.synchronize()
    kern_ms = k0.elapsed_time(k1)
    grad_ms = None
    if wl == "grad":
        g0, g1 = _events(torch)
        g0.record(stream)
        sim.grad(goal, weights, stream=stream)
        g1.record(stream)
        torch.cuda.synchronize()
        grad_ms = g0.elapsed_time(g1)
    flops = jevals * flops_per_joint_eval(K_mean)
    achieved = flops / (kern_ms * 1e-3) / 1e12
    value = ju / (ms * 1e-3)

    # plain per-instance form: one launch per robot, serial on one stream
    pi_idx = np.linspace(0, B - 1, args.per_instance).astype(int)
    sims = [V.VineSim(work.subset([i])) for i in pi_idx]
    for s in sims:
        s.rollout(-1, stream=stream)
    torch.cuda.synchronize()
    for s in sims:
        s.reset(stream=stream)
    p0, p1 = _events(torch)
    p0.record(stream)
    for s in sims:
        s.rollout(-1, stream=stream)
    p1.record(stream)
    torch.cuda.synchronize()
    pi_ms = p0.elapsed_time(p1)
    pi_ju = work.subset(pi_idx).joint_updates()
    pi_rate = pi_ju / (pi_ms * 1e-3)
    for s in sims:
        s.close()

    cpu = None
    if not args.no_cpu:
        import oracle as O
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        threads = max(1, min(int(threads), 16))
        idx = np.arange(min(args.cpu_robots, B)) if wl != "uneven" else \
            np.nonzero(work.inst_i[:, 0] <= 128)[0][:args.cpu_robots]
        sub = work.subset(idx)
        c0 = time.perf_counter()
        O.rollout(sub, threads=threads)
        csec = time.perf_counter() - c0
        cpu = {"value": sub.joint_updates() / csec, "unit": "joint-updates/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{len(idx)} robots of the same batch"
                         f"{' (those of <= 128 links)' if wl == 'uneven' else ''}, full rollouts "
                         f"({sub.joint_updates()} joint-updates in {csec:.1f} s)"}

    meas = measured_counters(wl, B)
    traffic = meas["hbm_bytes_per_launch"] if meas else None
    counters = None
    if meas:  # executed FP64 VALU work (wave instructions x 64 lanes, FMA = 2)
        cflop = meas["fp64_flop_per_launch_from_counters"]
        counters = {"fp64_flop_per_launch": cflop,
                    "achieved": cflop / (kern_ms * 1e-3) / 1e12,
                    "frac": cflop / (kern_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                    "source": os.path.relpath(COUNTERS, ROOT)}
    rec = {
        "metric": METRIC, "value": value, "unit": "joint-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "robots": B, "links_max": int(n.max()), "graph": bool(args.graph),
                   "schedule": "measured by the warm-up rollout" if tuned else "create-time estimate",
                   "obstacles_work_weighted": K_mean, "joint_updates_per_step": ju},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": "rollout_kernel", "kernel_ms": kern_ms,
                     "counters": counters,
                     "joint_evaluations": jevals,
                     "flop_per_joint_eval": flops_per_joint_eval(K_mean),
                     "linear_solves": nsolves},
        "per_instance": {"value": pi_rate, "unit": "joint-updates/s", "robots": int(len(pi_idx)),
                         "speedup_batched": value / pi_rate},
        "cpu_baseline": cpu,
        "quality": {"converged_steps": int((status == 0).sum()),
                    "other_steps": int(((status != 0) & (status != -1)).sum()),
                    "max_penetration_m": float(out["maxpen"].max())},
        "wall_s": wall,
    }
    if grad_ms is not None:
        rec["adjoint_ms"] = grad_ms
    print(json.dumps(rec), flush=True)


def serve(args, torch, V, W):
    """Open-loop stream: requests arrive on their Poisson clock whether or not the
    server keeps up; latency = completion - arrival."""
    horizon = args.warm + args.duration
    n_req = max(1, int(args.rate * horizon * 1.05) + 1)
    # requests are generated lazily in blocks (a saturated stream would otherwise build
    # far more than the server can take)
    block = 64
    gen = {"next": 0, "buf": []}

    def upcoming():
        if not gen["buf"] and gen["next"] < n_req:
            k = min(block, n_req - gen["next"])
            gen["buf"] = W.config5_requests(k, rate=args.rate, start=gen["next"])
            gen["next"] += k
        return gen["buf"][0] if gen["buf"] else None

    stream = torch.cuda.current_stream()
    srv = V.VineServer(slots=args.slots, max_links=512, max_obstacles=128, max_spams=8)
    arrival, size = {}, {}
    done_at = {}
    t0 = time.perf_counter()
    ju0 = None
    ticks = 0
    while True:
        now = time.perf_counter() - t0
        if now > horizon:
            break
        r = upcoming()
        while r is not None and r.arrival <= now:
            srv.submit(r.rid, r.work)
            arrival[r.rid] = r.arrival
            size[r.rid] = r.work.joint_updates()
            gen["buf"].pop(0)
            r = upcoming()
        st = srv.stats()
        if ju0 is None and now >= args.warm:
            ju0, tw = st["joint_updates"], now
        if st["active"] + st["queued"] == 0:
            if r is not None:
                time.sleep(max(0.0, min(r.arrival - now, 0.01)))
            continue
        srv.tick(args.tick_steps, stream=stream)
        ticks += 1
        t_done = time.perf_counter() - t0
        for rid, _ in srv.poll():
            done_at[rid] = t_done
            srv.release(rid)
    st = srv.stats()
    t_end = time.perf_counter() - t0
    ju_rate = (st["joint_updates"] - (ju0 or 0)) / max(t_end - (tw if ju0 is not None else 0.0), 1e-9)
    lat = np.array([done_at[i] - arrival[i] for i in done_at if arrival[i] >= args.warm])
    offered = float(np.mean(list(size.values()))) * args.rate if size else 0.0
    rec = {
        "metric": METRIC, "value": ju_rate, "unit": "joint-updates/s", "n_gpus": 1,
        "steps": ticks, "warmup": 0, "ms_per_step": 1e3 * t_end / max(ticks, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"request stream: Poisson {args.rate}/s, designs of 16-512 links and "
                               f"0-128 obstacles on 1-64 jittered environment samples; "
                               f"{args.slots} slots, {args.tick_steps} growth steps per round",
                   "rate_per_s": args.rate, "warmup_s": args.warm, "measured_s": args.duration},
        "serving": {"submitted": len(arrival), "completed": len(done_at),
                    "completed_after_warmup": int(lat.size),
                    "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
                    "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
                    "queued_at_end": st["queued"], "active_at_end": st["active"],
                    "offered_joint_updates_per_s": offered},
        "roofline": None, "cpu_baseline": None, "wall_s": t_end,
    }
    srv.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
