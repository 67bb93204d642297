"""Write the oracle's outputs that the GPU parity tests compare against.

Calls only ``oracle/`` (the FP64 CPU oracle) on the seeded workloads of
``paper_2509_15180_amd.workloads``; nothing here comes from the HIP path.  Each file
records the SHA-256 of the oracle source and of the workload generator, and the tests
refuse a file whose hashes no longer match (regenerate with this script then).

  python tests/golden/make_oracle_outputs.py [--threads 7] [--only cfg2,...]

Files (numpy .npz, compressed):
  oracle_cfg1.npz   the one-robot workload, all 64 seeds, every step's joint angles
  oracle_cfg2.npz   the uniform batch, robots 0..1023 of the 4096
  oracle_cfg3.npz   the uneven batch: 1024 of its 16384 robots, 64 from each of the 16
                    strata of link count (16-64, 65-128, 129-192, 193-256) and obstacle
                    count (0-16, 17-32, 33-48, 49-64), the lowest indices in each, at
                    full length
  oracle_cfg5.npz   16 robots of the request stream with 257-512 links and 65-128
                    obstacles (the first environment sample of the first such requests),
                    their first 300 growth steps
  oracle_cfg5_full.npz  the first environment sample of requests 31 and 32 of the stream
                    (481 and 453 links among 125 and 126 obstacles) at full length
  oracle_cfg4_grad.npz  the differentiation batch, robots 0..511: final-step and
                    weighted-loss gradients with respect to every sPAM's pressure and ends

The uniform, uneven and differentiation files also hold the contact hashes of the same robots
with every body pressure scaled by 1 + 1e-14 (``perturbed_chash``): how often the
oracle's own descent changes its result under a rounding-size change of an input.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2509_15180_amd import workloads as W  # noqa: E402

SOURCES = ("oracle/vine_oracle.c", "oracle/__init__.py", "paper_2509_15180_amd/workloads.py")


def source_hash() -> str:
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cfg3_strata(work: W.Workload, per: int = 64) -> np.ndarray:
    n, K = work.inst_i[:, 0], work.inst_i[:, 4]
    idx = []
    for lo, hi in ((16, 64), (65, 128), (129, 192), (193, 256)):
        for klo, khi in ((0, 16), (17, 32), (33, 48), (49, 64)):
            cand = np.nonzero((n >= lo) & (n <= hi) & (K >= klo) & (K <= khi))[0]
            assert len(cand) >= per, (lo, hi, klo, khi, len(cand))
            idx += [int(i) for i in cand[:per]]
    return np.asarray(idx)


def cfg5_long(count: int = 16):
    items, rids = [], []
    j = 0
    while len(items) < count:
        r = W.config5_requests(1, start=j)[0]
        n, K = int(r.work.inst_i[0, 0]), int(r.work.inst_i[0, 4])
        if 257 <= n and 65 <= K:
            items.append(r.work.instance(0))
            rids.append(r.rid)
        j += 1
    return W.pack(items, "cfg5-long"), np.asarray(rids)


WEIGHTS4 = None


def weights_cfg4(T: int = 96) -> np.ndarray:
    w = np.zeros(T)
    w[T // 4::6] = 0.25
    w[-1] = 1.0
    return w


def pressure_perturbed(work: W.Workload, rel: float = 1e-14) -> W.Workload:
    w = W.pack([work.instance(i) for i in range(work.n_inst)], work.name + "[p]", dict(work.meta))
    w.inst_d[:, 2] *= 1.0 + rel
    return w


def save(name: str, **arrays):
    path = os.path.join(HERE, name)
    np.savez_compressed(path, source_sha256=np.array(source_hash()), **arrays)
    print(f"wrote {path} ({os.path.getsize(path) / 1e6:.2f} MB)", flush=True)


def rollout_arrays(work, out, steps):
    return dict(theta=out["theta"], tip=out["tip"][:, :steps, :2].astype(np.float32),
                tip_final=out["tip"][:, steps - 1], chash=out["chash"][:, :steps],
                status=out["status"][:, :steps].astype(np.int8),
                maxpen=out["maxpen"][:, :steps].astype(np.float32),
                ncont=out["ncont"][:, :steps].astype(np.int16),
                negsteps=out["stats"][:, 4], iters=out["stats"][:, 0])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=7)
    ap.add_argument("--only", default="cfg1,cfg2,cfg4,cfg5,cfg3,cfg5full")
    args = ap.parse_args()
    todo = args.only.split(",")
    th = args.threads
    if "cfg1" in todo:
        t = time.time()
        w = W.config1(64)
        out = O.rollout(w, traj=True, threads=th)
        save("oracle_cfg1.npz", idx=np.arange(64), traj=out["traj"],
             **rollout_arrays(w, out, 40))
        print(f"cfg1 {time.time() - t:.0f} s", flush=True)
    if "cfg2" in todo:
        t = time.time()
        w = W.config2(1024)
        out = O.rollout(w, threads=th)
        pert = O.rollout(pressure_perturbed(w), threads=th)
        save("oracle_cfg2.npz", idx=np.arange(1024), perturbed_chash=pert["chash"],
             **rollout_arrays(w, out, 64))
        print(f"cfg2 {time.time() - t:.0f} s", flush=True)
    if "cfg4" in todo:
        t = time.time()
        w = W.config4(512)
        out = O.rollout(w, traj=True, threads=th)
        pert = O.rollout(pressure_perturbed(w), threads=th)
        dP, d0, d1, loss = O.gradient(w, out["traj"], threads=th)
        wt = weights_cfg4()
        wP, w0, w1, wloss = O.gradient(w, out["traj"], weights=wt, threads=th)
        save("oracle_cfg4_grad.npz", idx=np.arange(512), weights=wt, chash=out["chash"],
             perturbed_chash=pert["chash"],
             status=out["status"].astype(np.int8), theta=out["theta"], negsteps=out["stats"][:, 4],
             dP=dP, ds0=d0, ds1=d1, loss=loss, wdP=wP, wds0=w0, wds1=w1, wloss=wloss)
        print(f"cfg4 {time.time() - t:.0f} s", flush=True)
    if "cfg5" in todo:
        t = time.time()
        w, rids = cfg5_long(16)
        out = O.rollout(w, n_steps=300, threads=th)
        save("oracle_cfg5.npz", rid=rids, **rollout_arrays(w, out, 300))
        print(f"cfg5 {time.time() - t:.0f} s", flush=True)
    if "cfg5full" in todo:
        t = time.time()
        rids = np.array([31, 32])
        reqs = {r.rid: r for r in W.config5_requests(33)}
        w = W.pack([reqs[int(i)].work.instance(0) for i in rids], "cfg5-full")
        out = O.rollout(w, threads=th)
        save("oracle_cfg5_full.npz", rid=rids, **rollout_arrays(w, out, int(w.n_max)))
        print(f"cfg5full {time.time() - t:.0f} s", flush=True)
    if "cfg3" in todo:
        t = time.time()
        full = W.config3(16384)
        idx = cfg3_strata(full)
        sub = full.subset(idx)
        out = O.rollout(sub, threads=th)
        pert = O.rollout(pressure_perturbed(sub), threads=th)
        save("oracle_cfg3.npz", idx=idx, perturbed_chash=pert["chash"],
             **rollout_arrays(sub, out, 256))
        print(f"cfg3 {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main()
