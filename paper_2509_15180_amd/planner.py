"""Batched SST* design search (Sec. 5.2, Alg. 2) on top of the batched rollout.

A node of the search tree is a vine design grown to some length: its sPAMs (one per
edge that actuates), its link count and the pose of its tip in SE(2).  Each iteration
selects B nodes to expand, lowest estimated total cost first, samples for each an action
-- grow T more links, bending them with one sPAM on a sampled side at a sampled pressure,
or leave them passive -- and simulates all B children at once.  The children are pruned
against the tree within a radius r of the SE(2) metric, keeping the cheapest state of
each neighbourhood (the sparsity SST* maintains), and r decays on the schedule of Alg. 2.
The search stops when a node's tip reaches the goal region (the command line can keep
searching for a cheaper design); the design is the chain of actions from the root.

Readings (the paper leaves these open):

* Action.  The paper samples the actuator's strain and length and the step count T; here
  an action is (T, side, pressure): an sPAM spanning the T links the edge grows, on side
  +1 or -1 at a pressure drawn uniformly from the action range, or no sPAM (a passive
  segment) with a set probability.  The sPAM model turns pressure into bending moment.
* Propagation.  A child starts from its parent's joint angles and grows its T links
  (Alg. 2's T repetitions of Alg. 1).  Its new sPAM covers only the new links, so this is
  bitwise the state a rollout of the child's whole design from zero reaches (the search
  can also be run that way, ``resume=False``).
* Cost.  The number of sPAMs (the paper's actuator count) with the grown length as the
  tie-breaker: cost = sPAMs + length / max_length (the tie-breaker stays below 1).
* Cost-to-go.  The paper's reverse geometric RRT* tree (OMPL) is not built; the
  selection estimate is cost + w_goal * distance(tip, goal) / max_length.
* Metric.  The SE(2) distance combines millimetres and degrees: 1000 |dp| + (180/pi) |dpsi|,
  so the initial radius 60 is 60 mm at equal heading.
* Schedule.  next = i + sst_iter0 (1 + log2 j) alpha^(-(d + l + 1) j) with d = 3 (the
  state's SE(2) dimensions) and l = 2 (the action's actuation dimensions: side x
  pressure, and T), which the paper does not define.

The simulator is a function (designs, starting joint angles) -> (tip poses, worst step
statuses, final joint angles); ``GpuSimulator`` is the HIP path (libvinesim's server).
Run ``python -m paper_2509_15180_amd.planner`` for one search as a JSON line.
"""
from __future__ import annotations

import dataclasses
import json
import math
import sys
import time

import numpy as np

from . import workloads as W


@dataclasses.dataclass
class Problem:
    """A planning problem: the vine's body, the environment and the goal."""
    obstacles: np.ndarray          # [K][4] cx, cy, a, b (a circle's radius is a)
    kinds: np.ndarray              # [K] 0 circle, 1 rectangle (half sides a, b)
    goal: tuple                    # (x, y) in m
    goal_radius: float = 0.05      # m
    link_len: float = 0.02         # m
    tube_radius: float = 0.025     # m
    body_pressure: float = 4000.0  # Pa
    max_links: int = 120
    t_range: tuple = (4, 16)       # links grown per action
    p_range: tuple = (2000.0, 20000.0)  # sPAM pressure, Pa
    p_passive: float = 0.3         # probability of an action without an sPAM
    w_goal: float = 4.0            # weight of the distance-to-goal estimate

    @property
    def max_length(self) -> float:
        return self.max_links * self.link_len


@dataclasses.dataclass
class Node:
    parent: int
    n: int                 # links
    spams: list            # [(s_start, s_end, side, pressure)] of the whole design
    action: tuple          # (T, side, pressure) of the edge from the parent; side 0: passive
    tip: np.ndarray        # (x, y, heading)
    cost: float
    active: bool = True
    theta: np.ndarray = None  # joint angles of its n links (the state children start from)


def se2_distance(a, b) -> float:
    """Millimetres of position plus degrees of heading (wrapped to [-180, 180])."""
    dp = math.hypot(a[0] - b[0], a[1] - b[1])
    dpsi = (a[2] - b[2] + math.pi) % (2.0 * math.pi) - math.pi
    return 1000.0 * dp + math.degrees(abs(dpsi))



def design_instances(prob: Problem, designs) -> W.Workload:
    """One robot per design (n, spams) in the problem's environment; every robot refers to
    the same obstacle rows."""
    B = len(designs)
    n = np.fromiter((d[0] for d in designs), np.int32, B)
    cnt = np.fromiter((len(d[1]) for d in designs), np.int32, B)
    so = np.zeros(B, np.int32)
    if B:
        so[1:] = np.cumsum(cnt)[:-1]
    spam = np.array([row for _, sp in designs for row in sp], np.float64).reshape(-1, 4)
    K = len(prob.kinds)
    inst_i = np.column_stack([n, so, cnt, np.zeros(B, np.int32),
                              np.full(B, K, np.int32)]).astype(np.int32)
    inst_d = np.tile(np.array([prob.link_len, prob.tube_radius, prob.body_pressure, 0.0, 0.0,
                               0.0]), (B, 1))
    return W.Workload("plan", inst_i, inst_d, np.ascontiguousarray(spam),
                      np.ascontiguousarray(prob.kinds, np.int32),
                      np.ascontiguousarray(np.asarray(prob.obstacles, np.float64).reshape(-1, 4)),
                      np.zeros((B, 2)), {})


class GpuSimulator:
    """(designs, starts) -> (tip poses [B][3], worst step statuses [B], joint angles) on
    the HIP path: one vine server (libvinesim's continuous batching, device memory
    allocated once) kept for the whole search, each design queued as its own request,
    starting from the joint angles in starts (None: every design from zero).  ``clock``
    accumulates the seconds spent queueing, running and reading back."""

    def __init__(self, prob: Problem, batch: int, params=None, limit_s: float = 600.0):
        import torch

        from . import vinesim as V
        torch.cuda.set_device(0)
        self.prob = prob
        max_spams = min(V.MAX_SPAMS, prob.max_links // prob.t_range[0] + 1)
        self.srv = V.VineServer(slots=max(1, int(batch)), max_links=prob.max_links,
                                max_obstacles=max(1, len(prob.kinds)), max_spams=max_spams,
                                params=params)
        self.next_id = 0
        self.limit_s = limit_s  # per batch: raise rather than wait for ever
        self.clock = {"queue": 0.0, "run": 0.0, "read": 0.0}

    def __call__(self, designs, starts=None):
        t0 = time.perf_counter()
        first, m = self.next_id, len(designs)
        self.next_id += m
        self.srv.submit_each(first, design_instances(self.prob, designs), start=starts)
        t1 = time.perf_counter()
        status = np.zeros(m, np.int64)
        left = m
        while left:
            self.srv.tick()
            for rid, st in self.srv.poll(cap=m):
                status[rid - first] = st
                left -= 1
            if left and time.perf_counter() - t1 > self.limit_s:
                raise RuntimeError(f"{left} of {m} designs not done after {self.limit_s} s")
        t2 = time.perf_counter()
        tips, thetas = np.zeros((m, 3)), []
        for q in range(m):
            tips[q], th = self.srv.result(first + q, 0)
            thetas.append(th)
            self.srv.release(first + q)
        self.clock["queue"] += t1 - t0
        self.clock["run"] += t2 - t1
        self.clock["read"] += time.perf_counter() - t2
        return tips, status, thetas

    def close(self):
        self.srv.close()


class BatchedSST:
    """Alg. 2 with batch size B; ``simulate(designs, starts)`` maps designs (n, spams),
    each starting from the joint angles in starts (None: from zero), to their tip poses,
    worst step statuses and final joint angles."""

    def __init__(self, prob: Problem, simulate, batch: int, seed: int = 0,
                 r_init: float = 60.0, alpha: float = 0.8, sst_iter0: int = 7,
                 d: int = 3, l: int = 2, resume: bool = True):
        self.prob, self.sim, self.B, self.resume = prob, simulate, int(batch), resume
        self.rng = np.random.default_rng(seed)
        self.r, self.alpha, self.sst_iter0, self.d, self.l = r_init, alpha, sst_iter0, d, l
        self.i, self.j = 1, 1
        self.next_update = sst_iter0
        root = Node(parent=-1, n=1, spams=[], action=(1, 0, 0.0), tip=None,
                    cost=self.cost_of([], 1))
        tips, _, thetas = self.sim([(1, [])], None)
        root.tip, root.theta = np.asarray(tips[0], np.float64), np.asarray(thetas[0])
        self.nodes = []
        # per-node arrays for the neighbour searches (rows beyond len(nodes) unused)
        self._tip = np.zeros((64, 3))
        self._cost = np.zeros(64)
        self._active = np.zeros(64, bool)
        self._grow = np.zeros(64, bool)
        self._add(root)
        self.solution = -1
        self.grown_links = 1  # growth steps simulated
        self.rejected_status = 0

    # -- costs --------------------------------------------------------------------
    def cost_of(self, spams, n) -> float:
        return len(spams) + n * self.prob.link_len / self.prob.max_length

    def at_goal(self, tip) -> bool:
        g = self.prob.goal
        return math.hypot(tip[0] - g[0], tip[1] - g[1]) <= self.prob.goal_radius

    # -- one iteration of Alg. 2 --------------------------------------------------
    def _add(self, nd: Node) -> int:
        k = len(self.nodes)
        if k == len(self._cost):
            self._tip = np.concatenate([self._tip, np.zeros_like(self._tip)])
            self._cost = np.concatenate([self._cost, np.zeros_like(self._cost)])
            self._active = np.concatenate([self._active, np.zeros_like(self._active)])
            self._grow = np.concatenate([self._grow, np.zeros_like(self._grow)])
        self.nodes.append(nd)
        self._tip[k], self._cost[k], self._active[k] = nd.tip, nd.cost, nd.active
        self._grow[k] = nd.n + self.prob.t_range[0] <= self.prob.max_links
        return k

    def _deactivate(self, k: int):
        self.nodes[k].active = False
        self._active[k] = False

    def select(self):
        """B nodes to expand: the active nodes that can still grow, lowest estimated total
        cost first (ties: older node), repeated in that order when fewer than B."""
        m = len(self.nodes)
        cand = np.nonzero(self._active[:m] & self._grow[:m])[0]
        if not len(cand):
            return []
        g = self.prob.goal
        tips = self._tip[cand]
        est = self._cost[cand] + self.prob.w_goal * np.hypot(
            tips[:, 0] - g[0], tips[:, 1] - g[1]) / self.prob.max_length
        cand = cand[np.lexsort((cand, est))]
        return [int(cand[q % len(cand)]) for q in range(self.B)]

    def sample_actions(self, count):
        """(T, side, pressure) per expansion; side 0 is a passive segment."""
        t0, t1 = self.prob.t_range
        T = self.rng.integers(t0, t1 + 1, size=count)
        passive = self.rng.random(count) < self.prob.p_passive
        side = np.where(self.rng.random(count) < 0.5, 1, -1)
        p = self.rng.uniform(*self.prob.p_range, size=count)
        return [(int(T[q]), 0 if passive[q] else int(side[q]), 0.0 if passive[q] else float(p[q]))
                for q in range(count)]

    def prune_insert(self, children):
        """Children (in expansion order) against the tree: a child within r of an active
        node at most as costly is dropped; otherwise it is inserted and the active nodes
        within r that cost more are deactivated (their subtrees stay, as witnesses).
        Children are taken cheapest first (ties: expansion order).  Candidates come from
        k-d trees over the tip positions (a position farther than r is farther in the
        metric too), and every decision uses the metric itself."""
        from scipy.spatial import cKDTree
        added = []
        if not children:
            return added
        r = self.r
        reach = r * (1.0 + 1e-9) / 1000.0  # a superset of the metric's ball, in m
        ctip = np.array([ch.tip for ch in children], np.float64)
        ccost = np.array([ch.cost for ch in children])
        m = len(self.nodes)
        act = np.nonzero(self._active[:m])[0]
        near_e = (cKDTree(self._tip[act, :2]).query_ball_point(ctip[:, :2], reach)
                  if len(act) else [[] for _ in children])
        near_c = cKDTree(ctip[:, :2]).query_ball_point(ctip[:, :2], reach)
        within_e = self._within(near_e, ctip, self._tip[act], r)
        within_c = self._within(near_c, ctip, ctip, r)
        cost_e = self._cost[act].tolist()
        cost_c = ccost.tolist()
        alive = [True] * len(act)       # existing active nodes not yet deactivated
        node_of = [-1] * len(children)  # tree index of each inserted child, while active
        for q in sorted(range(len(children)), key=lambda q: (cost_c[q], q)):
            e = [k for k in within_e[q] if alive[k]]
            c = [k for k in within_c[q] if node_of[k] >= 0]
            if any(cost_e[k] <= cost_c[q] for k in e) or any(cost_c[k] <= cost_c[q] for k in c):
                continue
            for k in e:
                self._deactivate(int(act[k]))
                alive[k] = False
            for k in c:
                self._deactivate(node_of[k])
                node_of[k] = -1
            node_of[q] = self._add(children[q])
            added.append(node_of[q])
        return added

    @staticmethod
    def _within(cands, ctip, tips, r):
        """Per child q, the candidates of cands[q] within r of it in the metric (one
        vectorised evaluation over all candidate pairs)."""
        sizes = [len(c) for c in cands]
        if not sum(sizes):
            return [[] for _ in cands]
        q = np.repeat(np.arange(len(cands)), sizes)
        k = np.fromiter((v for c in cands for v in c), np.int64, sum(sizes))
        a, b = ctip[q], tips[k]
        dpsi = (b[:, 2] - a[:, 2] + math.pi) % (2.0 * math.pi) - math.pi
        ok = 1000.0 * np.hypot(b[:, 0] - a[:, 0], b[:, 1] - a[:, 1]) + np.degrees(np.abs(dpsi)) <= r
        out = [[] for _ in cands]
        for qq, kk in zip(q[ok].tolist(), k[ok].tolist()):
            out[qq].append(kk)
        return out

    def iterate(self):
        exp = self.select()
        if not exp:
            return []
        acts = self.sample_actions(len(exp))
        designs, children = [], []
        for k, (T, side, p) in zip(exp, acts):
            par = self.nodes[k]
            n = min(par.n + T, self.prob.max_links)
            spams = list(par.spams)
            if side != 0:
                spams.append((par.n * self.prob.link_len, n * self.prob.link_len, float(side), p))
            designs.append((n, spams))
            children.append(Node(parent=k, n=n, spams=spams, action=(n - par.n, side, p),
                                 tip=None, cost=self.cost_of(spams, n)))
        starts = [self.nodes[k].theta for k in exp] if self.resume else None
        tips, status, thetas = self.sim(designs, starts)
        self.grown_links += int(sum(ch.action[0] for ch in children)) if self.resume else \
            int(sum(n for n, _ in designs))
        valid = []
        for ch, tp, st, th in zip(children, tips, status, thetas):
            ch.tip, ch.theta = np.asarray(tp, np.float64), np.asarray(th)
            if st != 0:  # a step that did not converge: not a state of the model
                self.rejected_status += 1
                continue
            valid.append(ch)
        added = self.prune_insert(valid)
        for k in added:
            if self.at_goal(self.nodes[k].tip) and (
                    self.solution < 0 or self.nodes[k].cost < self.nodes[self.solution].cost):
                self.solution = k
        if self.i == self.next_update:
            self.r *= self.alpha
            self.j += 1
            self.next_update = self.i + int(round(
                self.sst_iter0 * (1.0 + math.log2(self.j))
                * self.alpha ** (-(self.d + self.l + 1) * self.j)))
        self.i += 1
        return added

    def run(self, max_iters: int):
        """Iterate until a node reaches the goal or max_iters; the solution node or -1."""
        while self.solution < 0 and self.i <= max_iters:
            if not self.iterate() and not self.select():
                break
        return self.solution

    def path(self, k: int):
        """Actions (T, side, pressure) from the root to node k."""
        acts = []
        while k > 0:
            acts.append(self.nodes[k].action)
            k = self.nodes[k].parent
        return acts[::-1]


def maze(seed: int = 0) -> Problem:
    """A synthetic maze: two walls across the way with offset gaps and a few circles; the
    goal behind the second wall (the paper's environments are not available)."""
    rng = np.random.default_rng(seed)
    obs, kinds = [], []
    # wall 1 at x = 0.5 with a gap around y = +0.15; wall 2 at x = 1.0 with a gap at y = -0.15
    for x, gap in ((0.5, 0.15 + rng.uniform(-0.03, 0.03)), (1.0, -0.15 + rng.uniform(-0.03, 0.03))):
        half_gap = 0.09
        lo_top, hi_bot = gap - half_gap, gap + half_gap
        obs.append((x, (lo_top - 0.6) / 2, 0.03, (lo_top + 0.6) / 2)); kinds.append(1)
        obs.append((x, (hi_bot + 0.6) / 2, 0.03, (0.6 - hi_bot) / 2)); kinds.append(1)
    for _ in range(3):
        obs.append((rng.uniform(0.65, 0.85), rng.uniform(-0.4, 0.4), rng.uniform(0.02, 0.05), 0.0))
        kinds.append(0)
    return Problem(obstacles=np.asarray(obs), kinds=np.asarray(kinds, np.int32),
                   goal=(1.35, -0.1), goal_radius=0.06)


def tube(seed: int = 0) -> Problem:
    """A channel 18 cm wide from x = 0.15 to 0.85 m, its exit partly closed by a block, and
    the goal up and to the side of the exit: the body must leave the channel and turn."""
    rng = np.random.default_rng(seed)
    obs = [(0.5, 0.12, 0.35, 0.03), (0.5, -0.12, 0.35, 0.03),
           (1.05, -0.05 + rng.uniform(-0.02, 0.02), 0.03, 0.15)]
    return Problem(obstacles=np.asarray(obs), kinds=np.ones(3, np.int32),
                   goal=(1.15, 0.3), goal_radius=0.06)


def gap(seed: int = 0) -> Problem:
    """A wall across the way at x = 0.6 m with one 12 cm gap off the axis, the goal behind
    it on the other side of the axis."""
    rng = np.random.default_rng(seed)
    g = 0.14 + rng.uniform(-0.02, 0.02)
    lo, hi = g - 0.06, g + 0.06
    obs = [(0.6, (lo - 0.7) / 2, 0.03, (lo + 0.7) / 2), (0.6, (hi + 0.7) / 2, 0.03, (0.7 - hi) / 2)]
    return Problem(obstacles=np.asarray(obs), kinds=np.ones(2, np.int32),
                   goal=(1.1, -0.1), goal_radius=0.06)


def pillars(seed: int = 0) -> Problem:
    """Ten circular pillars (radius 3-6 cm) scattered between x = 0.3 and 1.0 m, none
    closer than 0.2 m to the base; the goal straight ahead behind them."""
    rng = np.random.default_rng(seed)
    obs = []
    while len(obs) < 10:
        c = (rng.uniform(0.3, 1.0), rng.uniform(-0.35, 0.35), rng.uniform(0.03, 0.06), 0.0)
        if all(math.hypot(c[0] - o[0], c[1] - o[1]) > c[2] + o[2] + 0.07 for o in obs):
            obs.append(c)
    return Problem(obstacles=np.asarray(obs), kinds=np.zeros(10, np.int32),
                   goal=(1.25, 0.0), goal_radius=0.06)


ENVIRONMENTS = {"maze": maze, "tube": tube, "gap": gap, "pillars": pillars}


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--iters", type=int, default=40, help="iteration limit")
    ap.add_argument("--refine", type=int, default=0,
                    help="iterations to keep searching for a cheaper design after the first")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--env", choices=sorted(ENVIRONMENTS), default="maze")
    args = ap.parse_args(argv)
    prob = ENVIRONMENTS[args.env](args.seed)
    t0 = time.perf_counter()
    sim = GpuSimulator(prob, args.batch)
    pl = BatchedSST(prob, sim, args.batch, seed=args.seed)
    setup_s = time.perf_counter() - t0  # device set-up, the server and the root
    it_times, solve_s, first_cost, after = [], None, None, 0
    while pl.i <= args.iters and (pl.solution < 0 or after < args.refine):
        a = time.perf_counter()
        if not pl.iterate() and not pl.select():
            break
        it_times.append(time.perf_counter() - a)
        if pl.solution >= 0:
            if solve_s is None:
                solve_s, first_cost = time.perf_counter() - t0, pl.nodes[pl.solution].cost
            else:
                after += 1
    sol = pl.solution
    rec = {"environment": f"synthetic {args.env}", "iterations": pl.i - 1, "batch": args.batch,
           "nodes": len(pl.nodes), "solved": sol >= 0, "setup_s": setup_s, "solve_s": solve_s,
           "s_per_iteration": float(np.mean(it_times)) if it_times else None,
           "growth_steps": pl.grown_links, "wall_s": time.perf_counter() - t0,
           "radius_mm": pl.r, "rejected_nonconverged": pl.rejected_status,
           "sim_seconds": sim.clock}
    if sol >= 0:
        rec.update({"first_cost": first_cost, "best_cost": pl.nodes[sol].cost,
                    "sPAMs": len(pl.nodes[sol].spams), "links": pl.nodes[sol].n,
                    "path": pl.path(sol), "tip": [float(v) for v in pl.nodes[sol].tip]})
    sim.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    sys.exit(main())
