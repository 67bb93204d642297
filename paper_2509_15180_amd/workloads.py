"""Seeded synthetic workloads for the vine-robot growth step.

This module only draws random inputs (robot descriptors, sPAM placements,
obstacle sets, goals, request streams).  It holds none of the model's
arithmetic, so both the FP64 oracle and the HIP path consume it.

Every instance ``i`` of workload ``cfg`` draws from its own generator
``PCG64(SeedSequence([250915180, cfg, i]))``, so the first ``B`` instances of
a large batch are the same robots as a batch of size ``B``.

Units are SI (m, Pa, rad).  The robot base sits at the origin and heads along
+x in every workload, so the straight initial body is exactly parallel or
perpendicular to every axis-aligned rectangle side; head-on contacts are then
exactly symmetric buckling points, which the solvers resolve by their
negative-curvature rule.

Layout of a :class:`Workload` (structure of arrays, host memory):

* ``inst_i``  int32  [B, 5]  n_target, spam_off, spam_cnt, obs_off, obs_cnt
* ``inst_d``  float64[B, 6]  link_len, tube_radius, body_pressure, base_x, base_y, base_heading
* ``spam``    float64[S, 4]  s_start, s_end (arc length from the base), side (+1/-1), pressure
* ``obs_kind`` int32 [O]     0 = circle, 1 = axis-aligned rectangle
* ``obs_d``   float64[O, 4]  cx, cy, a, b  (circle: a = radius, b = 0; rectangle: half-width, half-height)
* ``goal``    float64[B, 2]  goal point for the tip-to-goal loss (zeros when unused)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 250915180

CIRCLE = 0
RECT = 1


def instance_rng(cfg: int, i: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, cfg, i])))


@dataclass
class Workload:
    name: str
    inst_i: np.ndarray
    inst_d: np.ndarray
    spam: np.ndarray
    obs_kind: np.ndarray
    obs_d: np.ndarray
    goal: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_inst(self) -> int:
        return int(self.inst_i.shape[0])

    @property
    def n_max(self) -> int:
        return int(self.inst_i[:, 0].max()) if self.n_inst else 0

    @property
    def k_max(self) -> int:
        return int(self.inst_i[:, 4].max()) if self.n_inst else 0

    def joint_updates(self, n_steps: int | None = None) -> int:
        """Joints brought to equilibrium over a rollout: sum over steps of the link count."""
        n = self.inst_i[:, 0].astype(np.int64)
        if n_steps is not None and n_steps >= 0:
            n = np.minimum(n, n_steps)
        return int((n * (n + 1) // 2).sum())

    def subset(self, idx) -> "Workload":
        """Instances ``idx`` (in that order) with their sPAM and obstacle rows re-packed."""
        idx = np.asarray(idx, dtype=np.int64)
        return pack([self.instance(int(i)) for i in idx], self.name + "[sub]", dict(self.meta))

    def instance(self, i: int) -> dict:
        n, so, sc, oo, oc = (int(v) for v in self.inst_i[i])
        return dict(n=n, d=self.inst_d[i].copy(), spam=self.spam[so:so + sc].copy(),
                    kind=self.obs_kind[oo:oo + oc].copy(), obs=self.obs_d[oo:oo + oc].copy(),
                    goal=self.goal[i].copy())


def pack(items: list[dict], name: str, meta: dict | None = None) -> Workload:
    """Pack per-instance dicts (keys n, d, spam, kind, obs, goal) into a Workload."""
    B = len(items)
    inst_i = np.zeros((B, 5), np.int32)
    inst_d = np.zeros((B, 6), np.float64)
    goal = np.zeros((B, 2), np.float64)
    spams, kinds, obss = [], [], []
    so = oo = 0
    for b, it in enumerate(items):
        sp = np.asarray(it["spam"], np.float64).reshape(-1, 4)
        kd = np.asarray(it["kind"], np.int32).reshape(-1)
        ob = np.asarray(it["obs"], np.float64).reshape(-1, 4)
        inst_i[b] = (it["n"], so, len(sp), oo, len(kd))
        inst_d[b] = it["d"]
        goal[b] = it.get("goal", (0.0, 0.0))
        spams.append(sp)
        kinds.append(kd)
        obss.append(ob)
        so += len(sp)
        oo += len(kd)
    spam = np.concatenate(spams) if spams else np.zeros((0, 4))
    kind = np.concatenate(kinds) if kinds else np.zeros((0,), np.int32)
    obs = np.concatenate(obss) if obss else np.zeros((0, 4))
    return Workload(name, inst_i, inst_d, np.ascontiguousarray(spam, np.float64),
                    np.ascontiguousarray(kind, np.int32), np.ascontiguousarray(obs, np.float64),
                    goal, meta or {})


# ---------------------------------------------------------------------------
# obstacle sampling


def _meets_first_link(kind: int, cx: float, cy: float, a: float, b: float, l: float, R: float,
                      psi: float = 0.0) -> bool:
    """Conservative overlap test between an obstacle's bounding box and the
    bounding box of the first link's tube (the segment from the base to
    l (cos psi, sin psi), widened by R); rejection sampling keeps the base clear."""
    hx, hy = (a, a) if kind == CIRCLE else (a, b)
    ex, ey = l * np.cos(psi), l * np.sin(psi)
    x0, x1 = min(0.0, ex) - R, max(0.0, ex) + R
    y0, y1 = min(0.0, ey) - R, max(0.0, ey) + R
    return (cx + hx > x0) and (cx - hx < x1) and (cy + hy > y0) and (cy - hy < y1)


def _sample_obstacles(rng, n_circ: int, n_rect: int, box, r_rng, side_rng, l, R, psi=0.0):
    (x0, x1), (y0, y1) = box
    kinds, rows = [], []
    for kind, cnt in ((CIRCLE, n_circ), (RECT, n_rect)):
        for _ in range(cnt):
            for _attempt in range(1000):
                cx = rng.uniform(x0, x1)
                cy = rng.uniform(y0, y1)
                if kind == CIRCLE:
                    a = rng.uniform(*r_rng)
                    b = 0.0
                else:
                    a = 0.5 * rng.uniform(*side_rng)
                    b = 0.5 * rng.uniform(*side_rng)
                if not _meets_first_link(kind, cx, cy, a, b, l, R, psi):
                    break
            kinds.append(kind)
            rows.append((cx, cy, a, b))
    return np.asarray(kinds, np.int32), np.asarray(rows, np.float64).reshape(-1, 4)


def _sample_spams_links(rng, n: int, count: int, l: float, p_rng, span_rng=(4, 16)):
    """sPAMs over whole links: start link U{0..n-1}, span U{span_rng}, clipped at the tip."""
    rows = []
    for _ in range(count):
        start = int(rng.integers(0, n))
        span = int(rng.integers(span_rng[0], span_rng[1] + 1))
        end = min(start + span, n)
        side = 1.0 if rng.random() < 0.5 else -1.0
        p = rng.uniform(*p_rng)
        rows.append((start * l, end * l, side, p))
    return np.asarray(rows, np.float64).reshape(-1, 4)


# ---------------------------------------------------------------------------
# the five workloads


def config1(n_seeds: int = 64) -> Workload:
    """One FP64 robot per seed: 2.5 cm links, 5 cm tube, 3 kPa, 40 links; one sPAM on
    links 10..20 (side +, 5 kPa); 8 circles r ~ U[3, 8] cm in [0,1] x [-0.5,0.5] m."""
    items = []
    l, R = 0.025, 0.025
    for i in range(n_seeds):
        rng = instance_rng(1, i)
        kind, obs = _sample_obstacles(rng, 8, 0, ((0.0, 1.0), (-0.5, 0.5)), (0.03, 0.08), None, l, R)
        spam = np.asarray([(10 * l, 21 * l, 1.0, 5000.0)])
        items.append(dict(n=40, d=(l, R, 3000.0, 0.0, 0.0, 0.0), spam=spam, kind=kind, obs=obs))
    return pack(items, "cfg1", dict(cfg=1, n_seeds=n_seeds))


def config2(B: int = 4096, start: int = 0) -> Workload:
    """Uniform batch: 64 links of 2 cm, 5 cm tube, body pressure U[2,6] kPa, 0-4 sPAMs
    (span U{4..16} links, side +/-, U[0,20] kPa), 10 circles r ~ U[2,10] cm and 10
    rectangles with sides U[4,20] cm in a 1.5 x 1.5 m box ahead of the base."""
    items = []
    l, R = 0.02, 0.025
    for i in range(start, start + B):
        rng = instance_rng(2, i)
        psi = 0.0
        pv = rng.uniform(2000.0, 6000.0)
        spam = _sample_spams_links(rng, 64, int(rng.integers(0, 5)), l, (0.0, 20000.0))
        kind, obs = _sample_obstacles(rng, 10, 10, ((0.0, 1.5), (-0.75, 0.75)), (0.02, 0.10),
                                      (0.04, 0.20), l, R, psi)
        items.append(dict(n=64, d=(l, R, pv, 0.0, 0.0, psi), spam=spam, kind=kind, obs=obs))
    return pack(items, "cfg2", dict(cfg=2, start=start))


def config3(B: int = 16384, start: int = 0) -> Workload:
    """Uneven batch: link count U{16..256}, obstacle count U{0..64} (ceil(K/2) circles),
    0-6 sPAMs; otherwise as the uniform batch."""
    items = []
    l, R = 0.02, 0.025
    for i in range(start, start + B):
        rng = instance_rng(3, i)
        psi = 0.0
        n = int(rng.integers(16, 257))
        K = int(rng.integers(0, 65))
        pv = rng.uniform(2000.0, 6000.0)
        spam = _sample_spams_links(rng, n, int(rng.integers(0, 7)), l, (0.0, 20000.0))
        kind, obs = _sample_obstacles(rng, (K + 1) // 2, K // 2, ((0.0, 1.5), (-0.75, 0.75)),
                                      (0.02, 0.10), (0.04, 0.20), l, R, psi)
        items.append(dict(n=n, d=(l, R, pv, 0.0, 0.0, psi), spam=spam, kind=kind, obs=obs))
    return pack(items, "cfg3", dict(cfg=3, start=start))


def config4(B: int = 4096, start: int = 0) -> Workload:
    """Differentiation batch: 96 links, 12 circles + 12 rectangles, 1-4 sPAMs with
    continuous placement s_start ~ U[0, 92 l], span ~ U[4 l, 16 l]; goal ~ U(box)."""
    items = []
    l, R, n = 0.02, 0.025, 96
    for i in range(start, start + B):
        rng = instance_rng(4, i)
        psi = 0.0
        pv = rng.uniform(2000.0, 6000.0)
        rows = []
        for _ in range(int(rng.integers(1, 5))):
            s0 = rng.uniform(0.0, 92 * l)
            span = rng.uniform(4 * l, 16 * l)
            side = 1.0 if rng.random() < 0.5 else -1.0
            p = rng.uniform(0.0, 20000.0)
            rows.append((s0, min(s0 + span, n * l), side, p))
        kind, obs = _sample_obstacles(rng, 12, 12, ((0.0, 1.5), (-0.75, 0.75)), (0.02, 0.10),
                                      (0.04, 0.20), l, R, psi)
        goal = (rng.uniform(0.0, 1.5), rng.uniform(-0.75, 0.75))
        items.append(dict(n=n, d=(l, R, pv, 0.0, 0.0, psi), spam=np.asarray(rows), kind=kind,
                          obs=obs, goal=goal))
    return pack(items, "cfg4", dict(cfg=4, start=start))


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    work: Workload          # one instance per environment sample


def config5_requests(n_req: int, rate: float = 2000.0, start: int = 0,
                     n_max: int = 512, k_max: int = 128, s_max: int = 64) -> list[Request]:
    """Serving stream: Poisson arrivals at ``rate``/s.  Each request is one design
    (links U{16..n_max}, obstacles U{0..k_max}, 0-8 sPAMs) run on 1..s_max environment
    samples whose obstacle centres are jittered by N(0, (1 cm)^2)."""
    out = []
    t = 0.0
    gap_rng = instance_rng(5, 1 << 30)
    gaps = gap_rng.exponential(1.0 / rate, size=start + n_req)
    t = float(gaps[:start].sum())
    l, R = 0.02, 0.025
    for j in range(start, start + n_req):
        t += float(gaps[j])
        rng = instance_rng(5, j)
        psi = 0.0
        n = int(rng.integers(16, n_max + 1))
        K = int(rng.integers(0, k_max + 1))
        S = int(rng.integers(1, s_max + 1))
        pv = rng.uniform(2000.0, 6000.0)
        spam = _sample_spams_links(rng, n, int(rng.integers(0, 9)), l, (0.0, 20000.0))
        kind, obs = _sample_obstacles(rng, (K + 1) // 2, K // 2, ((0.0, 1.5), (-0.75, 0.75)),
                                      (0.02, 0.10), (0.04, 0.20), l, R, psi)
        items = []
        for s in range(S):
            o = obs.copy()
            if len(o):
                o[:, :2] += rng.normal(0.0, 0.01, size=(len(o), 2))
            items.append(dict(n=n, d=(l, R, pv, 0.0, 0.0, psi), spam=spam, kind=kind, obs=o))
        out.append(Request(j, t, pack(items, f"req{j}", dict(cfg=5, rid=j))))
    return out


# ---------------------------------------------------------------------------
# robustness and funnelling studies (Sec. 6 of the paper): one design in one
# environment, rolled out many times under perturbation


def study_rng(*keys: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 6, *keys])))


def perturbed(work: Workload, i: int, trials: int, sigma_env: float = 0.0,
              sigma_act: float = 0.0, tag: int = 0) -> Workload:
    """``trials`` copies of instance ``i`` with Gaussian perturbations (trial t draws
    from ``study_rng(i, tag, t)``):

    * environment, relative level ``sigma_env``: each obstacle centre moves by
      N(0, (sigma_env |c - base|)^2) per axis (an error proportional to its range from
      the base) and each size (radius, half-sides) is scaled by 1 + N(0, sigma_env^2),
      floored at 10 % of its nominal value; a draw that would meet the first link is
      redrawn (up to 100 times, else the obstacle keeps its nominal placement);
    * actuation, relative level ``sigma_act``: each sPAM's pressure and span length are
      scaled by 1 + N(0, sigma_act^2) (floored at 0 and at one tenth of the span), the
      start kept, the end clipped to the body.

    Level 0 reproduces the instance exactly."""
    base = work.instance(i)
    l, R = float(base["d"][0]), float(base["d"][1])
    bx, by, psi = (float(v) for v in base["d"][3:6])
    L_body = base["n"] * l
    items = []
    for t in range(trials):
        rng = study_rng(i, tag, t)
        obs = base["obs"].copy()
        for k in range(len(obs)):
            cx, cy, a, b = base["obs"][k]
            rng_k = np.hypot(cx - bx, cy - by)
            for _attempt in range(100):
                dc = rng.normal(0.0, 1.0, size=2) * sigma_env * rng_k
                fa, fb = 1.0 + sigma_env * rng.normal(0.0, 1.0, size=2)
                na = max(a * fa, 0.1 * a)
                nb = max(b * fb, 0.1 * b) if base["kind"][k] == RECT else 0.0
                if not _meets_first_link(int(base["kind"][k]), cx + dc[0] - bx, cy + dc[1] - by,
                                         na, nb, l, R, psi):
                    obs[k] = (cx + dc[0], cy + dc[1], na, nb)
                    break
        spam = base["spam"].copy()
        for j in range(len(spam)):
            s0, s1, side, p = base["spam"][j]
            fp, fs = 1.0 + sigma_act * rng.normal(0.0, 1.0, size=2)
            span = max((s1 - s0) * fs, 0.1 * (s1 - s0))
            spam[j] = (s0, min(s0 + span, L_body), side, max(p * fp, 0.0))
        items.append(dict(n=base["n"], d=base["d"].copy(), spam=spam, kind=base["kind"].copy(),
                          obs=obs, goal=base["goal"].copy()))
    return pack(items, f"{work.name}[{i}] perturbed", dict(instance=i, sigma_env=sigma_env,
                                                          sigma_act=sigma_act, tag=tag))


def start_angles(work: Workload, i: int, count: int, spread: float) -> Workload:
    """``count`` copies of instance ``i`` whose base headings are evenly spaced over
    [psi - spread/2, psi + spread/2] (psi the instance's own heading)."""
    base = work.instance(i)
    psi = float(base["d"][5])
    heads = psi + spread * (np.arange(count) / max(count - 1, 1) - 0.5)
    items = []
    for h in heads:
        d = base["d"].copy()
        d[5] = h
        items.append(dict(n=base["n"], d=d, spam=base["spam"].copy(), kind=base["kind"].copy(),
                          obs=base["obs"].copy(), goal=base["goal"].copy()))
    return pack(items, f"{work.name}[{i}] start angles", dict(instance=i, spread=spread))


def by_name(name: str, B: int | None = None) -> Workload:
    if name == "cfg1":
        return config1(B or 64)
    if name == "cfg2":
        return config2(B or 4096)
    if name == "cfg3":
        return config3(B or 16384)
    if name == "cfg4":
        return config4(B or 4096)
    raise KeyError(name)
