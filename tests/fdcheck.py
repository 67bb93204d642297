"""Central finite differences of the rollout loss with respect to sPAM parameters.

Shared by the oracle-gradient pins and the GPU gradient tests: it only builds
perturbed copies of a workload and combines losses; the rollouts themselves are
run by the caller (oracle or HIP library).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from paper_2509_15180_amd import workloads as W

COLS = {"P": 3, "s0": 0, "s1": 1}


@dataclass
class Case:
    robot: int      # instance index in the base workload
    spam: int       # global sPAM row in the base workload
    name: str       # "P", "s0" or "s1"
    h: float


# Finite-difference steps (h_P in Pa for pressures, h_s in m for sPAM ends, relative
# tolerance).  The first is the stated step, h = 1e-4 in SI units for every variable:
# central differences are second-order, and at 1e-4 m their truncation error in the
# placement derivatives is ~7e-4 relative on the differentiation batch, while 1e-4 Pa is
# near the rounding floor of the converged losses (~3e-4 relative).  The second pins the
# adjoint more tightly: 0.1 Pa and 1e-5 m (errors ~2e-7 and ~7e-6).
H_P, H_S = 1e-4, 1e-4
STEPS = [(1e-4, 1e-4, 2e-3), (0.1, 1e-5, 2e-5)]


def cases_for(work: W.Workload, robots, h_P: float = H_P, h_s: float = H_S) -> list[Case]:
    """Every sPAM parameter of ``robots`` whose loss is smooth within +-h: ends
    closer than 2h to a link boundary or the robot's end are left out (the joint
    coverage has a kink there)."""
    out = []
    for b in robots:
        n, so, sc = (int(v) for v in work.inst_i[b, :3])
        l = float(work.inst_d[b, 0])
        for s in range(so, so + sc):
            out.append(Case(b, s, "P", h_P))
            for name in ("s0", "s1"):
                x = float(work.spam[s, COLS[name]])
                k = np.round(x / l)
                if abs(x - k * l) < 2 * h_s or x > n * l - 2 * h_s or x < 2 * h_s:
                    continue
                if float(work.spam[s, 1] - work.spam[s, 0]) < 4 * h_s:
                    continue
                out.append(Case(b, s, name, h_s))
    return out


def perturbed(work: W.Workload, cases: list[Case]) -> W.Workload:
    """One instance per (case, sign): rows 2c (+h) and 2c + 1 (-h)."""
    items = []
    for c in cases:
        for sign in (1.0, -1.0):
            it = work.instance(c.robot)
            so = int(work.inst_i[c.robot, 1])
            it["spam"][c.spam - so, COLS[c.name]] += sign * c.h
            items.append(it)
    return W.pack(items, work.name + "[fd]", dict(work.meta))


def losses(tip: np.ndarray, goal: np.ndarray, weights=None) -> np.ndarray:
    """L_b = sum_t w_t |tip_b(t) - goal_b|^2 from the per-step tip records [B][T][3]
    (weights None: the last step only)."""
    e = ((tip[:, :, :2] - goal[:, None, :]) ** 2).sum(-1)
    if weights is None:
        return e[:, -1]
    return (e * np.asarray(weights)[None, :]).sum(1)


def fd_values(cases: list[Case], Lpm: np.ndarray) -> np.ndarray:
    return np.array([(Lpm[2 * i] - Lpm[2 * i + 1]) / (2 * c.h) for i, c in enumerate(cases)])


def smooth(cases: list[Case], chash_pm: np.ndarray, chash_base: np.ndarray,
           neg_pm=None, neg_base=None) -> np.ndarray:
    """True where neither perturbed rollout changed the contact set at any step and (when
    the counts are given) neither took a different number of steps along negative
    curvature than the base rollout: a changed count means the descent passed a
    bifurcation of the equilibrium within +-h, where the loss is not differentiable."""
    ok = []
    for i, c in enumerate(cases):
        same = bool((chash_pm[2 * i] == chash_base[c.robot]).all()
                    and (chash_pm[2 * i + 1] == chash_base[c.robot]).all())
        if neg_pm is not None:
            same = same and neg_pm[2 * i] == neg_base[c.robot] == neg_pm[2 * i + 1]
        ok.append(same)
    return np.array(ok)
