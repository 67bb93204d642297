"""Actuator synthesis (Sec. 4.2) written out plainly on the oracle's sPAM model (Eq. 1,
``vo_spam_state``) and wrinkling law (Eq. 2, ``vo_wr_h``).  Test infrastructure, like the
rest of ``oracle``: only ``tests/`` may import it.

A joint whose link is covered by one sPAM of unit length l0 at pressure P rests in free
space (Sec. 3.3: the net moment of Eq. 3b vanishes) at the angle theta where the
wrinkling moment of Eq. 2 equals the actuator's moment,

    pi P_vine R^3 h(theta) = arm P G(eps; l0),   eps = arm theta / l  (Eq. 3a),
    arm = 2 R + R_act,   G = F_t / P  (Eq. 1d).

Along the sPAM's states m in [m0, 1/2] (m0: zero strain) the strain eps(m) rises from 0 to
its slack value and G(m) falls to 0, so the difference of the two sides rises from
-arm P G(m0) to pi P_vine R^3 h > 0: bisection on m finds the one root.

Synthesis, for a target angle: the highest pressure of the given set for which some unit
length of the given grid rests within tol of the target, and of those unit lengths the
one whose angle is nearest (the first of equal ones); (0, 0, 0) when no pressure does.
"""
from __future__ import annotations

import math

import numpy as np

from . import params, spam_state, wr_h


def zero_strain_m(l0: float, prm=None) -> float:
    """m0: the contraction parameter at which the strain of Eq. 1a vanishes."""
    a, b = 1e-6, 0.5
    for _ in range(200):
        if b - a <= 1e-17:
            break
        c = 0.5 * (a + b)
        if spam_state(c, l0, prm)[0] < 0.0:
            a = c
        else:
            b = c
    return 0.5 * (a + b)


def free_angle(P: float, l0: float, link_len: float, R: float, P_vine: float, prm=None):
    """(theta, m, phi): the free-space rest angle of a joint fully covered by one sPAM of
    unit length l0 at pressure P, and the sPAM's state there."""
    prm = params() if prm is None else prm
    R_act, eps_c = float(prm[1]), float(prm[3])
    arm = 2.0 * R + R_act
    M_max = math.pi * P_vine * R ** 3
    a, b = zero_strain_m(l0, prm), 0.5
    for _ in range(200):
        if b - a <= 1e-17:
            break
        c = 0.5 * (a + b)
        eps, G, _, _ = spam_state(c, l0, prm)
        q = M_max * wr_h(eps * link_len / arm, eps_c) - arm * P * G
        if q < 0.0:
            a = c
        else:
            b = c
    m = 0.5 * (a + b)
    eps, _, phi, _ = spam_state(m, l0, prm)
    return eps * link_len / arm, m, phi


def angle_grid(pressures, unit_lengths, link_len: float, R: float, P_vine: float, prm=None):
    """theta[k][j] = free_angle(pressures[k], unit_lengths[j], ...)."""
    return np.array([[free_angle(float(P), float(l0), link_len, R, P_vine, prm)[0]
                      for l0 in unit_lengths] for P in pressures])


def select(grid, pressures, unit_lengths, targets, tol: float):
    """The synthesis rule over a computed angle grid: rows are the pressures in rising
    order, columns the unit lengths; one (P, l0, theta) row per target."""
    out = np.zeros((len(targets), 3))
    for i, t in enumerate(targets):
        for k in range(len(pressures) - 1, -1, -1):
            best = -1
            for j in range(len(unit_lengths)):
                if best < 0 or abs(grid[k][j] - t) < abs(grid[k][best] - t):
                    best = j
            if abs(grid[k][best] - t) <= tol:
                out[i] = (pressures[k], unit_lengths[best], grid[k][best])
                break
    return out


def synthesize(targets, pressures, unit_lengths, tol: float, link_len: float, R: float,
               P_vine: float, prm=None):
    """(designs [n][3] = (P, l0, theta), angle grid)."""
    grid = angle_grid(pressures, unit_lengths, link_len, R, P_vine, prm)
    return select(grid, pressures, unit_lengths, targets, tol), grid


def spam_inverse(eps: float, l0: float, prm=None):
    """(m, phi, G): the sPAM state of strain eps (Eq. 1a inverted by bisection on m in
    [m0, 1/2], where the strain rises with m); the slack state (m = 1/2) at or beyond the
    slack strain, the state m0 at or below zero strain."""
    a = zero_strain_m(l0, prm)
    if eps >= spam_state(0.5, l0, prm)[0]:
        m = 0.5
    elif eps > 0.0:
        b = 0.5
        for _ in range(200):
            if b - a <= 1e-17:
                break
            c = 0.5 * (a + b)
            if spam_state(c, l0, prm)[0] < eps:
                a = c
            else:
                b = c
        m = 0.5 * (a + b)
    else:
        m = a
    _, G, phi, _ = spam_state(m, l0, prm)
    return m, phi, G
