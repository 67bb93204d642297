"""Pins of the actuator-synthesis oracle (Sec. 4.2) against what the paper and the
mathematics fix, independently of the oracle's own routines:

* the rest angle it returns satisfies Eq. 1a, 1b, 1d (incomplete elliptic integrals from
  scipy, not the oracle's Carlson forms), Eq. 3a and the moment balance with Eq. 2's
  wrinkling moment evaluated from the printed formula;
* at a vanishing pressure the joint rests in the linear branch below the wrinkling onset,
  theta = 2 theta_on arm P G(0) / (pi P_vine R^3), with G(0) from an independent scipy
  solve of Eq. 1 at zero strain;
* the angle rises with the pressure and tends to the slack angle eps_max l / arm, the
  gap falling as 1/P (G vanishes linearly at the slack strain);
* the selection rule matches brute force over every (pressure, unit length) pair."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.special import ellipeinc, ellipkinc

import oracle as O
from oracle import synthesis as S

RC, RACT, A, EPSC = 0.005, 0.01718, 1e-4, 0.01
L, R, PV = 0.025, 0.03335, 10342.0  # the paper's segment, vine radius and pressure (1.5 psi)
ARM = 2 * R + RACT
MMAX = math.pi * PV * R ** 3


def h_printed(theta):
    """Eq. 2 as printed above the onset; the linear reading below it."""
    th_on = 2 * math.asin(EPSC)
    if theta <= th_on:
        return theta / (2 * th_on)
    g = math.acos(2 * EPSC / math.sin(theta / 2) - 1)
    return (math.sin(2 * g) + 2 * math.pi - 2 * g) / (4 * (math.sin(g) + (math.pi - g) * math.cos(g)))


def eq1_state(m, phi, l0):
    """(eps, G, l_a) of Eq. 1 at (m, phi) with scipy's integrals: unsaturated (l_a = l0)
    when phi is below phi_Rc, else saturated (l_a from Eq. 1b)."""
    c = math.cos(phi)
    F, E = ellipkinc(phi, m), ellipeinc(phi, m)
    phi_rc = math.acos(RC / RACT)
    la = l0 if phi < phi_rc - 1e-9 else RC * F / (math.sqrt(m) * c * (1 + A / (2 * m * c * c)))
    eps = (la - 2 * RC * (E - F / 2) / (math.sqrt(m) * c)) / l0
    G = math.pi * RC ** 2 * (1 - 2 * m) / (2 * m * c * c)
    return eps, G, la


@pytest.mark.parametrize("P,l0", [(2000.0, 0.02), (8000.0, 0.035), (14000.0, 0.05),
                                  (20000.0, 0.08)])
def test_rest_angle_satisfies_eq1_eq2_eq3(P, l0):
    theta, m, phi = S.free_angle(P, l0, L, R, PV)
    eps, G, la = eq1_state(m, phi, l0)
    c = math.cos(phi)
    if la == l0:  # unsaturated: Eq. 1b holds at phi
        lhs = ellipkinc(phi, m) / (math.sqrt(m) * c)
        assert abs(lhs - (l0 / RC) * (1 + A / (2 * m * c * c))) <= 1e-9 * lhs
    else:
        assert abs(phi - math.acos(RC / RACT)) <= 1e-12 and la <= l0 + 1e-12
    assert abs(theta - eps * L / ARM) <= 1e-12  # Eq. 3a
    assert 0 < theta < math.pi
    balance = MMAX * h_printed(theta) - ARM * P * G
    assert abs(balance) <= 1e-9 * ARM * P * G


def test_vanishing_pressure_rests_in_the_linear_branch():
    l0, P = 0.04, 1e-4
    # G(0): the state of zero strain, solved here with scipy (phi from Eq. 1b, m from eps = 0)
    phi_rc = math.acos(RC / RACT)

    def phi_of(m):
        f = lambda p: ellipkinc(p, m) * math.cos(p) / math.sqrt(m) - (l0 / RC) * (
            math.cos(p) ** 2 + A / (2 * m))
        grid = np.linspace(1e-9, phi_rc, 2001)
        v = [f(p) for p in grid]
        for i in range(len(grid) - 1):
            if v[i] < 0 <= v[i + 1]:
                return brentq(f, grid[i], grid[i + 1], xtol=1e-15)
        return phi_rc

    m0 = brentq(lambda m: eq1_state(m, phi_of(m), l0)[0], 1e-4, 0.5, xtol=1e-15)
    G0 = eq1_state(m0, phi_of(m0), l0)[1]
    theta_on = 2 * math.asin(EPSC)
    expect = 2 * theta_on * ARM * P * G0 / MMAX
    theta, _, _ = S.free_angle(P, l0, L, R, PV)
    assert theta < theta_on
    assert abs(theta - expect) <= 1e-6 * expect


def test_angle_rises_with_pressure_to_the_slack_angle():
    for l0 in (0.02, 0.05, 0.08):
        th = [S.free_angle(P, l0, L, R, PV)[0] for P in (1e3, 4e3, 1.6e4, 6.4e4)]
        assert all(b > a for a, b in zip(th, th[1:]))
        eps_max = O.spam_state(0.5, l0)[0]
        slack = eps_max * L / ARM
        assert th[-1] < slack
        # G vanishes linearly at the slack strain, so the gap to the slack angle falls as 1/P
        g10, g12 = (slack - S.free_angle(P, l0, L, R, PV)[0] for P in (1e10, 1e12))
        assert g10 > 0 and g12 > 0 and abs(g10 / g12 - 100.0) <= 0.1
        assert abs(S.free_angle(1e14, l0, L, R, PV)[0] - slack) <= 1e-9 * slack


def _brute(grid, Ps, Ls, t, tol):
    feas = [(Ps[k], abs(grid[k][j] - t), j, k) for k in range(len(Ps)) for j in range(len(Ls))
            if abs(grid[k][j] - t) <= tol]
    if not feas:
        return (0.0, 0.0, 0.0)
    Pbest = max(f[0] for f in feas)
    _, _, j, k = min((f for f in feas if f[0] == Pbest), key=lambda f: (f[1], f[2]))
    return (Ps[k], Ls[j], grid[k][j])


def test_selection_is_the_rule_over_every_pair():
    Ps = np.array([3000.0, 9000.0, 15000.0])
    Ls = np.array([0.02, 0.03, 0.045, 0.06, 0.08])
    grid = S.angle_grid(Ps, Ls, L, R, PV)
    rng = np.random.default_rng(3)
    targets = np.concatenate([grid.ravel(), rng.uniform(grid.min() * 0.8, grid.max() * 1.1, 40),
                              [1.0]])
    for tol in (0.0, math.radians(0.02), math.radians(0.1)):
        got = S.select(grid, Ps, Ls, targets, tol)
        for i, t in enumerate(targets):
            assert tuple(got[i]) == _brute(grid, Ps, Ls, t, tol), (i, t, tol)
    # an angle beyond every design: none; an exact grid angle at tol 0: that angle
    assert tuple(S.select(grid, Ps, Ls, [1.0], 0.1)[0]) == (0.0, 0.0, 0.0)
    k, j = 1, 2
    d = S.select(grid, Ps, Ls, [grid[k][j]], 0.0)[0]
    assert d[2] == grid[k][j] and d[0] >= Ps[k]


@pytest.mark.parametrize("eps,l0", [(0.05, 0.02), (0.2, 0.03), (0.1, 0.05), (0.15, 0.08),
                                    (0.0, 0.04)])
def test_inverse_state_reproduces_the_strain(eps, l0):
    """The state the inverse returns has the asked strain and force by Eq. 1 evaluated with
    scipy's elliptic integrals."""
    m, phi, G = S.spam_inverse(eps, l0)
    e2, G2, _ = eq1_state(m, phi, l0)
    assert abs(e2 - eps) <= 1e-12
    assert abs(G2 - G) <= 1e-12 * G
    # beyond the slack strain: the slack state
    m, phi, G = S.spam_inverse(5.0, l0)
    assert m == 0.5 and G == 0.0
