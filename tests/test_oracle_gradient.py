"""Pins of the oracle's adjoint gradient (dL/d pressure, start, end of each sPAM)
against central finite differences of full oracle rollouts.

The adjoint differentiates each converged step's fixed point r(theta; p) = 0 of the
Eq. 4 energy; finite differences re-run the whole growth sequence, so a dropped
term, a wrong sign or a transposed Hessian in the adjoint shows up as a mismatch.
Parameters whose +-h rollouts change the contact set, or pass a bifurcation of the
equilibrium (a different number of steps along negative curvature), are excluded: the
loss is not differentiable there."""
import numpy as np
import pytest

import oracle as O
from paper_2509_15180_amd import workloads as W

from fdcheck import STEPS, cases_for, fd_values, losses, perturbed, smooth

ROBOTS = [1, 2, 3, 6]  # config-4 robots whose full rollouts take well under a second


@pytest.fixture(scope="module")
def base():
    w = W.config4(8).subset(ROBOTS)
    a = O.rollout(w, traj=True, threads=8)
    return w, a


@pytest.mark.parametrize("h_P,h_s,rtol", STEPS)
@pytest.mark.parametrize("weighted", [False, True])
def test_adjoint_matches_central_fd(base, weighted, h_P, h_s, rtol):
    w, a = base
    T = a["traj"].shape[1]
    weights = None
    if weighted:
        weights = np.zeros(T)
        weights[T // 3::7] = 0.5
        weights[-1] = 1.0
    dP, d0, d1, loss = O.gradient(w, a["traj"], weights=weights, threads=8)
    np.testing.assert_allclose(loss, losses(a["tip"], w.goal, weights), rtol=1e-12, atol=0)
    cases = cases_for(w, range(w.n_inst), h_P=h_P, h_s=h_s)
    wp = perturbed(w, cases)
    o = O.rollout(wp, threads=8)
    fd = fd_values(cases, losses(o["tip"], wp.goal, weights))
    ok = smooth(cases, o["chash"], a["chash"], o["stats"][:, 4], a["stats"][:, 4])
    grads = {"P": dP, "s0": d0, "s1": d1}
    adj = np.array([grads[c.name][c.spam] for c in cases])
    assert ok.sum() >= 10, "too few smooth cases to pin the adjoint"
    err = np.abs(adj - fd)[ok]
    scale = np.maximum(np.abs(fd[ok]), 1e-3 * np.abs(adj[ok]).max())
    # truncation and rounding: below 7e-4 relative at h = 1e-4 (SI), 7e-6 at 1e-5 m / 0.1 Pa
    assert (err / scale).max() < rtol, (adj[ok], fd[ok])
    # every name is exercised
    assert {c.name for c, k in zip(cases, ok) if k} == {"P", "s0", "s1"}


def test_gradient_is_linear_in_weights(base):
    w, a = base
    T = a["traj"].shape[1]
    wa, wb = np.zeros(T), np.zeros(T)
    wa[10], wa[40] = 1.0, 2.0
    wb[40], wb[-1] = 0.5, 1.0
    ga = O.gradient(w, a["traj"], weights=wa, threads=8)
    gb = O.gradient(w, a["traj"], weights=wb, threads=8)
    gs = O.gradient(w, a["traj"], weights=wa + wb, threads=8)
    for x, y, z in zip(ga, gb, gs):
        np.testing.assert_allclose(x + y, z, rtol=1e-10, atol=1e-14)


def test_shared_spam_records_sum():
    """Two robots that reference the same sPAM rows: the gradient is the sum of the
    two robots' gradients."""
    w = W.config4(8).subset([2])
    a = O.rollout(w, traj=True, threads=2)
    g1 = O.gradient(w, a["traj"], threads=2)
    w2 = W.pack([w.instance(0), w.instance(0)], "twice")
    w2.inst_i[1, 1] = w2.inst_i[0, 1]   # second robot points at the first one's sPAMs
    a2 = O.rollout(w2, traj=True, threads=2)
    g2 = O.gradient(w2, a2["traj"], threads=2)
    ns = int(w.inst_i[0, 2])
    for x, y in zip(g1[:3], g2[:3]):
        np.testing.assert_allclose(y[:ns], 2 * x[:ns], rtol=1e-12)
