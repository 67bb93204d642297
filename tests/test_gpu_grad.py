"""GPU adjoint (vine_sim_grad) against the oracle's adjoint and against central
finite differences of GPU rollouts, on the differentiation workload (96 links,
12 circles + 12 rectangles, 1-4 sPAMs with continuous placement, a goal each).

Bars: where the GPU and oracle rollouts reach the same contact sets, the two
adjoints agree to 1e-6 relative (they solve the same linear system at states that
agree to ~1e-12 rad); the GPU adjoint matches central differences of GPU rollouts
to 2e-5 relative (truncation at h = 1e-5 m is below 4e-6)."""
import numpy as np
import pytest

import oracle as O
from paper_2509_15180_amd import workloads as W

from fdcheck import STEPS, cases_for, fd_values, losses, perturbed, smooth

pytestmark = pytest.mark.gpu

ROBOTS = [1, 2, 3, 6, 9, 10, 11, 12]


def _sim(work):
    import torch

    from paper_2509_15180_amd import vinesim as V
    torch.cuda.set_device(0)
    return V.VineSim(work)


def _gpu(work, weights=None, traj=True, ckpt=0):
    import torch
    with _sim(work) as sim:
        s = torch.cuda.current_stream()
        sim.rollout(-1, record_every=1 if traj else 0, ckpt_every=ckpt, stream=s)
        g = sim.grad(work.goal, weights, stream=s)
        s.synchronize()
        out = sim.read_all()
        return out, tuple(x.cpu().numpy() for x in g)


def _rel(a, b, floor):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


@pytest.mark.parametrize("weighted", [False, True])
def test_grad_matches_oracle(weighted):
    w = W.config4(16).subset(ROBOTS)
    T = 96
    weights = None
    if weighted:
        weights = np.zeros(T)
        weights[20::9] = 0.25
        weights[-1] = 1.0
    out, (dP, d0, d1, loss, st) = _gpu(w, weights)
    ref = O.rollout(w, traj=True, threads=16)
    rP, r0, r1, rloss = O.gradient(w, ref["traj"], weights=weights, threads=16)
    assert np.all(st == 0)
    same = np.all(out["chash"] == ref["chash"], 1)
    print(f"weighted={weighted}: contact sets identical on {same.sum()}/{len(same)} robots",
          flush=True)
    assert same.sum() >= len(same) - 1
    np.testing.assert_allclose(loss[same], rloss[same], rtol=1e-9)
    rows = np.concatenate([np.arange(w.inst_i[b, 1], w.inst_i[b, 1] + w.inst_i[b, 2])
                           for b in np.nonzero(same)[0]])
    for got, want in ((dP, rP), (d0, r0), (d1, r1)):
        floor = 1e-6 * np.abs(want[rows]).max()
        r = _rel(got[rows], want[rows], floor)
        print(f"  max rel {r.max():.2e}", flush=True)
        assert r.max() < 1e-6


@pytest.mark.parametrize("h_P,h_s,rtol", STEPS)
def test_grad_matches_fd_of_gpu_rollouts(h_P, h_s, rtol):
    w = W.config4(16).subset(ROBOTS[:5])
    base, (dP, d0, d1, loss, st) = _gpu(w)
    cases = cases_for(w, range(w.n_inst), h_P=h_P, h_s=h_s)
    wp = perturbed(w, cases)
    import torch
    with _sim(wp) as sim:
        s = torch.cuda.current_stream()
        sim.rollout(-1, stream=s)
        s.synchronize()
        o = sim.read_all()
    fd = fd_values(cases, losses(o["tip"], wp.goal))
    ok = smooth(cases, o["chash"], base["chash"], o["negsteps"], base["negsteps"])
    g = {"P": dP, "s0": d0, "s1": d1}
    adj = np.array([g[c.name][c.spam] for c in cases])
    assert ok.sum() >= 10
    r = _rel(adj[ok], fd[ok], 1e-3 * np.abs(adj[ok]).max())
    print(f"FD at h = {h_P:g} Pa, {h_s:g} m: {ok.sum()} smooth cases, max rel {r.max():.2e}", flush=True)
    assert r.max() < rtol


def test_grad_needs_recorded_trajectory():
    from paper_2509_15180_amd import vinesim as V
    import torch
    w = W.config4(16).subset([1])
    with _sim(w) as sim:
        s = torch.cuda.current_stream()
        sim.rollout(10, record_every=1, stream=s)
        sim.rollout(-1, record_every=0, stream=s)
        with pytest.raises(V.VineError) as ei:
            sim.grad(w.goal, np.ones(sim.T), stream=s)
        assert ei.value.code == V.VINE_ESTATE
        # the final-state loss needs no trajectory
        g = sim.grad(w.goal, None, stream=s)
        s.synchronize()
        assert np.isfinite(g[0].cpu().numpy()).all()


@pytest.mark.parametrize("ce", [32, 7])
def test_grad_from_checkpoints_is_bitwise_the_full_trajectory(ce):
    """A trajectory loss from checkpoints every ce steps (the states recomputed segment
    by segment) equals, bit for bit, the one from the recorded trajectory; also when the
    rollout is taken in several calls."""
    import torch
    w = W.config4(16).subset(ROBOTS)
    weights = np.zeros(96)
    weights[3::5] = 0.3
    weights[-1] = 1.0
    _, full = _gpu(w, weights, traj=True)
    _, ck = _gpu(w, weights, traj=False, ckpt=ce)
    with _sim(w) as sim:
        s = torch.cuda.current_stream()
        for _ in range(5):
            sim.step(20, ckpt_every=ce, stream=s)
        parts = tuple(x.cpu().numpy() for x in sim.grad(w.goal, weights, stream=s))
        ck_rows = sim.read("ckpt")
    assert ck_rows.shape == (w.n_inst, -(-96 // ce), 96)
    print(f"ckpt_every={ce}: checkpoint rows {ck_rows.shape[1]}, "
          f"loss {full[3].sum():.6e}", flush=True)
    for a, b, c in zip(full, ck, parts):
        assert np.array_equal(a, b) and np.array_equal(a, c)


def test_adjoint_flags_unconverged_steps():
    """A rollout cut off by the iteration limit (max_iter = 1) is flagged (bit 1) by the
    adjoint of its weighted steps, and the autograd bridge refuses it."""
    import torch

    from paper_2509_15180_amd import vinesim as V
    from paper_2509_15180_amd.autograd import rollout_loss
    w = W.config4(16).subset([1, 2])
    with V.VineSim(w, V.default_params(max_iter=1)) as sim:
        s = torch.cuda.current_stream()
        sim.rollout(-1, record_every=1, stream=s)
        dP, d0, d1, loss, st = sim.grad(w.goal, np.ones(96), stream=s)
        s.synchronize()
        status = sim.read("status")
        assert (status == 1).any()
        assert np.all((st.cpu().numpy() & 2) == 2)
        P = torch.tensor(w.spam[:, 3], dtype=torch.float64, requires_grad=True)
        with pytest.raises(V.VineError):
            rollout_loss(sim, P, torch.tensor(w.spam[:, 0]), torch.tensor(w.spam[:, 1]),
                         w.spam[:, 2], w.goal, np.ones(96))


def test_set_spams_equals_fresh_handle():
    import torch
    w = W.config4(16).subset([1, 2, 3])
    w2 = W.pack([w.instance(i) for i in range(w.n_inst)], "moved")
    w2.spam[:, 3] *= 0.7
    w2.spam[:, 0] += 0.003
    w2.spam[:, 1] = np.minimum(w2.spam[:, 1] + 0.001, 96 * 0.02)
    with _sim(w) as sim:
        s = torch.cuda.current_stream()
        sim.rollout(-1, stream=s)
        sim.set_spams(w2.spam, stream=s)
        sim.reset(stream=s)
        sim.rollout(-1, stream=s)
        s.synchronize()
        a = sim.read_all()
    with _sim(w2) as sim:
        s = torch.cuda.current_stream()
        sim.rollout(-1, stream=s)
        s.synchronize()
        b = sim.read_all()
    assert np.array_equal(a["theta"], b["theta"]) and np.array_equal(a["chash"], b["chash"])


def test_autograd_function_and_descent():
    """rollout_loss backward returns the adjoint; a few gradient steps on the
    pressures lower the loss (a miniature of the design search)."""
    import torch

    from paper_2509_15180_amd.autograd import rollout_loss
    w = W.config4(16).subset([1, 2, 3, 6])
    with _sim(w) as sim:
        P = torch.tensor(w.spam[:, 3], dtype=torch.float64, requires_grad=True)
        s0 = torch.tensor(w.spam[:, 0], dtype=torch.float64, requires_grad=True)
        s1 = torch.tensor(w.spam[:, 1], dtype=torch.float64, requires_grad=True)
        side = w.spam[:, 2]
        L0 = rollout_loss(sim, P, s0, s1, side, w.goal)
        L0.backward()
        _, (dP, d0, d1, loss, st) = _gpu(w, None, traj=False)
        np.testing.assert_allclose(P.grad.numpy(), dP, rtol=1e-12, atol=0)
        np.testing.assert_allclose(s0.grad.numpy(), d0, rtol=1e-12, atol=0)
        assert abs(L0.item() - loss.sum()) <= 1e-12 * loss.sum()
        # one projected gradient step on the pressures, backtracking until the loss drops
        g = P.grad.clone()
        step = 0.05 * P.detach().abs().max().item() / max(g.abs().max().item(), 1e-30)
        Ls = [L0.item()]
        for _ in range(10):
            with torch.no_grad():
                Pt = (P.detach() - step * g).clamp(min=0.0)
                Ls.append(rollout_loss(sim, Pt, s0.detach(), s1.detach(), side, w.goal).item())
            if Ls[-1] < Ls[0]:
                break
            step *= 0.5
        print("loss along the descent line search:", Ls, flush=True)
        assert Ls[-1] < Ls[0]
