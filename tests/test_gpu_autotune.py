"""Waves per robot and the autotuner: one wave per robot (the obstacle phase on the solver's
own wave), two (on a helper wave beside the joint law) and four (helpers splitting the joint
law and the obstacle phase by chunks) give bitwise the same results, in hard and in soft
growth, eager and captured, and so does a head launch of the slowest robots (rollouts and
gradients from checkpoints); the autotuner measures each class every way and the whole
batch with and without a head, keeps a valid choice, and a second handle of the same
configuration takes it from the cache without measuring."""
import numpy as np
import pytest

from paper_2509_15180_amd import workloads as W

pytestmark = pytest.mark.gpu

TIMING = ("cycles", "time")


def _mixed():
    full = W.config3(400)
    n = full.inst_i[:, 0]
    idx = []
    for lo, hi in ((16, 64), (65, 128), (129, 200)):
        idx += [int(i) for i in np.nonzero((n >= lo) & (n <= hi))[0][:3]]
    return full.subset(idx)


def _run(work, waves, graph=False, **params):
    import torch

    from paper_2509_15180_amd import vinesim as V
    torch.cuda.set_device(0)
    s = torch.cuda.current_stream()
    with V.VineSim(work, V.default_params(**params)) as sim:
        sim.set_waves(waves)
        if graph:
            sim.rollout_graph(stream=s)
            s.synchronize()
            sim.rollout_graph(stream=s)
        else:
            sim.rollout(-1, stream=s)
        s.synchronize()
        return sim.read_all()


def _equal(a, b):
    for k in a:
        if k not in TIMING:
            assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("soft", [0.0, 2000.0])
def test_one_and_two_waves_are_bitwise_equal(soft):
    w = _mixed()
    two = _run(w, [2, 2, 2, 2], growth_stiffness=soft)
    for waves in ([1, 1, 1, 1], [4, 4, 4, 4]):
        _equal(two, _run(w, waves, growth_stiffness=soft))
    _equal(two, _run(w, [1, 4, 2, 4], graph=True, growth_stiffness=soft))


def test_autotune_measures_chooses_and_caches():
    import torch

    from paper_2509_15180_amd import vinesim as V
    s = torch.cuda.current_stream()
    w = _mixed()
    ref = _run(w, [2, 2, 2, 2])
    with V.VineSim(w) as sim:
        a = sim.autotune(stream=s)
        print(f"autotune: {a}", flush=True)
        assert not a["cached"]
        for c in range(3):
            assert a["waves"][c] in (1, 2, 4)
            assert min(a["ms_one_wave"][c], a["ms_two_waves"][c], a["ms_four_waves"][c]) > 0.0
        assert a["waves"][3] == 0 and a["ms_one_wave"][3] == 0.0
        assert np.all(sim.read("nlinks") == 0)  # the robots end reset
        sim.rollout_graph(stream=s)
        s.synchronize()
        _equal(ref, sim.read_all())
    with V.VineSim(w) as sim:
        b = sim.autotune(stream=s)
        assert b["cached"] and b["waves"] == a["waves"]
        assert b["ms_one_wave"] == [0.0] * 4
        assert b["head"]["fraction"] == a["head"]["fraction"]
    # the whole batch measured with and without a head once the robots are measured
    with V.VineSim(w) as sim:
        sim.rollout(-1, stream=s)
        sim.tune_order(stream=s)
        r = sim.autotune(stream=s)
        print(f"autotune after measuring: {r}", flush=True)
        hd = r["head"]
        assert r["cached"]  # the classes' own measurements from the cache
        assert r["waves"] in (a["waves"], [2 if x else 0 for x in a["waves"]])
        assert hd["fraction"] in (0.0, 0.5, 0.25) and hd["waves"] == 4
        assert min(hd["ms_whole_batch"]["fastest_alone"].values()) > 0.0  # measured once
        sim.rollout_graph(stream=s)
        s.synchronize()
        _equal(ref, sim.read_all())


def _rollout_with_head(work, fraction, waves=4, graph=False, ckpt=0, goal=None):
    """First rollout to measure the robots, then the launch order with a head of the robots
    at or above `fraction` of the slowest's cycles (0: none), then a rollout from zero."""
    import torch

    from paper_2509_15180_amd import vinesim as V
    torch.cuda.set_device(0)
    s = torch.cuda.current_stream()
    with V.VineSim(work) as sim:
        sim.rollout(-1, stream=s)
        sim.tune_order(stream=s)
        sim.set_head(fraction, waves, stream=s)
        head = sim.head()
        sim.reset(stream=s)
        if graph:
            sim.rollout_graph(ckpt_every=ckpt, stream=s)
            s.synchronize()
            sim.rollout_graph(ckpt_every=ckpt, stream=s)
        else:
            sim.rollout(-1, ckpt_every=ckpt, stream=s)
        s.synchronize()
        out = sim.read_all()
        grads = None
        if goal is not None:
            grads = [x.cpu().numpy() for x in sim.grad(goal, torch.ones(sim.T, dtype=torch.float64,
                                                                        device="cuda"), stream=s)]
        return out, head, grads


def test_head_launch_is_bitwise_the_classes_launches():
    """The slowest robots in a launch of their own (sized for the longest of them, so short
    chains run in a longer class's kernel) with 4, 2 or 1 waves: the same results."""
    w = _mixed()
    ref, head0, _ = _rollout_with_head(w, 0.0)
    assert head0["robots"] == 0
    for frac, waves, graph in ((0.02, 4, False), (0.02, 2, True), (0.5, 4, True), (0.02, 1, False)):
        got, head, _ = _rollout_with_head(w, frac, waves, graph)
        print(f"head fraction {frac}, {waves} waves: {head['robots']} robots", flush=True)
        assert head["robots"] > 0 and head["fraction"] == frac and head["waves"] == waves
        _equal(ref, got)
    # a fraction that takes every robot of two classes and some of the third
    got, head, _ = _rollout_with_head(w, 0.02, 4)
    assert head["robots"] >= 4


def test_head_launch_gradients_from_checkpoints_are_bitwise():
    import torch
    w = W.config4(48)
    goal = torch.as_tensor(w.goal, dtype=torch.float64).cuda()
    ref, _, g0 = _rollout_with_head(w, 0.0, ckpt=32, goal=goal)
    got, head, g1 = _rollout_with_head(w, 0.3, 4, ckpt=32, goal=goal)
    assert head["robots"] > 0
    _equal(ref, got)
    for a, b in zip(g0, g1):
        assert np.array_equal(a, b)
