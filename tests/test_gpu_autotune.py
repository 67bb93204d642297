"""Waves per robot and the autotuner: one wave per robot (the obstacle phase on the solver's
own wave), two (on a helper wave beside the joint law) and four (helpers splitting the joint
law and the obstacle phase by chunks) give bitwise the same results, in hard and in soft
growth, eager and captured; the autotuner measures each class every way, keeps a valid
choice, and a second handle of the same configuration takes it from the cache without
measuring."""
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
