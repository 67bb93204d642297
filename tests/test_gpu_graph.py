"""The captured rollout (vine_sim_rollout_graph) against the eager vine_sim_reset +
vine_sim_rollout: bitwise equal results on every replay, with eager work on the same
stream between replays, for one chain-length class and for three classes at once (whose
launches fork onto the handle's streams and join back inside the graph)."""
import numpy as np
import pytest

from paper_2509_15180_amd import workloads as W

pytestmark = pytest.mark.gpu


def _replays_match(work, record):
    import torch

    from paper_2509_15180_amd import vinesim as V
    torch.cuda.set_device(0)
    s = torch.cuda.current_stream()
    with V.VineSim(work) as sim, V.VineSim(work.subset([0])) as other:
        sim.reset(stream=s)
        sim.rollout(-1, record_every=1 if record else 0, ckpt_every=32 if record else 0, stream=s)
        s.synchronize()
        ref = sim.read_all(traj=record)
        if record:
            ref["ckpt"] = sim.read("ckpt")
        for rep in range(3):
            print(f"replay {rep} (record={record}, {work.n_inst} robots)", flush=True)
            sim.rollout_graph(record_every=1 if record else 0, ckpt_every=32 if record else 0,
                              stream=s)
            # eager work between replays: another handle's launches and a torch reduction
            other.reset(stream=s)
            other.rollout(-1, stream=s)
            total = torch.ones(1 << 20, device="cuda", dtype=torch.float64).sum()
            s.synchronize()
            assert float(total) == float(1 << 20)
            got = sim.read_all(traj=record)
            if record:
                got["ckpt"] = sim.read("ckpt")
            for k in ref:
                if k not in ("cycles", "time"):  # timing, not a result
                    assert np.array_equal(got[k], ref[k]), (rep, k)


def test_graph_replays_one_class():
    _replays_match(W.config2(24), record=False)


def test_graph_replays_three_classes_with_trajectory():
    full = W.config3(400)
    n = full.inst_i[:, 0]
    idx = []
    for lo, hi in ((16, 64), (65, 128), (129, 200)):
        idx += [int(i) for i in np.nonzero((n >= lo) & (n <= hi))[0][:2]]
    assert len(idx) == 6
    _replays_match(full.subset(idx), record=True)
