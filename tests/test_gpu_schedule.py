"""Launch-order autotuning (vine_sim_tune_order): after a rollout every robot has a
positive cycle count, and rolling the batch out again in the measured order (eagerly and
through a graph captured before the reordering) gives bitwise the same results."""
import numpy as np
import pytest

from paper_2509_15180_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_measured_order_changes_no_result():
    import torch

    from paper_2509_15180_amd import vinesim as V
    torch.cuda.set_device(0)
    s = torch.cuda.current_stream()
    full = W.config3(300)
    n = full.inst_i[:, 0]
    idx = []
    for lo, hi in ((16, 64), (65, 128), (129, 160)):
        idx += [int(i) for i in np.nonzero((n >= lo) & (n <= hi))[0][:6]]
    work = full.subset(idx)
    with V.VineSim(work) as sim:
        sim.rollout_graph(stream=s)  # captured with the create-time order
        s.synchronize()
        ref = sim.read_all()
        assert np.all(ref["cycles"] > 0) and np.all(ref["time"] > 0)
        sim.tune_order(stream=s)
        sim.reset(stream=s)
        sim.rollout(-1, stream=s)
        s.synchronize()
        got = sim.read_all()
        for k in ref:
            if k not in ("cycles", "time"):
                assert np.array_equal(got[k], ref[k]), k
        sim.rollout_graph(stream=s)  # the captured launches read the new order
        s.synchronize()
        again = sim.read_all()
        for k in ref:
            if k not in ("cycles", "time"):
                assert np.array_equal(again[k], ref[k]), k
