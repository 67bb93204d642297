"""Per-step status paths, forced from the host through the parameters and inputs the
boundary accepts, on the HIP path and on the oracle (which follows the same descent):

  1 iteration limit     max_iter = 2
  2 no descent          k_c = 1e200: the damped systems overflow, every damping fails
  3 contact capacity    100 identical circles on the first link: 200 penetrating
                        (disk, obstacle) pairs, more than the device's contact list holds

Status 4 (a non-finite residual or energy) cannot be reached from validated inputs: the
boundary rejects non-finite numbers, and no finite parameter set makes the energy
overflow before the systems do (status 2).  The statuses agree with the oracle's up to
each robot's first forced step; after it the unconverged states may drift apart by
rounding.  A robot with a forced status leaves its neighbours in the launch untouched."""
import numpy as np
import pytest

import oracle as O
from paper_2509_15180_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu(work, **over):
    import torch

    from paper_2509_15180_amd import vinesim as V
    torch.cuda.set_device(0)
    with V.VineSim(work, V.default_params(**over)) as sim:
        s = torch.cuda.current_stream()
        sim.rollout(-1, stream=s)
        s.synchronize()
        return sim.read_all()


def _agree_to_first(got, ref, code):
    """Statuses equal on every step up to each robot's first step with `code`, and that
    step the same on both sides; returns the number of robots that reach it."""
    hits = 0
    for b in range(ref.shape[0]):
        where = np.nonzero(ref[b] == code)[0]
        t = int(where[0]) if where.size else ref.shape[1] - 1
        np.testing.assert_array_equal(got[b, :t + 1], ref[b, :t + 1], err_msg=f"robot {b}")
        hits += int(where.size > 0)
    return hits


def test_iteration_limit():
    w = W.config2(8)
    ref = O.rollout(w, prm=O.params(max_iter=2), threads=8)
    got = _gpu(w, max_iter=2)
    assert _agree_to_first(got["status"], ref["status"], 1) == w.n_inst
    assert (got["status"] == 1).sum() > 100


def test_no_descent_at_extreme_stiffness():
    w = W.config2(8)
    ref = O.rollout(w, prm=O.params(kc=1e200), threads=8)
    got = _gpu(w, k_c=1e200)
    assert _agree_to_first(got["status"], ref["status"], 2) >= 6
    assert (got["status"] == 2).sum() > 100


def _crowded(n=8):
    return dict(n=n, d=(0.02, 0.025, 4000.0, 0.0, 0.0, 0.0), spam=np.zeros((0, 4)),
                kind=np.zeros(100, np.int32), obs=np.tile([0.015, 0.0, 0.01, 0.0], (100, 1)))


def test_contact_capacity_and_neighbours_unaffected():
    normal = W.config2(6)
    items = [normal.instance(i) for i in range(3)] + [_crowded()] + \
            [normal.instance(i) for i in range(3, 6)]
    mixed = W.pack(items, "crowded")
    ref = O.rollout(mixed.subset([3]), threads=1)
    assert ref["ncont"][0, 0] == 100  # 100 (link, obstacle) pairs, two disks each
    got = _gpu(mixed)
    assert np.all(got["status"][3, :8] == 3) and np.all(got["status"][3, 8:] == -1)
    alone = _gpu(normal)
    rows = [0, 1, 2, 4, 5, 6]
    for k in ("theta", "tip", "chash", "status", "iters"):
        assert np.array_equal(got[k][rows][:, :alone[k].shape[1]], alone[k]), k
