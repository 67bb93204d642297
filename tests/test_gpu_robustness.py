"""Robustness and funnelling batches on the GPU against the FP64 oracle: perturbed
copies of one design (obstacles and actuation jittered) and the same design from evenly
spread start headings, rolled out in one batch each; tolerances as in the parity tests."""
import numpy as np
import pytest

import oracle as O
from paper_2509_15180_amd import robustness as Rb
from paper_2509_15180_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_TH, TOL_TIP = 1e-5, 1e-4


def _gpu(work):
    import torch

    from paper_2509_15180_amd import vinesim as V
    torch.cuda.set_device(0)
    with V.VineSim(work) as sim:
        s = torch.cuda.current_stream()
        sim.rollout(-1, stream=s)
        s.synchronize()
        return sim.read_all()


def _check(work):
    got = _gpu(work)
    ref = O.rollout(work, threads=16)
    T = work.n_max
    dth = np.abs(got["theta"] - ref["theta"]).max(1)
    dtip = np.abs(got["tip"][:, :T] - ref["tip"][:, :T]).max((1, 2))
    same = np.all(got["chash"][:, :T] == ref["chash"][:, :T], 1)
    print(f"{work.name}: B={work.n_inst} max dtheta {dth.max():.2e} max dtip {dtip.max():.2e} "
          f"sets identical {same.sum()}/{len(same)}", flush=True)
    ok = (dth <= TOL_TH) & (dtip <= TOL_TIP) & same
    assert ok.sum() >= len(ok) - 1, np.nonzero(~ok)[0]
    from test_gpu_parity import _misses_are_minima
    _misses_are_minima(work, ref, ok, T)
    return got


def test_perturbed_design_batch_matches_oracle():
    w = W.config2(2)
    got = _check(W.perturbed(w, 1, 16, sigma_env=0.05, sigma_act=0.1, tag=7))
    n = got["nlinks"]
    tips = got["tip"][np.arange(len(n)), n - 1, :2]
    rate = Rb.success_rate(tips, tips.mean(0), 0.1)
    assert 0.0 <= rate <= 1.0


def test_start_angle_batch_matches_oracle():
    w = W.config2(1)
    got = _check(W.start_angles(w, 0, 12, np.deg2rad(20.0)))
    n = got["nlinks"]
    ends = got["tip"][np.arange(len(n)), n - 1, :2]
    assert Rb.knn_density_ratio(ends, k=3) >= 1.0
