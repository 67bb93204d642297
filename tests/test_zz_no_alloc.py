"""vine_sim_grad_noalloc (the allocation-free adjoint, its segment buffers in a static
device array) against vine_sim_grad through the C ABI: bitwise the same outputs on two
calls in a row, the second on a smaller problem (the array keeps the first call's
contents), and a clear capacity error beyond the array."""
import ctypes as C

import numpy as np
import pytest

from paper_2509_15180_amd import workloads as W

pytestmark = pytest.mark.gpu


def _grad_pair(sim, work, weights, first_noalloc):
    import torch

    from paper_2509_15180_amd import vinesim as V
    L = V.lib()
    dev = torch.device("cuda", 0)
    s = torch.cuda.current_stream()
    g = torch.as_tensor(work.goal, dtype=torch.float64, device=dev).contiguous()
    w = torch.as_tensor(weights, dtype=torch.float64, device=dev).contiguous()
    outs = {}
    for noalloc in ((True, False) if first_noalloc else (False, True)):
        S = max(sim.S, 1)
        bufs = [torch.full((S,), np.nan, dtype=torch.float64, device=dev) for _ in range(3)]
        loss = torch.full((sim.B,), np.nan, dtype=torch.float64, device=dev)
        st = torch.full((sim.B,), -7, dtype=torch.int32, device=dev)
        fn = L.vine_sim_grad_noalloc if noalloc else L.vine_sim_grad
        p = lambda t: C.c_void_p(t.data_ptr())
        rc = fn(sim.h, p(g), p(w), p(bufs[0]), p(bufs[1]), p(bufs[2]), p(loss), p(st),
                C.c_void_p(s.cuda_stream))
        assert rc == V.VINE_OK, L.vine_sim_last_error(sim.h)
        s.synchronize()
        outs[noalloc] = [b.cpu().numpy()[:sim.S] for b in bufs] + [loss.cpu().numpy(),
                                                                   st.cpu().numpy()]
    return outs


def test_noalloc_grad_equals_grad_twice_then_smaller():
    import torch

    from paper_2509_15180_amd import vinesim as V
    torch.cuda.set_device(0)
    s = torch.cuda.current_stream()
    big = W.config4(24).subset(list(range(4, 24)))
    small = W.config4(8).subset([1, 2, 3])
    for k, (work, ce, first_noalloc) in enumerate(((big, 32, True), (small, 16, False))):
        print(f"call {k}: {work.n_inst} robots, checkpoints every {ce} steps", flush=True)
        weights = np.zeros(96)
        weights[5::4] = 0.5
        weights[-1] = 1.0
        with V.VineSim(work) as sim:
            sim.rollout(-1, ckpt_every=ce, stream=s)
            outs = _grad_pair(sim, work, weights, first_noalloc)
        for a, b in zip(outs[True], outs[False]):
            assert np.array_equal(a, b)
        assert np.isfinite(outs[True][3]).all() and np.all(outs[True][4] >= 0)


def test_noalloc_grad_rejects_needs_beyond_the_scratch():
    import torch

    from paper_2509_15180_amd import vinesim as V
    torch.cuda.set_device(0)
    s = torch.cuda.current_stream()
    one = dict(n=512, d=(0.02, 0.025, 3000.0, 0.0, 0.0, 0.0), spam=[], kind=[], obs=[])
    work = W.pack([one] * 1200, "wide")
    with V.VineSim(work) as sim:
        sim.rollout(1, ckpt_every=32, stream=s)
        with pytest.raises(V.VineError) as ei:
            sim.grad(work.goal, np.ones(sim.T), stream=s, noalloc=True)
        assert ei.value.code == V.VINE_ECAPACITY
        assert "scratch" in str(ei.value)
