"""Serving (continuous batching) through the C ABI: requests of mixed size streamed
through a server with few slots give bitwise the results of the same robots rolled
out alone with the batch entry points, and every request completes."""
import numpy as np
import pytest

from paper_2509_15180_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_mixed_stream_equals_alone():
    import torch

    from paper_2509_15180_amd import vinesim as V
    torch.cuda.set_device(0)
    reqs = W.config5_requests(10, n_max=160, k_max=48, s_max=6)
    stream = torch.cuda.current_stream()
    with V.VineServer(slots=24, max_links=160, max_obstacles=48, max_spams=8) as srv:
        pending = list(reqs)
        done = {}
        rounds = 0
        while len(done) < len(reqs):
            # two new requests per round while any remain
            for _ in range(2):
                if pending:
                    r = pending.pop(0)
                    srv.submit(r.rid, r.work)
            srv.tick(8, stream=stream)
            for rid, worst in srv.poll():
                done[rid] = worst
            rounds += 1
            assert rounds < 10000
        st = srv.stats()
        print(f"server: {rounds} rounds, {st['joint_updates']} joint-updates, "
              f"worst statuses {sorted(set(done.values()))}", flush=True)
        assert st["completed"] == len(reqs) and st["queued"] == 0 and st["active"] == 0
        assert st["joint_updates"] == sum(r.work.joint_updates() for r in reqs)
        for r in reqs:
            with V.VineSim(r.work) as sim:
                sim.rollout(-1, stream=stream)
                stream.synchronize()
                out = sim.read_all()
            for k in range(r.work.n_inst):
                tip, th = srv.result(r.rid, k)
                n = int(r.work.inst_i[k, 0])
                assert np.array_equal(th, out["theta"][k, :n]), (r.rid, k)
                assert np.array_equal(tip, out["tip"][k, n - 1]), (r.rid, k)
            srv.release(r.rid)
