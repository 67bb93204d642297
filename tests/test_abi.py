"""The C-ABI library loads, exports every entry point include/vinesim.h declares, and
rejects invalid inputs before touching the device (no GPU needed)."""
import math
import os
import re

import numpy as np
import pytest

from paper_2509_15180_amd import vinesim as V
from paper_2509_15180_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vinesim.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|int64_t|void|const char\*)\s+(vine_\w+)\s*\(",
                                 src, re.M)))


def test_exports_every_declared_symbol():
    L = V.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(V.EXPORTS)


def test_default_params():
    p = V.default_params()
    assert p.R_c == 0.005 and p.R_act == 0.01718 and p.a_corr == 1e-4
    assert p.eps_crit == 0.01 and p.k_c == 1e4 and p.tol == 1e-10
    assert p.growth_substeps == 2 and p.max_iter == 500


def _work():
    return W.pack([dict(n=8, d=(0.02, 0.025, 3000.0, 0, 0, 0), spam=[(0.0, 0.04, 1.0, 1000.0)],
                        kind=[0], obs=[(0.5, 0.1, 0.05, 0.0)])], "one")


@pytest.mark.parametrize("mutate,code", [
    (lambda w: w.inst_d.__setitem__((0, 2), float("nan")), V.VINE_EINVAL),
    (lambda w: w.inst_d.__setitem__((0, 0), -0.02), V.VINE_EINVAL),
    (lambda w: w.spam.__setitem__((0, 2), 0.0), V.VINE_EINVAL),
    (lambda w: w.spam.__setitem__((0, 0), 0.05), V.VINE_EINVAL),
    (lambda w: w.spam.__setitem__((0, 3), float("nan")), V.VINE_EINVAL),
    (lambda w: w.obs_kind.__setitem__(0, 7), V.VINE_EINVAL),
    (lambda w: w.obs_d.__setitem__((0, 2), 0.0), V.VINE_EINVAL),
    (lambda w: w.inst_i.__setitem__((0, 0), 0), V.VINE_EINVAL),
    (lambda w: w.inst_i.__setitem__((0, 0), V.MAX_LINKS + 1), V.VINE_ECAPACITY),
    (lambda w: w.inst_i.__setitem__((0, 4), 3), V.VINE_EINVAL),
])
def test_create_rejects_invalid_input(mutate, code):
    w = _work()
    mutate(w)
    with pytest.raises(V.VineError) as ei:
        V.VineSim(w)
    assert ei.value.code == code


def test_create_rejects_bad_params():
    with pytest.raises(V.VineError) as ei:
        V.VineSim(_work(), V.default_params(growth_substeps=0))
    assert ei.value.code == V.VINE_EINVAL
    with pytest.raises(V.VineError):
        V.VineSim(_work(), V.default_params(tol=-1.0))


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(V, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(V, "_lib", None)
    with pytest.raises(ImportError):
        V.lib()


def test_null_handle_calls_fail_cleanly():
    L = V.lib()
    assert L.vine_sim_set_spams(None, None, 0, None) == V.VINE_EINVAL
    assert L.vine_sim_grad(None, None, None, None, None, None, None, None, None) == V.VINE_EINVAL
    assert L.vine_sim_reset(None, None) == V.VINE_EINVAL
    assert L.vine_sim_rollout_graph(None, 0, 0, None) == V.VINE_EINVAL
    assert L.vine_sim_tune_order(None, None) == V.VINE_EINVAL
    assert L.vine_sim_set_head(None, 0.5, 4, None) == V.VINE_EINVAL
    assert L.vine_sim_head(None, None, None, None, None) == V.VINE_EINVAL


def test_server_rejects_bad_sizes_before_the_device():
    import ctypes as C
    L = V.lib()
    h = C.c_void_p()
    p = V.default_params()
    assert L.vine_server_create(C.byref(p), 0, 1 << 30, 64, 8, 4, C.byref(h)) == V.VINE_EINVAL
    assert L.vine_server_create(C.byref(p), 8, 1 << 30, V.MAX_LINKS + 1, 8, 4, C.byref(h)) == \
        V.VINE_ECAPACITY
    # a budget below one robot at the bounds (92 B per link row, 36 B per obstacle)
    assert L.vine_server_create(C.byref(p), 8, 92 * 64 + 36 * 8, 64, 8, 4, C.byref(h)) == \
        V.VINE_EINVAL
    assert L.vine_server_tick(None, 4, None) == V.VINE_EINVAL
    inst = V.Instance(n_links=4, link_len=0.02, tube_radius=0.025, body_pressure=3000.0)
    cnt, th = C.c_int32(2), (C.c_double * 2)()
    assert L.vine_server_submit_from(None, 1, C.byref(inst), 1, None, 0, None, 0, C.byref(cnt),
                                     th) == V.VINE_EINVAL
    assert L.vine_server_poll(None, None, None, 0) == V.VINE_EINVAL


def test_server_submit_each_marshals_one_robot_per_request():
    """submit_each hands the library one instance at a time from one packed array (the
    planner's path); on a null server the call is rejected before any device work."""
    srv = object.__new__(V.VineServer)
    srv.h, srv.n_links = None, {}
    work = W.pack([dict(n=5, d=(0.02, 0.025, 4000.0, 0, 0, 0), spam=[(0.0, 0.04, 1.0, 3000.0)],
                        kind=[0], obs=[(0.5, 0.0, 0.05, 0.0)]),
                   dict(n=7, d=(0.02, 0.025, 4000.0, 0, 0, 0), spam=[], kind=[], obs=[])], "two")
    with pytest.raises(V.VineError) as e:
        srv.submit_each(10, work)
    assert e.value.code == V.VINE_EINVAL


def test_synthesis_rejects_bad_inputs_before_the_device():
    import ctypes as C
    L = V.lib()
    dp = C.POINTER(C.c_double)
    p = V.default_params()

    def call(P, Lu, t, tol=1e-3, geo=(0.025, 0.03335, 10342.0), prm=p):
        P, Lu, t = (np.ascontiguousarray(x, np.float64) for x in (P, Lu, t))
        des = np.zeros(3 * max(1, len(t)))
        return L.vine_spam_synth(C.byref(prm) if prm is not None else None, *geo,
                                 P.ctypes.data_as(dp), len(P), Lu.ctypes.data_as(dp), len(Lu),
                                 t.ctypes.data_as(dp), len(t), tol, des.ctypes.data_as(dp), None,
                                 None)

    good_P, good_L, good_t = [2e3, 4e3], [0.02, 0.03], [0.01]
    assert call(good_P, good_L, good_t, prm=None) == V.VINE_EINVAL
    assert call([4e3, 2e3], good_L, good_t) == V.VINE_EINVAL        # pressures not rising
    assert b"rising" in L.vine_sim_last_error(None)
    assert call([2e3, 2e3], good_L, good_t) == V.VINE_EINVAL
    assert call([-1.0, 2e3], good_L, good_t) == V.VINE_EINVAL
    assert call(good_P, [0.03, 0.02], good_t) == V.VINE_EINVAL      # lengths not rising
    assert call(good_P, [0.0, 0.02], good_t) == V.VINE_EINVAL
    assert call(good_P, good_L, [math.nan]) == V.VINE_EINVAL
    assert call(good_P, good_L, good_t, tol=-1.0) == V.VINE_EINVAL
    assert call(good_P, good_L, good_t, geo=(0.0, 0.03335, 10342.0)) == V.VINE_EINVAL
    assert call(np.arange(1, 4098) * 1e3, good_L, good_t) == V.VINE_ECAPACITY  # 4097 pressures
