"""The FP64 oracle built with gcc's address and undefined-behaviour sanitizers (host code
only) and run on small workloads: no sanitizer report, and the same results as the normal
build (the contact-heavy, head-on and gradient paths included)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2509_15180_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    out = str(tmp_path_factory.mktemp("asan") / "oracle_sanitized")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-o", out,
           os.path.join(ROOT, "oracle", "sanitize_main.c"),
           os.path.join(ROOT, "oracle", "vine_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _write(path, work, n_steps, prm):
    with open(path, "wb") as f:
        np.array([work.n_inst, len(work.spam), len(work.obs_kind), n_steps, work.n_max],
                 np.int32).tofile(f)
        np.ascontiguousarray(work.inst_i, np.int32).tofile(f)
        np.ascontiguousarray(work.inst_d, np.float64).tofile(f)
        np.ascontiguousarray(work.spam, np.float64).tofile(f)
        np.ascontiguousarray(work.obs_kind, np.int32).tofile(f)
        np.ascontiguousarray(work.obs_d, np.float64).tofile(f)
        np.ascontiguousarray(prm, np.float64).tofile(f)
        np.ascontiguousarray(work.goal, np.float64).tofile(f)


def _read(path, work, T):
    B, N, S = work.n_inst, work.n_max, len(work.spam)
    raw = open(path, "rb").read()
    off = 0

    def take(dt, count):
        nonlocal off
        a = np.frombuffer(raw, dt, count, off)
        off += a.nbytes
        return a

    out = dict(theta=take(np.float64, B * N).reshape(B, N), tip=take(np.float64, B * T * 3).reshape(B, T, 3),
               status=take(np.int32, B * T).reshape(B, T), chash=take(np.uint64, B * T).reshape(B, T),
               dP=take(np.float64, S), ds0=take(np.float64, S), ds1=take(np.float64, S),
               loss=take(np.float64, B))
    assert off == len(raw)
    return out


def test_sanitized_oracle_matches(driver, tmp_path):
    l = 0.02
    work = W.pack([W.config4(8).instance(i) for i in (1, 2)] +
                  [dict(n=30, d=(l, 0.025, 3000.0, 0.0, 0.0, 0.0), spam=[], kind=[1],
                        obs=[(0.3, 0.0, 0.05, 0.05)], goal=(0.3, 0.3))], "asan")
    work = W.pack([dict(work.instance(i), n=min(int(work.inst_i[i, 0]), 40)) for i in range(3)],
                  "asan")
    prm = O.params()
    T = work.n_max
    _write(tmp_path / "in.bin", work, T, prm)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", OMP_NUM_THREADS="1")
    r = subprocess.run([driver, str(tmp_path / "in.bin"), str(tmp_path / "out.bin")], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    got = _read(tmp_path / "out.bin", work, T)
    ref = O.rollout(work, traj=True, threads=1)
    dP, d0, d1, loss = O.gradient(work, ref["traj"], threads=1)
    assert np.array_equal(got["status"], ref["status"]) and np.array_equal(got["chash"], ref["chash"])
    np.testing.assert_allclose(got["theta"], ref["theta"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(got["tip"], ref["tip"], rtol=0, atol=1e-12)
    for a, b in ((got["dP"], dP), (got["ds0"], d0), (got["ds1"], d1), (got["loss"], loss)):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * max(1.0, np.abs(b).max()))
