"""FP64 CPU oracle for the vine-robot growth step (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``vine_oracle.c`` (plain C,
built with gcc) through ctypes and shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

# parameter vector layout (see prm_from in vine_oracle.c)
PARAM_NAMES = ("Rc", "Ract", "acorr", "epsc", "kc", "tol", "max_iter", "substeps", "fd_h", "c1",
               "c_mu", "cheb_n", "step_max", "mu_up", "pd_shift", "wg")
DEFAULTS = dict(Rc=0.005, Ract=0.01718, acorr=1e-4, epsc=0.01, kc=1e4, tol=1e-10, max_iter=500,
                substeps=2, fd_h=0.0, c1=1e-4, c_mu=1.0, cheb_n=128,
                step_max=0.05, mu_up=10.0, pd_shift=1e-8, wg=0.0)


def params(**over) -> np.ndarray:
    d = dict(DEFAULTS)
    for k, v in over.items():
        if k not in d:
            raise KeyError(k)
        d[k] = v
    return np.asarray([float(d[k]) for k in PARAM_NAMES], np.float64)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        for name in ("vo_rf", "vo_rd"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double] * 3
        for name in ("vo_ellf", "vo_elle", "vo_wr_h", "vo_wr_dh", "vo_wr_int"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double] * 2
        L.vo_spam_state.restype = C.c_int
        L.vo_spam_state.argtypes = [C.c_double, C.c_double, dp, dp, dp, dp]
        L.vo_spam_G_exact.restype = C.c_double
        L.vo_spam_G_exact.argtypes = [C.c_double, C.c_double, dp]
        for name in ("vo_dist_circle", "vo_dist_box"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double, C.c_double, dp, dp, dp, dp]
        L.vo_chain_eval.restype = C.c_double
        L.vo_chain_eval.argtypes = [C.c_int, dp, dp, C.c_int, C.c_int, ip, dp, dp, C.c_double, dp,
                                    dp, ip, dp, C.c_int]
        L.vo_chain_hessian.restype = None
        L.vo_chain_hessian.argtypes = [C.c_int, dp, dp, C.c_int, C.c_int, ip, dp, dp, C.c_double,
                                       dp, dp]
        L.vo_chain_solve.restype = C.c_int
        L.vo_chain_solve.argtypes = [C.c_int, dp, dp, C.c_int, C.c_int, ip, dp, dp, C.c_double, dp,
                                     dp]
        L.vo_chain_eval_soft.restype = C.c_double
        L.vo_chain_eval_soft.argtypes = L.vo_chain_eval.argtypes
        L.vo_chain_hessian_soft.restype = None
        L.vo_chain_hessian_soft.argtypes = L.vo_chain_hessian.argtypes
        L.vo_chain_solve_soft.restype = C.c_int
        L.vo_chain_solve_soft.argtypes = L.vo_chain_solve.argtypes
        L.vo_gfit_eval.restype = None
        L.vo_gfit_eval.argtypes = [C.c_double, dp, C.c_int, dp, dp, dp, dp, dp]
        L.vo_spam_coverage.restype = None
        L.vo_spam_coverage.argtypes = [C.c_int, C.c_double, dp, C.c_int, dp, dp]
        L.vo_joint_law.restype = None
        L.vo_joint_law.argtypes = [dp, C.c_double, C.c_double, dp, C.c_int, dp, dp, dp]
        L.vo_rollout.restype = C.c_int
        L.vo_rollout.argtypes = [C.c_int, ip, dp, dp, ip, dp, dp, C.c_int, C.c_int, C.c_int, dp,
                                 dp, dp, ip, ip, ip, C.POINTER(C.c_uint64), dp, dp, dp, dp]
        L.vo_gradient.restype = C.c_int
        L.vo_gradient.argtypes = [C.c_int, ip, dp, dp, ip, dp, dp, C.c_int, C.c_int, dp, dp, dp,
                                  C.c_int, dp, dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, np.int32))


# ---------------------------------------------------------------------------
# elementary functions


def rf(x, y, z):
    return lib().vo_rf(x, y, z)


def rd(x, y, z):
    return lib().vo_rd(x, y, z)


def ellf(phi, m):
    return lib().vo_ellf(phi, m)


def elle(phi, m):
    return lib().vo_elle(phi, m)


def spam_state(m, l0, prm=None):
    """(eps, G, phi, saturated) for contraction parameter m (Eq. 1a-d)."""
    prm = params() if prm is None else prm
    e, g, p = C.c_double(), C.c_double(), C.c_double()
    sat = lib().vo_spam_state(m, l0, _d(prm), C.byref(e), C.byref(g), C.byref(p))
    return e.value, g.value, p.value, bool(sat)


def G_exact(eps, l0, prm=None):
    prm = params() if prm is None else prm
    return lib().vo_spam_G_exact(eps, l0, _d(prm))


def gfit(l0, eps, prm=None):
    """Chebyshev G, dG/deps, int_0^eps G at eps; plus (G0, eps_max, tail)."""
    prm = params() if prm is None else prm
    eps = _f64(np.atleast_1d(eps))
    G, dG, IG, info = (np.zeros_like(eps), np.zeros_like(eps), np.zeros_like(eps), np.zeros(3))
    lib().vo_gfit_eval(l0, _d(prm), len(eps), _d(eps), _d(G), _d(dG), _d(IG), _d(info))
    return G, dG, IG, info


def wr_h(x, epsc=0.01):
    return lib().vo_wr_h(x, epsc)


def wr_dh(x, epsc=0.01):
    return lib().vo_wr_dh(x, epsc)


def wr_int(x, epsc=0.01):
    return lib().vo_wr_int(x, epsc)


def dist(kind, x, obs):
    """(signed distance, unit normal, curvature) from point x to one obstacle row."""
    o = _f64(obs)
    nx, ny, kap = C.c_double(), C.c_double(), C.c_double()
    f = lib().vo_dist_circle if kind == 0 else lib().vo_dist_box
    d = f(x[0], x[1], _d(o), C.byref(nx), C.byref(ny), C.byref(kap))
    return d, np.array([nx.value, ny.value]), kap.value


def coverage(n, l, spam):
    spam = _f64(np.asarray(spam).reshape(-1, 4))
    Pp, Pm = np.zeros(n), np.zeros(n)
    lib().vo_spam_coverage(n, l, _d(spam), len(spam), _d(Pp), _d(Pm))
    return Pp, Pm


def joint_law(d, pp, pm, th, prm=None):
    prm = params() if prm is None else prm
    th = _f64(np.atleast_1d(th))
    q, E = np.zeros_like(th), np.zeros_like(th)
    lib().vo_joint_law(_d(_f64(d)), pp, pm, _d(prm), len(th), _d(th), _d(q), _d(E))
    return q, E


# ---------------------------------------------------------------------------
# one chain


def _chain_args(inst: dict):
    d = _f64(inst["d"])
    spam = _f64(np.asarray(inst["spam"]).reshape(-1, 4))
    kind = _i32(np.asarray(inst["kind"]).reshape(-1))
    obs = _f64(np.asarray(inst["obs"]).reshape(-1, 4))
    return d, spam, kind, obs


def chain_eval(inst: dict, th, prm=None, last_len=0.0):
    """(Pi, r, contacts[c, 8]) for the chain of len(th) links of an instance dict."""
    prm = params() if prm is None else prm
    d, spam, kind, obs = _chain_args(inst)
    th = _f64(th)
    n = len(th)
    r = np.zeros(n)
    cap = max(1, 2 * n * max(1, len(kind)))
    cont = np.zeros((cap, 8))
    nc = C.c_int()
    Pi = lib().vo_chain_eval(n, _d(d), _d(spam), len(spam), len(kind), _i(kind), _d(obs),
                             _d(prm), last_len, _d(th), _d(r), C.byref(nc), _d(cont), cap)
    return Pi, r, cont[:nc.value].copy()


def chain_hessian(inst: dict, th, prm=None, last_len=0.0):
    """Analytic Hessian of Pi at th."""
    prm = params() if prm is None else prm
    d, spam, kind, obs = _chain_args(inst)
    th = _f64(th)
    n = len(th)
    H = np.zeros((n, n))
    lib().vo_chain_hessian(n, _d(d), _d(spam), len(spam), len(kind), _i(kind), _d(obs), _d(prm),
                           last_len, _d(th), _d(H))
    return H


def chain_eval_soft(inst: dict, x, tgt, prm=None):
    """Soft growth: (Pi, r, contacts) at x = (theta_0..theta_{n-1}, u), the tip link's length
    u l, with the growth term's target tgt (link lengths); r has n + 1 entries."""
    prm = params() if prm is None else prm
    d, spam, kind, obs = _chain_args(inst)
    x = _f64(x)
    n = len(x) - 1
    r = np.zeros(n + 1)
    cap = max(1, 2 * n * max(1, len(kind)))
    cont = np.zeros((cap, 8))
    nc = C.c_int()
    Pi = lib().vo_chain_eval_soft(n, _d(d), _d(spam), len(spam), len(kind), _i(kind), _d(obs),
                                  _d(prm), tgt, _d(x), _d(r), C.byref(nc), _d(cont), cap)
    return Pi, r, cont[:nc.value].copy()


def chain_hessian_soft(inst: dict, x, tgt, prm=None):
    """Soft growth: the analytic (n + 1) x (n + 1) Hessian at x = (theta, u)."""
    prm = params() if prm is None else prm
    d, spam, kind, obs = _chain_args(inst)
    x = _f64(x)
    n = len(x) - 1
    H = np.zeros((n + 1, n + 1))
    lib().vo_chain_hessian_soft(n, _d(d), _d(spam), len(spam), len(kind), _i(kind), _d(obs),
                                _d(prm), tgt, _d(x), _d(H))
    return H


def chain_solve_soft(inst: dict, x0, tgt, prm=None):
    """Soft growth: the equilibrium from x0 = (theta, u): (x, status, info)."""
    prm = params() if prm is None else prm
    d, spam, kind, obs = _chain_args(inst)
    x = _f64(x0).copy()
    info = np.zeros(5)
    st = lib().vo_chain_solve_soft(len(x) - 1, _d(d), _d(spam), len(spam), len(kind), _i(kind),
                                   _d(obs), _d(prm), tgt, _d(x), _d(info))
    return x, st, info


def chain_solve(inst: dict, th0, prm=None, last_len=0.0):
    """Equilibrium from th0: (theta, status, info[iters, backtracks, mu raises, rho,
    steps along negative curvature])."""
    prm = params() if prm is None else prm
    d, spam, kind, obs = _chain_args(inst)
    th = _f64(th0).copy()
    info = np.zeros(5)
    st = lib().vo_chain_solve(len(th), _d(d), _d(spam), len(spam), len(kind), _i(kind), _d(obs),
                              _d(prm), last_len, _d(th), _d(info))
    return th, st, info


# ---------------------------------------------------------------------------
# rollouts


def rollout(work, n_steps: int | None = None, prm=None, threads: int = 0, traj: bool = False):
    """Roll every instance of a Workload forward ``n_steps`` growth steps (default: to
    its full length).  Returns a dict of numpy arrays (see vo_rollout)."""
    prm = params() if prm is None else prm
    B = work.n_inst
    n_max = max(1, work.n_max)
    T = n_max if n_steps is None else int(n_steps)
    out = dict(
        theta=np.zeros((B, n_max)), tip=np.zeros((B, T, 3)), rho=np.zeros((B, T)),
        iters=np.zeros((B, T), np.int32), status=np.zeros((B, T), np.int32),
        ncont=np.zeros((B, T), np.int32), chash=np.zeros((B, T), np.uint64),
        maxpen=np.zeros((B, T)), stats=np.zeros((B, 6)), tiplen=np.zeros((B, T)))
    tr = np.zeros((B, T, n_max)) if traj else None
    inst_i, inst_d = _i32(work.inst_i), _f64(work.inst_d)
    spam, kind, obs = _f64(work.spam.reshape(-1, 4)), _i32(work.obs_kind), _f64(work.obs_d.reshape(-1, 4))
    lib().vo_rollout(B, _i(inst_i), _d(inst_d), _d(spam), _i(kind), _d(obs), _d(prm), T, threads,
                     n_max, _d(out["theta"]), _d(out["tip"]), _d(out["rho"]), _i(out["iters"]),
                     _i(out["status"]), _i(out["ncont"]),
                     out["chash"].ctypes.data_as(C.POINTER(C.c_uint64)), _d(out["maxpen"]),
                     _d(tr), _d(out["stats"]), _d(out["tiplen"]))
    if traj:
        out["traj"] = tr
    return out


def gradient(work, traj, weights=None, prm=None, threads: int = 0):
    """dL/d(pressure, s_start, s_end) of every sPAM for L = sum_t w_t |tip_t - goal|^2 on
    the equilibria in ``traj`` ([B][T][n_max], as rollout(traj=True) returns it); weights
    None = the last step only.  Returns (dP, ds0, ds1, loss[B])."""
    prm = params() if prm is None else prm
    B = work.n_inst
    traj = _f64(traj)
    T, n_max = traj.shape[1], traj.shape[2]
    ns = len(work.spam)
    dP, d0, d1, loss = np.zeros(ns), np.zeros(ns), np.zeros(ns), np.zeros(B)
    wts = None if weights is None else _f64(weights)
    lib().vo_gradient(B, _i(_i32(work.inst_i)), _d(_f64(work.inst_d)),
                      _d(_f64(work.spam.reshape(-1, 4))), _i(_i32(work.obs_kind)),
                      _d(_f64(work.obs_d.reshape(-1, 4))), _d(prm), T, n_max, _d(traj), _d(wts),
                      _d(_f64(work.goal)), threads, _d(dP), _d(d0), _d(d1), _d(loss))
    return dP, d0, d1, loss
