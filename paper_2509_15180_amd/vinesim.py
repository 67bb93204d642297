"""Python binding of libvinesim.so (include/vinesim.h).

Argument marshalling only: every step of the growth-step path runs in the HIP
library.  The binding fails loudly when the library is missing; it never falls
back to another implementation.

Names follow the C ABI: ``create`` -> vine_sim_create, ``VineSim.step`` ->
vine_sim_step, ``VineSim.rollout`` -> vine_sim_rollout, ``VineSim.rollout_graph`` ->
vine_sim_rollout_graph, ``VineSim.read`` ->
vine_sim_read, ``VineSim.grad`` -> vine_sim_grad, ``VineSim.close`` ->
vine_sim_destroy.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvinesim.so")

VINE_OK, VINE_EINVAL, VINE_ENOMEM, VINE_EDEVICE, VINE_ESTATE, VINE_ECAPACITY = 0, -1, -2, -3, -4, -5
ST_DONE, ST_CONVERGED, ST_MAXITER, ST_NODESCENT, ST_CAPACITY, ST_NONFINITE = -1, 0, 1, 2, 3, 4

FIELDS = dict(theta=(0, np.float64, "BN"), nlinks=(1, np.int32, "B"), tip=(2, np.float64, "BT3"),
              rho=(3, np.float64, "BT"), iters=(4, np.int32, "BT"), status=(5, np.int32, "BT"),
              ncont=(6, np.int32, "BT"), chash=(7, np.uint64, "BT"), maxpen=(8, np.float64, "BT"),
              traj=(9, np.float64, "BRN"), jevals=(10, np.float64, "B"),
              nsolves=(11, np.float64, "B"), cycles=(12, np.float64, "B"),
              negsteps=(13, np.float64, "B"), ckpt=(14, np.float64, "BCN"),
              time=(15, np.float64, "B"), tiplen=(16, np.float64, "BT"))

MAX_LINKS = 512
MAX_OBSTACLES = 128
MAX_SPAMS = 64


class VineError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vinesim error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("R_c", C.c_double), ("R_act", C.c_double), ("a_corr", C.c_double),
                ("eps_crit", C.c_double), ("k_c", C.c_double), ("tol", C.c_double),
                ("c_mu", C.c_double), ("step_max", C.c_double), ("armijo_c1", C.c_double),
                ("pd_shift", C.c_double), ("growth_stiffness", C.c_double), ("max_iter", C.c_int32),
                ("growth_substeps", C.c_int32), ("reserved", C.c_int32)]


class Instance(C.Structure):
    _fields_ = [("n_links", C.c_int32), ("spam_offset", C.c_int32), ("spam_count", C.c_int32),
                ("obs_offset", C.c_int32), ("obs_count", C.c_int32), ("reserved", C.c_int32),
                ("link_len", C.c_double), ("tube_radius", C.c_double),
                ("body_pressure", C.c_double), ("base_x", C.c_double), ("base_y", C.c_double),
                ("base_heading", C.c_double)]


class Spam(C.Structure):
    _fields_ = [("s_start", C.c_double), ("s_end", C.c_double), ("side", C.c_double),
                ("pressure", C.c_double)]


class Obstacle(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("cx", C.c_double),
                ("cy", C.c_double), ("a", C.c_double), ("b", C.c_double)]


EXPORTS = ("vine_params_default", "vine_sim_create", "vine_sim_step", "vine_sim_rollout",
           "vine_sim_rollout_graph", "vine_sim_tune_order",
           "vine_sim_reset", "vine_sim_read", "vine_sim_field_bytes", "vine_sim_dims",
           "vine_sim_destroy", "vine_sim_last_error", "vine_sim_spam_law", "vine_sim_trace",
           "vine_sim_trace_read", "vine_sim_grad", "vine_sim_grad_noalloc", "vine_sim_set_spams",
           "vine_sim_occupancy", "vine_sim_set_waves", "vine_sim_autotune", "vine_sim_set_head",
           "vine_sim_head",
           "vine_spam_synth", "vine_spam_solve", "vine_mlp_forward",
           "vine_server_create", "vine_server_submit", "vine_server_submit_from",
           "vine_server_tick", "vine_server_poll", "vine_server_result", "vine_server_release", "vine_server_stats", "vine_server_destroy",
           "vine_server_last_error")

_lib = None


def lib():
    """Load libvinesim.so (raises if it has not been built).  torch is imported first: the
    library and torch then share torch's HIP runtime (the same soname), whereas a library
    loaded first would bind the process, torch included, to the system's runtime, under
    which torch finds no GPU."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        import torch  # noqa: F401  (loads the process's HIP runtime)
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.vine_params_default.argtypes = [C.POINTER(Params)]
        L.vine_params_default.restype = None
        L.vine_sim_create.argtypes = [C.POINTER(Params), C.POINTER(Instance), C.c_int32,
                                      C.POINTER(Spam), C.c_int32, C.POINTER(Obstacle), C.c_int32,
                                      C.POINTER(vp)]
        L.vine_sim_create.restype = C.c_int32
        L.vine_sim_step.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp]
        L.vine_sim_step.restype = C.c_int32
        L.vine_sim_rollout.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp]
        L.vine_sim_rollout.restype = C.c_int32
        L.vine_sim_rollout_graph.argtypes = [vp, C.c_int32, C.c_int32, vp]
        L.vine_sim_rollout_graph.restype = C.c_int32
        L.vine_sim_tune_order.argtypes = [vp, vp]
        L.vine_sim_tune_order.restype = C.c_int32
        L.vine_sim_reset.argtypes = [vp, vp]
        L.vine_sim_reset.restype = C.c_int32
        L.vine_sim_read.argtypes = [vp, C.c_int32, vp, C.c_int32, vp]
        L.vine_sim_read.restype = C.c_int32
        L.vine_sim_field_bytes.argtypes = [vp, C.c_int32]
        L.vine_sim_field_bytes.restype = C.c_int64
        L.vine_sim_dims.argtypes = [vp, C.POINTER(C.c_int32)]
        L.vine_sim_dims.restype = None
        L.vine_sim_destroy.argtypes = [vp]
        L.vine_sim_destroy.restype = None
        L.vine_sim_last_error.argtypes = [vp]
        L.vine_sim_last_error.restype = C.c_char_p
        L.vine_sim_spam_law.argtypes = [vp, C.c_double, C.c_int32, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.vine_sim_spam_law.restype = C.c_int32
        dp_ = C.POINTER(C.c_double)
        L.vine_spam_synth.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_double, dp_,
                                      C.c_int32, dp_, C.c_int32, dp_, C.c_int32, C.c_double, dp_,
                                      dp_, vp]
        L.vine_spam_synth.restype = C.c_int32
        L.vine_spam_solve.argtypes = [C.POINTER(Params), C.c_int32, dp_, dp_, dp_, vp]
        L.vine_spam_solve.restype = C.c_int32
        L.vine_mlp_forward.argtypes = [dp_, C.c_int32, dp_, dp_, vp]
        L.vine_mlp_forward.restype = C.c_int32
        L.vine_sim_occupancy.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.vine_sim_occupancy.restype = C.c_int32
        L.vine_sim_set_waves.argtypes = [vp, C.POINTER(C.c_int32)]
        L.vine_sim_set_waves.restype = C.c_int32
        L.vine_sim_autotune.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                        C.POINTER(C.c_int32), vp]
        L.vine_sim_autotune.restype = C.c_int32
        L.vine_sim_set_head.argtypes = [vp, C.c_double, C.c_int32, vp]
        L.vine_sim_set_head.restype = C.c_int32
        L.vine_sim_head.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.vine_sim_head.restype = C.c_int32
        L.vine_sim_trace.argtypes = [vp, C.c_int32, C.c_int32]
        L.vine_sim_trace.restype = C.c_int32
        L.vine_sim_trace_read.argtypes = [vp, C.POINTER(C.c_double), C.c_int32]
        L.vine_sim_trace_read.restype = C.c_int32
        L.vine_sim_grad.argtypes = [vp] * 9
        L.vine_sim_grad.restype = C.c_int32
        L.vine_sim_grad_noalloc.argtypes = [vp] * 9
        L.vine_sim_grad_noalloc.restype = C.c_int32
        L.vine_sim_set_spams.argtypes = [vp, C.POINTER(Spam), C.c_int32, vp]
        L.vine_sim_set_spams.restype = C.c_int32
        L.vine_server_create.argtypes = [C.POINTER(Params), C.c_int32, C.c_int64, C.c_int32,
                                         C.c_int32, C.c_int32, C.POINTER(vp)]
        L.vine_server_create.restype = C.c_int32
        L.vine_server_submit.argtypes = [vp, C.c_int64, C.POINTER(Instance), C.c_int32,
                                         C.POINTER(Spam), C.c_int32, C.POINTER(Obstacle),
                                         C.c_int32]
        L.vine_server_submit.restype = C.c_int32
        L.vine_server_submit_from.argtypes = [vp, C.c_int64, C.POINTER(Instance), C.c_int32,
                                              C.POINTER(Spam), C.c_int32, C.POINTER(Obstacle),
                                              C.c_int32, C.POINTER(C.c_int32),
                                              C.POINTER(C.c_double)]
        L.vine_server_submit_from.restype = C.c_int32
        L.vine_server_tick.argtypes = [vp]
        L.vine_server_tick.restype = C.c_int32
        L.vine_server_poll.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.c_int32]
        L.vine_server_poll.restype = C.c_int32
        L.vine_server_result.argtypes = [vp, C.c_int64, C.c_int32, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]
        L.vine_server_result.restype = C.c_int32
        L.vine_server_release.argtypes = [vp, C.c_int64]
        L.vine_server_release.restype = C.c_int32
        L.vine_server_stats.argtypes = [vp, C.POINTER(C.c_int64)]
        L.vine_server_stats.restype = None
        L.vine_server_destroy.argtypes = [vp]
        L.vine_server_destroy.restype = None
        L.vine_server_last_error.argtypes = [vp]
        L.vine_server_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def default_params(**over) -> Params:
    p = Params()
    lib().vine_params_default(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def occupancy(waves: int = 2):
    """(robots per compute unit for the 64-, 128-, 256- and 512-link classes, compute units)
    of the current device with `waves` waves per robot (vine_sim_occupancy)."""
    per = (C.c_int32 * 4)()
    cus = C.c_int32()
    rc = lib().vine_sim_occupancy(waves, per, C.byref(cus))
    if rc != VINE_OK:
        raise VineError(rc, lib().vine_sim_last_error(None).decode())
    return [int(x) for x in per], int(cus.value)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def _struct_dtype(S):
    """A numpy dtype laid out like the ctypes Structure S (field offsets and size)."""
    fmt = {C.c_int32: "<i4", C.c_double: "<f8"}
    return np.dtype({"names": [f for f, _ in S._fields_],
                     "formats": [fmt[t] for _, t in S._fields_],
                     "offsets": [getattr(S, f).offset for f, _ in S._fields_],
                     "itemsize": C.sizeof(S)})


def _pack(work):
    """The Workload's arrays as the C structs (numpy buffers viewed as ctypes arrays; a
    zero count keeps one zeroed element so that every pointer is valid)."""
    B = work.n_inst
    ia = np.zeros(B, _struct_dtype(Instance))
    for k, f in enumerate(("n_links", "spam_offset", "spam_count", "obs_offset", "obs_count")):
        ia[f] = work.inst_i[:, k]
    for k, f in enumerate(("link_len", "tube_radius", "body_pressure", "base_x", "base_y",
                           "base_heading")):
        ia[f] = work.inst_d[:, k]
    inst = (Instance * B).from_buffer(ia) if B else (Instance * 0)()
    ns, no = len(work.spam), len(work.obs_kind)
    sa = np.zeros((max(1, ns), 4))
    sa[:ns] = work.spam
    spams = (Spam * max(1, ns)).from_buffer(sa)
    oa = np.zeros(max(1, no), _struct_dtype(Obstacle))
    oa["kind"][:no] = work.obs_kind
    for k, f in enumerate(("cx", "cy", "a", "b")):
        oa[f][:no] = work.obs_d[:, k]
    obs = (Obstacle * max(1, no)).from_buffer(oa)
    return inst, B, spams, ns, obs, no


def spam_synth(pressures, unit_lengths, targets, tol: float, link_len: float, tube_radius: float,
               body_pressure: float, params: Params | None = None, stream=None,
               want_angles: bool = True):
    """Actuator synthesis (vine_spam_synth): (designs [n][3] = (P, l0, rest angle) or zeros,
    rest angles [n_pressures][n_lengths] or None)."""
    dp = C.POINTER(C.c_double)
    P = np.ascontiguousarray(pressures, np.float64)
    Lu = np.ascontiguousarray(unit_lengths, np.float64)
    t = np.ascontiguousarray(np.atleast_1d(targets), np.float64)
    des = np.zeros((len(t), 3))
    ang = np.zeros((len(P), len(Lu))) if want_angles else None
    prm = params if params is not None else default_params()
    rc = lib().vine_spam_synth(C.byref(prm), float(link_len), float(tube_radius),
                               float(body_pressure), P.ctypes.data_as(dp), len(P),
                               Lu.ctypes.data_as(dp), len(Lu), t.ctypes.data_as(dp), len(t),
                               float(tol), des.ctypes.data_as(dp),
                               ang.ctypes.data_as(dp) if ang is not None else None,
                               _stream_ptr(stream))
    if rc != VINE_OK:
        raise VineError(rc, lib().vine_sim_last_error(None).decode())
    return des, ang


def spam_solve(eps, unit_lengths, params: Params | None = None, stream=None):
    """The sPAM state of each strain (vine_spam_solve): [n][4] = (m, phi, G, strain)."""
    dp = C.POINTER(C.c_double)
    e = np.ascontiguousarray(np.atleast_1d(eps), np.float64)
    Lu = np.ascontiguousarray(np.broadcast_to(unit_lengths, e.shape), np.float64)
    out = np.zeros((len(e), 4))
    prm = params if params is not None else default_params()
    rc = lib().vine_spam_solve(C.byref(prm), len(e), e.ctypes.data_as(dp), Lu.ctypes.data_as(dp),
                               out.ctypes.data_as(dp), _stream_ptr(stream))
    if rc != VINE_OK:
        raise VineError(rc, lib().vine_sim_last_error(None).decode())
    return out


def mlp_forward(weights, x, stream=None):
    """The 2-32-2 ReLU surrogate on the device (vine_mlp_forward): y [n][2]."""
    dp = C.POINTER(C.c_double)
    w = np.ascontiguousarray(weights, np.float64).ravel()
    if w.size != 162:
        raise ValueError("the surrogate has 162 weights")
    xx = np.ascontiguousarray(x, np.float64).reshape(-1, 2)
    y = np.zeros_like(xx)
    rc = lib().vine_mlp_forward(w.ctypes.data_as(dp), len(xx), xx.ctypes.data_as(dp),
                                y.ctypes.data_as(dp), _stream_ptr(stream))
    if rc != VINE_OK:
        raise VineError(rc, lib().vine_sim_last_error(None).decode())
    return y


class VineSim:
    """One handle of the C ABI (vine_sim_create ... vine_sim_destroy)."""

    def __init__(self, work, params: Params | None = None, **over):
        L = lib()
        self._p = params if params is not None else default_params(**over)
        inst, B, spams, ns, obs, no = _pack(work)
        h = C.c_void_p()
        rc = L.vine_sim_create(C.byref(self._p), inst, B, spams, ns, obs, no, C.byref(h))
        if rc != VINE_OK:
            raise VineError(rc, L.vine_sim_last_error(None).decode())
        self.h = h
        dims = (C.c_int32 * 3)()
        L.vine_sim_dims(h, dims)
        self.B, self.T, self.N = int(dims[0]), int(dims[1]), int(dims[2])
        self.S = int(len(work.spam))
        self.rec_every = 0   # as last passed with a nonzero value (shape of "traj")
        self.ckpt_every = 0  # likewise for "ckpt"

    def _check(self, rc):
        if rc != VINE_OK:
            raise VineError(rc, lib().vine_sim_last_error(self.h).decode())

    def _note(self, record_every, ckpt_every):
        if record_every:
            self.rec_every = int(record_every)
        if ckpt_every:
            self.ckpt_every = int(ckpt_every)

    def step(self, n_steps: int, record_every: int = 0, ckpt_every: int = 0, stream=None):
        self._check(lib().vine_sim_step(self.h, int(n_steps), int(record_every), int(ckpt_every),
                                        _stream_ptr(stream)))
        self._note(record_every, ckpt_every)

    def rollout(self, n_steps: int = -1, record_every: int = 0, ckpt_every: int = 0,
                stream=None):
        self._check(lib().vine_sim_rollout(self.h, int(n_steps), int(record_every),
                                           int(ckpt_every), _stream_ptr(stream)))
        self._note(record_every, ckpt_every)

    def rollout_graph(self, record_every: int = 0, ckpt_every: int = 0, stream=None):
        """Reset and roll every robot out to full length as one captured HIP graph
        (captured on the first call for each (record_every, ckpt_every), replayed
        afterwards)."""
        self._check(lib().vine_sim_rollout_graph(self.h, int(record_every), int(ckpt_every),
                                                 _stream_ptr(stream)))
        self._note(record_every, ckpt_every)

    def tune_order(self, stream=None):
        """Launch order by the cycles each robot measured since the last reset (longest first)."""
        self._check(lib().vine_sim_tune_order(self.h, _stream_ptr(stream)))

    def set_waves(self, waves):
        """Waves per robot (1, 2 or 4) of the 64-, 128-, 256- and 512-link classes."""
        w = (C.c_int32 * 4)(*[int(x) for x in waves])
        self._check(lib().vine_sim_set_waves(self.h, w))

    def set_head(self, fraction: float, waves: int = 4, stream=None):
        """Robots at or above `fraction` of the slowest's measured cycles in a launch of
        their own with `waves` per robot (vine_sim_set_head); 0: none."""
        self._check(lib().vine_sim_set_head(self.h, float(fraction), int(waves),
                                            _stream_ptr(stream)))

    def head(self) -> dict:
        """The head as set, and the autotuner's whole-batch times (vine_sim_head)."""
        f, w, n = C.c_double(), C.c_int32(), C.c_int32()
        ms = (C.c_double * 6)()
        self._check(lib().vine_sim_head(self.h, C.byref(f), C.byref(w), C.byref(n), ms))
        fr = ("0", "1/2", "1/4")
        return {"fraction": f.value, "waves": w.value, "robots": n.value,
                "ms_whole_batch": {
                    "fastest_alone": {fr[j]: ms[j] for j in range(3)},
                    "two_waves": {fr[j]: ms[3 + j] for j in range(3)}}}

    def autotune(self, stream=None) -> dict:
        """Measure 1, 2 and 4 waves per robot for each class, then the whole batch with
        and without a head of the slowest robots, keep the fastest (vine_sim_autotune);
        the robots end reset."""
        w = (C.c_int32 * 4)()
        ms = (C.c_double * 12)()
        cached = C.c_int32()
        self._check(lib().vine_sim_autotune(self.h, w, ms, C.byref(cached), _stream_ptr(stream)))
        return {"waves": [int(x) for x in w], "cached": bool(cached.value),
                "ms_one_wave": [ms[3 * c] for c in range(4)],
                "ms_two_waves": [ms[3 * c + 1] for c in range(4)],
                "ms_four_waves": [ms[3 * c + 2] for c in range(4)],
                "head": self.head()}

    def reset(self, stream=None):
        self._check(lib().vine_sim_reset(self.h, _stream_ptr(stream)))

    def field_shape(self, name: str):
        code, dt, shp = FIELDS[name]
        ceil = lambda a, b: -(-a // b) if b else 0
        dims = dict(B=self.B, T=self.T, N=self.N, R=ceil(self.T, self.rec_every),
                    C=ceil(self.T, self.ckpt_every), **{"3": 3})
        return tuple(dims[c] for c in shp), dt, code

    def read(self, name: str, out=None, stream=None):
        """Copy a field to a new numpy array, or into ``out`` (numpy array or device
        torch tensor of the right size)."""
        shape, dt, code = self.field_shape(name)
        if out is None:
            out = np.empty(shape, dt)
        if isinstance(out, np.ndarray):
            assert out.nbytes >= lib().vine_sim_field_bytes(self.h, code)
            self._check(lib().vine_sim_read(self.h, code, out.ctypes.data_as(C.c_void_p), 0,
                                            _stream_ptr(stream)))
            return out
        # torch tensor on the device
        assert out.is_cuda and out.numel() * out.element_size() >= lib().vine_sim_field_bytes(
            self.h, code)
        self._check(lib().vine_sim_read(self.h, code, C.c_void_p(out.data_ptr()), 1,
                                        _stream_ptr(stream)))
        return out

    def read_all(self, traj: bool = False) -> dict:
        names = [k for k in FIELDS if k not in ("traj", "ckpt")] + (["traj"] if traj else [])
        return {k: self.read(k) for k in names}

    def spam_law(self, l: float, eps):
        eps = np.ascontiguousarray(np.atleast_1d(eps), np.float64)
        G, dG, IG = np.zeros_like(eps), np.zeros_like(eps), np.zeros_like(eps)
        dp = C.POINTER(C.c_double)
        self._check(lib().vine_sim_spam_law(self.h, float(l), len(eps), eps.ctypes.data_as(dp),
                                            G.ctypes.data_as(dp), dG.ctypes.data_as(dp),
                                            IG.ctypes.data_as(dp)))
        return G, dG, IG

    def trace(self, robot: int, capacity: int = 100000):
        """Record the solver decisions of one robot on later step/rollout calls."""
        self._check(lib().vine_sim_trace(self.h, int(robot), int(capacity)))
        self._trace_cap = int(capacity)

    def trace_read(self):
        buf = np.zeros((self._trace_cap, 10))
        n = lib().vine_sim_trace_read(self.h, buf.ctypes.data_as(C.POINTER(C.c_double)),
                                      self._trace_cap)
        if n < 0:
            self._check(n)
        return buf[:n]

    def grad(self, goal, weights=None, stream=None, noalloc: bool = False):
        """vine_sim_grad (vine_sim_grad_noalloc with ``noalloc``) on device tensors.
        ``goal`` [B][2] and ``weights`` [T] (or None: the current state alone) may be numpy
        arrays or torch tensors; they are staged as float64 device tensors.  Returns device
        tensors (dL_dP, dL_ds_start, dL_ds_end, loss[B], adj_status[B]), valid once
        ``stream`` has been synchronised."""
        import torch

        dev = torch.device("cuda", torch.cuda.current_device())

        def staged(x, shape):
            t = torch.as_tensor(x, dtype=torch.float64).to(dev).contiguous()
            assert tuple(t.shape) == shape, (tuple(t.shape), shape)
            return t

        g = staged(goal, (self.B, 2))
        w = None if weights is None else staged(weights, (self.T,))
        S = max(self.S, 1)
        dP, d0, d1 = (torch.empty(S, dtype=torch.float64, device=dev) for _ in range(3))
        loss = torch.empty(self.B, dtype=torch.float64, device=dev)
        st = torch.empty(self.B, dtype=torch.int32, device=dev)
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        if stream is None:
            stream = torch.cuda.current_stream()
        fn = lib().vine_sim_grad_noalloc if noalloc else lib().vine_sim_grad
        self._check(fn(self.h, ptr(g), ptr(w), ptr(dP), ptr(d0), ptr(d1), ptr(loss), ptr(st),
                       _stream_ptr(stream)))
        self._keep = (g, w)  # inputs stay alive until the caller synchronises
        return dP[:self.S], d0[:self.S], d1[:self.S], loss, st

    def set_spams(self, spam, stream=None):
        """vine_sim_set_spams: new sPAM records [S][4] (s_start, s_end, side, pressure)."""
        spam = np.asarray(spam, np.float64).reshape(-1, 4)
        arr = (Spam * max(1, len(spam)))()
        for i, row in enumerate(spam):
            arr[i] = Spam(*(float(x) for x in row))
        self._check(lib().vine_sim_set_spams(self.h, arr, len(spam), _stream_ptr(stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().vine_sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class VineServer:
    """vine_server_*: continuous batching of rollout requests (one handle).  hbm_bytes:
    the device-memory budget of the robot pools (default: room for ``slots`` robots at
    the bounds)."""

    def __init__(self, slots: int, max_links: int = MAX_LINKS, max_obstacles: int = MAX_OBSTACLES,
                 max_spams: int = 8, hbm_bytes: int | None = None, params: Params | None = None,
                 **over):
        L = lib()
        self._p = params if params is not None else default_params(**over)
        if hbm_bytes is None:
            hbm_bytes = int(slots) * (92 * int(max_links) + 36 * int(max_obstacles) + 148)
        h = C.c_void_p()
        rc = L.vine_server_create(C.byref(self._p), int(slots), int(hbm_bytes), int(max_links),
                                  int(max_obstacles), int(max_spams), C.byref(h))
        if rc != VINE_OK:
            raise VineError(rc, L.vine_server_last_error(None).decode())
        self.h = h
        self.n_links = {}

    def _check(self, rc):
        if rc < 0:
            raise VineError(rc, lib().vine_server_last_error(self.h).decode())
        return rc

    def submit(self, request_id: int, work):
        """Queue every instance of a Workload as one request."""
        inst, B, spams, ns, obs, no = _pack(work)
        self._check(lib().vine_server_submit(self.h, int(request_id), inst, B, spams, ns, obs, no))
        self.n_links[int(request_id)] = [int(v) for v in work.inst_i[:, 0]]

    def submit_each(self, first_id: int, work, start=None):
        """Queue instance b of a Workload as its own request first_id + b (so that poll
        reports each robot's worst status); the arrays are packed once and each call
        copies only the robot's own sPAMs and obstacles.  start: None, or per robot the
        joint angles it starts with (an empty array: from zero), as
        vine_server_submit_from."""
        inst, B, spams, ns, obs, no = _pack(work)
        L = lib()
        for b in range(B):
            rid = int(first_id) + b
            th = None if start is None else np.ascontiguousarray(start[b], np.float64)
            if th is None or th.size == 0:
                rc = L.vine_server_submit(self.h, rid, C.byref(inst[b]), 1, spams, ns, obs, no)
            else:
                cnt = C.c_int32(th.size)
                rc = L.vine_server_submit_from(self.h, rid, C.byref(inst[b]), 1, spams, ns, obs,
                                               no, C.byref(cnt),
                                               th.ctypes.data_as(C.POINTER(C.c_double)))
            self._check(rc)
            self.n_links[rid] = [int(work.inst_i[b, 0])]

    def tick(self) -> int:
        """One non-blocking scheduling round; the number of requests it completed."""
        return self._check(lib().vine_server_tick(self.h))

    def poll(self, cap: int = 4096):
        ids = (C.c_int64 * cap)()
        st = (C.c_int32 * cap)()
        k = self._check(lib().vine_server_poll(self.h, ids, st, cap))
        return [(int(ids[i]), int(st[i])) for i in range(k)]

    def result(self, request_id: int, robot: int):
        tip = (C.c_double * 3)()
        n = self.n_links[int(request_id)][robot]
        th = np.zeros(n)
        self._check(lib().vine_server_result(self.h, int(request_id), int(robot), tip,
                                             th.ctypes.data_as(C.POINTER(C.c_double))))
        return np.array(tip[:]), th

    def release(self, request_id: int):
        self._check(lib().vine_server_release(self.h, int(request_id)))
        self.n_links.pop(int(request_id), None)

    def stats(self) -> dict:
        out = (C.c_int64 * 8)()
        lib().vine_server_stats(self.h, out)
        return dict(queued=out[0], active=out[1], completed=out[2], joint_updates=out[3],
                    rows_used=out[4], rows=out[5], hbm_bytes=out[6], groups=out[7])

    def close(self):
        if getattr(self, "h", None):
            lib().vine_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
