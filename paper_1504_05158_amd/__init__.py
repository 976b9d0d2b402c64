"""Python binding of the MI355X (gfx950) multi-swarm PSO library for the QAP.

Argument marshalling only: every step of the method runs in the HIP kernels of
``libqapswarm.so`` (built in-tree by ``build.py``).  The C entry points of
``include/qap_swarm.h`` are exposed under the same names; ``Swarm`` wraps a
handle with numpy in/out.  PyTorch, when present, only supplies the HIP stream.
There is no CPU fallback: importing the binding without the built library, or
calling it without a GPU, raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqapswarm.so")

QAP_OK = 0
QAP_ERR_INVALID_ARG = -1
QAP_ERR_RANGE = -2
QAP_ERR_NOMEM = -3
QAP_ERR_DEVICE = -4
QAP_ERR_UNSUPPORTED = -5
QAP_SV_RAW, QAP_SV_NORM = 0, 1
QAP_INDEPENDENT, QAP_MIGRATION = 0, 1
QAP_PATH_AUTO, QAP_PATH_INT8_MFMA, QAP_PATH_INT32, QAP_PATH_SPLIT_MFMA = 0, 1, 2, 3
QAP_ENGINE_FUSED, QAP_ENGINE_PLAIN = 0, 1
QAP_MAX_CHAINS = 4
QAP_SPLIT_SWARMS, QAP_SPLIT_INSTANCES, QAP_SPLIT_CLASSES = 0, 1, 2

EXPORTS = ["qap_swarm_init", "qap_swarm_init_batch", "qap_swarm_step", "qap_swarm_sync", "qap_swarm_best",
           "qap_swarm_swarm_bests", "qap_swarm_get_state", "qap_swarm_set_state", "qap_swarm_eval",
           "qap_swarm_deltas", "qap_swarm_path", "qap_swarm_graph", "qap_swarm_stats", "qap_swarm_profile",
           "qap_swarm_destroy", "qap_swarm_strerror", "qap_swarm_fail_alloc", "qap_swarm_live_allocations",
           "qap_swarm_stats_noalloc", "qap_swarm_get_plan", "qap_swarm_set_plan", "qap_swarm_tune",
           "qap_swarm_history_start", "qap_swarm_history_stop", "qap_swarm_history_read"]
STAGES = ["sx", "velocity", "goal_delta", "fused", "bests"]


class qap_instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("F", ctypes.POINTER(ctypes.c_int32)), ("D", ctypes.POINTER(ctypes.c_int32))]


class qap_params(ctypes.Structure):
    _fields_ = [("num_swarms", ctypes.c_int32), ("particles_per_swarm", ctypes.c_int32),
                ("c1", ctypes.c_float), ("c2", ctypes.c_float), ("c3", ctypes.c_float), ("vmax", ctypes.c_float),
                ("velocity_kernel", ctypes.c_int32), ("st_depth", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("migration_factor", ctypes.c_float), ("migration_period", ctypes.c_int32),
                ("local_search", ctypes.c_int32), ("delta_path", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("stream", ctypes.c_void_p), ("stream_groups", ctypes.c_int32),
                ("sx_procedure", ctypes.c_int32)]


class qap_plan(ctypes.Structure):
    _fields_ = [("stream_chains", ctypes.c_int32), ("split", ctypes.c_int32), ("iters_per_graph", ctypes.c_int32),
                ("ms_per_iteration", ctypes.c_float)]


class qap_state(ctypes.Structure):
    _fields_ = [("V", ctypes.POINTER(ctypes.c_float)), ("X", ctypes.POINTER(ctypes.c_int32)),
                ("PL", ctypes.POINTER(ctypes.c_int32)), ("goal", ctypes.POINTER(ctypes.c_int64)),
                ("goalPL", ctypes.POINTER(ctypes.c_int64)), ("PG", ctypes.POINTER(ctypes.c_int32)),
                ("goalPG", ctypes.POINTER(ctypes.c_int64)), ("best_perm", ctypes.POINTER(ctypes.c_int32)),
                ("best_goal", ctypes.c_int64), ("best_iter", ctypes.c_int32), ("best_swarm", ctypes.c_int32),
                ("best_particle", ctypes.c_int32), ("iteration", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libqapswarm.so is not built: run `python paper_1504_05158_amd/build.py` "
                          "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.qap_swarm_init.argtypes = [P(qap_instance), P(qap_params), P(vp)]
    L.qap_swarm_init_batch.argtypes = [P(qap_instance), P(qap_params), ctypes.c_int32, P(vp)]
    L.qap_swarm_step.argtypes = [vp, ctypes.c_int32]
    L.qap_swarm_sync.argtypes = [vp]
    L.qap_swarm_best.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_int32), P(ctypes.c_int32)]
    L.qap_swarm_swarm_bests.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int64)]
    L.qap_swarm_get_state.argtypes = [vp, ctypes.c_int32, P(qap_state)]
    L.qap_swarm_set_state.argtypes = [vp, ctypes.c_int32, P(qap_state)]
    L.qap_swarm_eval.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int32), ctypes.c_int32, P(ctypes.c_int64),
                                 P(ctypes.c_int64)]
    L.qap_swarm_deltas.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_int32)]
    L.qap_swarm_fail_alloc.argtypes = [ctypes.c_int32]
    L.qap_swarm_live_allocations.argtypes = []
    L.qap_swarm_live_allocations.restype = ctypes.c_int64
    L.qap_swarm_path.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32)]
    L.qap_swarm_graph.argtypes = [vp, P(ctypes.c_int32), P(ctypes.c_int32)]
    L.qap_swarm_stats.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int64),
                                  P(ctypes.c_int64), ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                  P(ctypes.c_int64), P(ctypes.c_int64)]
    L.qap_swarm_stats_noalloc.argtypes = L.qap_swarm_stats.argtypes
    L.qap_swarm_history_start.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32),
                                          ctypes.c_int32, ctypes.c_int64, ctypes.c_int64]
    L.qap_swarm_history_stop.argtypes = [vp, ctypes.c_int32]
    L.qap_swarm_history_read.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32),
                                         P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64)]
    L.qap_swarm_get_plan.argtypes = [vp, P(qap_plan)]
    L.qap_swarm_set_plan.argtypes = [vp, P(qap_plan)]
    L.qap_swarm_tune.argtypes = [vp, ctypes.c_int32, P(qap_plan)]
    L.qap_swarm_profile.argtypes = [vp, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_int64)]
    L.qap_swarm_destroy.argtypes = [vp]
    L.qap_swarm_destroy.restype = None
    L.qap_swarm_strerror.argtypes = [ctypes.c_int]
    L.qap_swarm_strerror.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("qap_swarm_destroy", "qap_swarm_strerror", "qap_swarm_live_allocations"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def __getattr__(name):
    # the C entry points under their own names: paper_1504_05158_amd.qap_swarm_step(...)
    if name in EXPORTS:
        return getattr(load_library(), name)
    raise AttributeError(name)


class QapError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = load_library().qap_swarm_strerror(code).decode()
        super().__init__("%s failed: %s (%d)" % (what, msg, code))


def _check(rc: int, what: str) -> None:
    if rc != QAP_OK:
        raise QapError(rc, what)


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


_ENGINES = {"fused": QAP_ENGINE_FUSED, "plain": QAP_ENGINE_PLAIN}
_PATHS = {"auto": QAP_PATH_AUTO, "int8": QAP_PATH_INT8_MFMA, "int32": QAP_PATH_INT32, "split": QAP_PATH_SPLIT_MFMA}


def make_params(*, num_swarms, particles_per_swarm, c1=0.8, c2=0.5, c3=0.5, vmax=1.0, norm=True, depth=2,
                migration=False, migration_factor=0.0, migration_period=1, local_search=True, delta_path="auto",
                engine="fused", seed=1, stream=None, stream_groups=0, sx="second_target") -> qap_params:
    p = qap_params()
    p.num_swarms = int(num_swarms)
    p.particles_per_swarm = int(particles_per_swarm)
    p.c1, p.c2, p.c3, p.vmax = float(c1), float(c2), float(c3), float(vmax)
    p.velocity_kernel = QAP_SV_NORM if norm else QAP_SV_RAW
    p.st_depth = int(depth)
    p.mode = QAP_MIGRATION if migration else QAP_INDEPENDENT
    p.migration_factor = float(migration_factor)
    p.migration_period = int(migration_period)
    p.local_search = int(local_search)  # True -> 1 exchange per particle-iteration
    p.delta_path = _PATHS[delta_path] if isinstance(delta_path, str) else int(delta_path)
    p.engine = _ENGINES[engine] if isinstance(engine, str) else int(engine)
    p.seed = int(seed)
    p.stream = stream
    p.stream_groups = int(stream_groups)
    p.sx_procedure = {"second_target": 0, "pick_column": 1}[sx] if isinstance(sx, str) else int(sx)
    return p


def _torch_stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # a torch.cuda.Stream


class Swarm:
    """One handle over one or more QAP instances (batched when several)."""

    def __init__(self, instances, params):
        if isinstance(instances, tuple):
            instances, params = [instances], [params]
        self._keep = []
        insts = (qap_instance * len(instances))()
        for k, (F, D) in enumerate(instances):
            F = np.ascontiguousarray(F, dtype=np.int32)
            D = np.ascontiguousarray(D, dtype=np.int32)
            if F.ndim != 2 or F.shape[0] != F.shape[1] or D.shape != F.shape:
                raise ValueError("F and D must be n x n")
            self._keep += [F, D]
            insts[k].n = F.shape[0]
            insts[k].F = _ptr(F, ctypes.c_int32)
            insts[k].D = _ptr(D, ctypes.c_int32)
        prms = (qap_params * len(params))(*params)
        self.ns = [int(insts[k].n) for k in range(len(instances))]
        self.ms = [int(p.num_swarms) for p in params]
        self.Ss = [int(p.particles_per_swarm) for p in params]
        h = ctypes.c_void_p()
        L = load_library()
        _check(L.qap_swarm_init_batch(insts, prms, len(instances), ctypes.byref(h)), "qap_swarm_init_batch")
        self.h = h

    @classmethod
    def create(cls, F, D, stream=None, **kw):
        return cls((F, D), make_params(stream=_torch_stream_ptr(stream), **kw))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load_library().qap_swarm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, iterations: int = 1) -> None:
        _check(load_library().qap_swarm_step(self.h, int(iterations)), "qap_swarm_step")

    def sync(self) -> None:
        _check(load_library().qap_swarm_sync(self.h), "qap_swarm_sync")

    def best(self, instance: int = 0):
        n = self.ns[instance]
        g = ctypes.c_int64()
        it = ctypes.c_int32()
        perm = np.zeros(n, np.int32)
        _check(load_library().qap_swarm_best(self.h, instance, ctypes.byref(g), _ptr(perm, ctypes.c_int32),
                                             ctypes.byref(it)), "qap_swarm_best")
        return int(g.value), perm, int(it.value)

    def swarm_bests(self, instance: int = 0) -> np.ndarray:
        out = np.zeros(self.ms[instance], np.int64)
        _check(load_library().qap_swarm_swarm_bests(self.h, instance, _ptr(out, ctypes.c_int64)),
               "qap_swarm_swarm_bests")
        return out

    def get_state(self, instance: int = 0) -> dict:
        n, m, S = self.ns[instance], self.ms[instance], self.Ss[instance]
        P = m * S
        st = dict(V=np.zeros((P, n, n), np.float32), X=np.zeros((P, n), np.int32), PL=np.zeros((P, n), np.int32),
                  goal=np.zeros(P, np.int64), goalPL=np.zeros(P, np.int64), PG=np.zeros((m, n), np.int32),
                  goalPG=np.zeros(m, np.int64), best_perm=np.zeros(n, np.int32))
        s = qap_state()
        s.V = _ptr(st["V"], ctypes.c_float)
        s.X = _ptr(st["X"], ctypes.c_int32)
        s.PL = _ptr(st["PL"], ctypes.c_int32)
        s.goal = _ptr(st["goal"], ctypes.c_int64)
        s.goalPL = _ptr(st["goalPL"], ctypes.c_int64)
        s.PG = _ptr(st["PG"], ctypes.c_int32)
        s.goalPG = _ptr(st["goalPG"], ctypes.c_int64)
        s.best_perm = _ptr(st["best_perm"], ctypes.c_int32)
        _check(load_library().qap_swarm_get_state(self.h, instance, ctypes.byref(s)), "qap_swarm_get_state")
        st["best_goal"] = int(s.best_goal)
        st["best_info"] = np.array([s.best_iter, s.best_swarm, s.best_particle], np.int32)
        st["t"] = int(s.iteration)
        return st

    def set_state(self, st: dict, instance: int = 0) -> None:
        arrs = dict(V=np.ascontiguousarray(st["V"], np.float32), X=np.ascontiguousarray(st["X"], np.int32),
                    PL=np.ascontiguousarray(st["PL"], np.int32), goal=np.ascontiguousarray(st["goal"], np.int64),
                    goalPL=np.ascontiguousarray(st["goalPL"], np.int64),
                    PG=np.ascontiguousarray(st["PG"], np.int32),
                    goalPG=np.ascontiguousarray(st["goalPG"], np.int64),
                    best_perm=np.ascontiguousarray(st["best_perm"], np.int32))
        s = qap_state()
        s.V = _ptr(arrs["V"], ctypes.c_float)
        s.X = _ptr(arrs["X"], ctypes.c_int32)
        s.PL = _ptr(arrs["PL"], ctypes.c_int32)
        s.goal = _ptr(arrs["goal"], ctypes.c_int64)
        s.goalPL = _ptr(arrs["goalPL"], ctypes.c_int64)
        s.PG = _ptr(arrs["PG"], ctypes.c_int32)
        s.goalPG = _ptr(arrs["goalPG"], ctypes.c_int64)
        s.best_perm = _ptr(arrs["best_perm"], ctypes.c_int32)
        s.best_goal = int(st["best_goal"])
        bi = st.get("best_info", (0, 0, 0))
        s.best_iter, s.best_swarm, s.best_particle = int(bi[0]), int(bi[1]), int(bi[2])
        s.iteration = int(st["t"])
        _check(load_library().qap_swarm_set_state(self.h, instance, ctypes.byref(s)), "qap_swarm_set_state")

    def eval(self, perms, deltas: bool = False, instance: int = 0):
        perms = np.ascontiguousarray(perms, np.int32)
        if perms.ndim == 1:
            perms = perms[None]
        cnt, n = perms.shape
        goals = np.zeros(cnt, np.int64)
        dl = np.zeros((cnt, n, n), np.int64) if deltas else None
        _check(load_library().qap_swarm_eval(self.h, instance, _ptr(perms, ctypes.c_int32), cnt,
                                             _ptr(goals, ctypes.c_int64),
                                             _ptr(dl, ctypes.c_int64) if deltas else None), "qap_swarm_eval")
        return (goals, dl) if deltas else goals

    def deltas(self, particle: int, instance: int = 0):
        """Pair-exchange delta matrix [n, n] of the particle's S_x output in the
        last step (before its exchanges), and that permutation."""
        n = self.ns[instance]
        out = np.zeros((n, n), np.int64)
        perm = np.zeros(n, np.int32)
        _check(load_library().qap_swarm_deltas(self.h, instance, int(particle), _ptr(out, ctypes.c_int64),
                                               _ptr(perm, ctypes.c_int32)), "qap_swarm_deltas")
        return out, perm

    def path(self, instance: int = 0):
        p = ctypes.c_int32()
        s = ctypes.c_int32()
        _check(load_library().qap_swarm_path(self.h, instance, ctypes.byref(p), ctypes.byref(s)), "qap_swarm_path")
        return {QAP_PATH_INT8_MFMA: "int8", QAP_PATH_INT32: "int32", QAP_PATH_SPLIT_MFMA: "split"}[p.value], bool(s.value)

    def plan(self) -> dict:
        """The launch plan: stream chains, split (0 swarms, 1 instances), iterations per graph (0 eager)."""
        p = qap_plan()
        _check(load_library().qap_swarm_get_plan(self.h, ctypes.byref(p)), "qap_swarm_get_plan")
        return dict(stream_chains=p.stream_chains, split=p.split, iters_per_graph=p.iters_per_graph)

    def set_plan(self, stream_chains: int, split: int = 0, iters_per_graph: int = 8) -> None:
        p = qap_plan(int(stream_chains), int(split), int(iters_per_graph), 0.0)
        _check(load_library().qap_swarm_set_plan(self.h, ctypes.byref(p)), "qap_swarm_set_plan")

    def tune(self, trial_iterations: int = 16) -> dict:
        """Time every launch plan on this handle's work, keep the fastest, return to iteration 0."""
        p = qap_plan()
        _check(load_library().qap_swarm_tune(self.h, int(trial_iterations), ctypes.byref(p)), "qap_swarm_tune")
        return dict(stream_chains=p.stream_chains, split=p.split, iters_per_graph=p.iters_per_graph,
                    ms_per_iteration=round(float(p.ms_per_iteration), 5))

    def graph_active(self) -> bool:
        """Whether stepping replays captured HIP graphs."""
        a = ctypes.c_int32()
        _check(load_library().qap_swarm_graph(self.h, ctypes.byref(a), None), "qap_swarm_graph")
        return bool(a.value)

    def stream_groups(self) -> int:
        """Concurrent stream groups (launches of each stage per iteration)."""
        g = ctypes.c_int32()
        _check(load_library().qap_swarm_graph(self.h, None, ctypes.byref(g)), "qap_swarm_graph")
        return int(g.value)

    def stats(self, q_ppm=(50000, 250000, 500000, 750000), bins: int = 0, lo: int = 0, hi: int = 1,
              instance: int = 0, noalloc: bool = False) -> dict:
        """Percentile ranks (nearest rank, q in parts per million) and PMF counts of
        the current goals, per swarm and over the population.  noalloc: through
        qap_swarm_stats_noalloc (fixed scratch, no allocation)."""
        m = self.ms[instance]
        q = np.ascontiguousarray(q_ppm, np.int32)
        nq = len(q)
        out = dict(swarm_q=np.zeros((m, nq), np.int64), pop_q=np.zeros(nq, np.int64),
                   swarm_hist=np.zeros((m, bins), np.int64), pop_hist=np.zeros(bins, np.int64))
        fn = load_library().qap_swarm_stats_noalloc if noalloc else load_library().qap_swarm_stats
        _check(fn(self.h, instance, nq, _ptr(q, ctypes.c_int32) if nq else None,
                  _ptr(out["swarm_q"], ctypes.c_int64), _ptr(out["pop_q"], ctypes.c_int64),
                  int(bins), int(lo), int(hi),
                  _ptr(out["swarm_hist"], ctypes.c_int64) if bins else None,
                  _ptr(out["pop_hist"], ctypes.c_int64) if bins else None),
               "qap_swarm_stats_noalloc" if noalloc else "qap_swarm_stats")
        return out

    def history_start(self, capacity: int, q_ppm=(50000, 250000, 500000, 750000), bins: int = 0, lo: int = 0,
                      hi: int = 1, instance: int = 0) -> None:
        """Record the percentile ranks and PMF counts after every iteration (a ring of `capacity` records)."""
        q = np.ascontiguousarray(q_ppm, np.int32)
        self._hist = getattr(self, "_hist", {})
        self._hist[instance] = (len(q), int(bins), int(capacity))
        _check(load_library().qap_swarm_history_start(self.h, instance, int(capacity), len(q),
                                                      _ptr(q, ctypes.c_int32) if len(q) else None, int(bins),
                                                      int(lo), int(hi)), "qap_swarm_history_start")

    def history_stop(self, instance: int = 0) -> None:
        _check(load_library().qap_swarm_history_stop(self.h, instance), "qap_swarm_history_stop")

    def history_read(self, max_records: int | None = None, instance: int = 0) -> dict:
        """The latest recorded iterations, oldest first."""
        # an instance that is not recording: the library reports it
        nq, bins, cap = getattr(self, "_hist", {}).get(instance, (0, 0, 0))
        R = cap if max_records is None else int(max_records)
        m = self.ms[instance]
        out = dict(iters=np.zeros(R, np.int32), swarm_q=np.zeros((R, m, nq), np.int64), pop_q=np.zeros((R, nq), np.int64),
                   swarm_hist=np.zeros((R, m, bins), np.int64), pop_hist=np.zeros((R, bins), np.int64))
        cnt = ctypes.c_int32()
        _check(load_library().qap_swarm_history_read(self.h, instance, R, ctypes.byref(cnt),
                                                     _ptr(out["iters"], ctypes.c_int32),
                                                     _ptr(out["swarm_q"], ctypes.c_int64), _ptr(out["pop_q"], ctypes.c_int64),
                                                     _ptr(out["swarm_hist"], ctypes.c_int64),
                                                     _ptr(out["pop_hist"], ctypes.c_int64)), "qap_swarm_history_read")
        c = int(cnt.value)
        return {k: v[:c] for k, v in out.items()}

    def profile(self, enable: bool):
        """Switch profiled stepping on/off; returns ({stage: ms}, iterations) so far."""
        ms = np.zeros(len(STAGES), np.float64)
        it = ctypes.c_int64()
        _check(load_library().qap_swarm_profile(self.h, 1 if enable else 0, _ptr(ms, ctypes.c_double),
                                                ctypes.byref(it)), "qap_swarm_profile")
        return dict(zip(STAGES, ms.tolist())), int(it.value)
