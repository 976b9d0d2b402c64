"""CPU oracle for the multi-swarm discrete PSO for the QAP (arXiv:1504.05158).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library never does.

The arithmetic lives in ``qap_oracle.c`` (plain C, double velocities, int64
costs); this module only compiles it (``build()``) and marshals numpy arrays.
Every function cites, in the C source, the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qap_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_c = ctypes


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
        L.orc_word.argtypes = [_c.c_uint64, _c.c_uint32, _c.c_uint32, _c.c_uint32, _c.c_uint32]
        L.orc_word.restype = _c.c_uint32
        L.orc_u01.argtypes = [_c.c_uint32]
        L.orc_u01.restype = _c.c_double
        L.orc_bounded.argtypes = [_c.c_uint32, _c.c_uint32]
        L.orc_bounded.restype = _c.c_uint32
        L.orc_cost.argtypes = [_c.c_int, _i32p, _i32p, _i32p]
        L.orc_cost.restype = _c.c_int64
        L.orc_delta.argtypes = [_c.c_int, _i32p, _i32p, _i32p, _c.c_int, _c.c_int]
        L.orc_delta.restype = _c.c_int64
        L.orc_deltas.argtypes = [_c.c_int, _i32p, _i32p, _i32p, _i64p]
        L.orc_local_search.argtypes = [_c.c_int, _i32p, _i32p, _i32p, _i64p, _i32p, _i32p, _i64p]
        L.orc_local_search.restype = _c.c_int
        L.orc_velocity.argtypes = [_c.c_int, _f64p, _i32p, _i32p, _i32p, _c.c_double, _c.c_double,
                                   _c.c_double, _c.c_double, _c.c_double, _c.c_double, _c.c_int, _f64p]
        L.orc_keys.argtypes = [_c.c_int, _f64p, _i32p, _f32p]
        L.orc_second_target.argtypes = [_c.c_int, _f32p, _i32p, _c.c_int, _c.c_uint64, _c.c_uint32,
                                        _c.c_uint32, _c.c_uint32, _i32p, _i32p]
        L.orc_init.argtypes = [_c.c_int, _i32p, _i32p, _c.c_int, _c.c_int, _c.c_double, _c.c_int,
                               _c.c_uint64, _f64p, _i32p, _i32p, _i64p, _i64p, _i32p, _i64p, _i64p,
                               _i32p, _i32p]
        L.orc_migrate.argtypes = [_c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_uint64, _c.c_uint32,
                                  _i32p, _i64p, _i32p, _i64p]
        L.orc_pick_column.argtypes = [_c.c_int, _f32p, _c.c_uint64, _c.c_uint32, _c.c_uint32, _c.c_uint32, _i32p]
        L.orc_step.argtypes = [_c.c_int, _i32p, _i32p, _c.c_int, _c.c_int, _c.c_double, _c.c_double,
                               _c.c_double, _c.c_double, _c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_int,
                               _c.c_int, _c.c_int, _c.c_uint64, _c.c_int32, _f64p, _i32p, _i32p,
                               _i64p, _i64p, _i32p, _i64p, _i64p, _i32p, _i32p, _c.c_void_p]
        L.orc_set_threads.argtypes = [_c.c_int]
        L.orc_get_threads.restype = _c.c_int
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------- primitives
def philox4x32(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def philox4x64(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(np.asarray(ctr, np.uint64), np.asarray(key, np.uint64), out)
    return out


def word(seed: int, element: int, t: int, particle: int, swarm: int) -> int:
    return int(lib().orc_word(seed, element, t, particle, swarm))


def u01(w: int) -> float:
    return float(lib().orc_u01(w))


def bounded(w: int, m: int) -> int:
    return int(lib().orc_bounded(w, m))


def cost(F, D, p) -> int:
    F, D = _i32(F), _i32(D)
    return int(lib().orc_cost(F.shape[0], F, D, _i32(p)))


def delta(F, D, p, a: int, b: int) -> int:
    F, D = _i32(F), _i32(D)
    return int(lib().orc_delta(F.shape[0], F, D, _i32(p), a, b))


def deltas(F, D, p) -> np.ndarray:
    F, D = _i32(F), _i32(D)
    n = F.shape[0]
    out = np.zeros((n, n), np.int64)
    lib().orc_deltas(n, F, D, _i32(p), out)
    return out


def local_search(F, D, p):
    """Returns (new p, new goal, (a, b, best delta), swapped?)."""
    F, D = _i32(F), _i32(D)
    n = F.shape[0]
    p = _i32(p).copy()
    g = np.array([cost(F, D, p)], np.int64)
    a = np.zeros(1, np.int32)
    b = np.zeros(1, np.int32)
    bd = np.zeros(1, np.int64)
    sw = lib().orc_local_search(n, F, D, p, g, a, b, bd)
    return p, int(g[0]), (int(a[0]), int(b[0]), int(bd[0])), bool(sw)


def velocity(V, p, pl, pg, c1, c2, c3, r2, r3, vmax, norm) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64)
    n = V.shape[0]
    out = np.zeros_like(V)
    lib().orc_velocity(n, V, _i32(p), _i32(pl), _i32(pg), c1, c2, c3, r2, r3, vmax, int(norm), out)
    return out


def keys(V, p) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64)
    n = V.shape[0]
    W = np.zeros((n, n), np.float32)
    lib().orc_keys(n, V, _i32(p), W)
    return W


def second_target(W, z, depth, seed=0, t=1, particle=0, swarm=0, return_ties=False):
    W = np.ascontiguousarray(W, dtype=np.float32)
    n = W.shape[0]
    out = np.full(n, -1, np.int32)
    ties = np.zeros(n, np.int32)
    lib().orc_second_target(n, W, _i32(z), int(depth), seed, t, particle, swarm, out, ties)
    return (out, ties) if return_ties else out


def pick_column(W, seed=0, t=1, particle=0, swarm=0):
    W = np.ascontiguousarray(W, dtype=np.float32)
    n = W.shape[0]
    out = np.full(n, -1, np.int32)
    lib().orc_pick_column(n, W, seed, t, particle, swarm, out)
    return out


def set_threads(k: int) -> None:
    lib().orc_set_threads(int(k))


def get_threads() -> int:
    return int(lib().orc_get_threads())


# ---------------------------------------------------------------- swarm state
def nearest_rank_quantiles(values, q_ppm) -> np.ndarray:
    """Percentile ranks of a population of goals (Sec. 4.2): for q in parts per
    million, the value at position ceil(q * N / 10^6) (at least 1) of the values
    in ascending order -- the nearest-rank reading of the paper's percentile
    ranks.  Integer arithmetic throughout."""
    v = np.sort(np.asarray(values, np.int64))
    N = len(v)
    out = []
    for q in q_ppm:
        r = max(1, -(-int(q) * N // 1000000))  # ceil(q N / 10^6)
        out.append(v[min(r, N) - 1])
    return np.asarray(out, np.int64)


def goal_histogram(values, bins: int, lo: int, hi: int) -> np.ndarray:
    """Probability mass function of goals as counts (Sec. 4.2): bin
    floor((g - lo) * bins / (hi - lo)) for lo <= g < hi; values outside
    [lo, hi) are not counted."""
    h = np.zeros(bins, np.int64)
    for g in np.asarray(values, np.int64):
        g = int(g)
        if lo <= g < hi:
            h[(g - lo) * bins // (hi - lo)] += 1
    return h


class OracleSwarm:
    """Whole-run oracle: state arrays in the layout the GPU library exports.

    V [P, n, n] float64 (row = location, column = facility); X, PL [P, n];
    goal, goalPL [P]; PG [m, n]; goalPG [m]; best_goal, best_perm [n],
    best_info = (iteration, swarm, member); t = iteration counter.
    """

    def __init__(self, F, D, *, num_swarms, particles_per_swarm, c1=0.8, c2=0.5, c3=0.5, vmax=1.0,
                 norm=True, depth=2, local_search=True, migration=False, migration_factor=0.0,
                 migration_period=1, seed=1, sx="second_target"):
        self.F, self.D = _i32(F), _i32(D)
        self.n = n = self.F.shape[0]
        self.m, self.S = int(num_swarms), int(particles_per_swarm)
        self.P = P = self.m * self.S
        self.c1, self.c2, self.c3 = float(np.float32(c1)), float(np.float32(c2)), float(np.float32(c3))
        self.vmax = float(np.float32(vmax))
        self.norm, self.depth, self.ls = bool(norm), int(depth), int(local_search)  # exchanges per iteration
        self.sx = {"second_target": 0, "pick_column": 1}[sx]
        self.migration = bool(migration)
        self.migr_d = int(np.floor(np.float32(migration_factor) * self.m)) if migration else 0
        self.period = int(migration_period)
        self.seed = int(seed)
        self.V = np.zeros((P, n, n), np.float64)
        self.X = np.zeros((P, n), np.int32)
        self.PL = np.zeros((P, n), np.int32)
        self.goal = np.zeros(P, np.int64)
        self.goalPL = np.zeros(P, np.int64)
        self.PG = np.zeros((self.m, n), np.int32)
        self.goalPG = np.zeros(self.m, np.int64)
        self.best_goal = np.zeros(1, np.int64)
        self.best_perm = np.zeros(n, np.int32)
        self.best_info = np.zeros(3, np.int32)
        self.t = 0
        lib().orc_init(n, self.F, self.D, self.m, self.S, self.vmax, int(self.norm), self.seed, self.V,
                       self.X, self.PL, self.goal, self.goalPL, self.PG, self.goalPG, self.best_goal,
                       self.best_perm, self.best_info)

    def step(self, iterations: int = 1, deltas_out: np.ndarray | None = None) -> None:
        for _ in range(iterations):
            self.t += 1
            dptr = None
            if deltas_out is not None:
                assert deltas_out.dtype == np.int64 and deltas_out.flags.c_contiguous
                assert deltas_out.shape == (self.P, self.n, self.n)
                dptr = deltas_out.ctypes.data_as(ctypes.c_void_p)
            lib().orc_step(self.n, self.F, self.D, self.m, self.S, self.c1, self.c2, self.c3, self.vmax,
                           int(self.norm), self.depth, self.sx, int(self.ls), int(self.migration), self.migr_d,
                           self.period, self.seed, self.t, self.V, self.X, self.PL, self.goal,
                           self.goalPL, self.PG, self.goalPG, self.best_goal, self.best_perm,
                           self.best_info, dptr)

    def state(self) -> dict:
        return dict(V=self.V.copy(), X=self.X.copy(), PL=self.PL.copy(), goal=self.goal.copy(),
                    goalPL=self.goalPL.copy(), PG=self.PG.copy(), goalPG=self.goalPG.copy(),
                    best_goal=int(self.best_goal[0]), best_perm=self.best_perm.copy(),
                    best_info=self.best_info.copy(), t=self.t)

    def load_state(self, st: dict) -> None:
        """Overwrite the state (e.g. with a state exported from the GPU)."""
        self.V[...] = np.asarray(st["V"], np.float64)
        self.X[...] = st["X"]
        self.PL[...] = st["PL"]
        self.goal[...] = st["goal"]
        self.goalPL[...] = st["goalPL"]
        self.PG[...] = st["PG"]
        self.goalPG[...] = st["goalPG"]
        self.best_goal[0] = st["best_goal"]
        self.best_perm[...] = st["best_perm"]
        self.best_info[...] = st["best_info"]
        self.t = int(st["t"])
