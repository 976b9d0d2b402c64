"""Helpers shared by the GPU parity tests (GPU library vs CPU oracle)."""
import sys

import numpy as np

VTOL = 1e-5  # FP32 velocities vs the FP64 oracle, relative to each entry itself
VFLOOR = 2.0 ** -126  # absolute floor: only exact zeros and binary32 subnormals lean on it


def run_cfg(**kw):
    """Parameter dict accepted by both paper_1504_05158_amd.make_params and OracleSwarm."""
    base = dict(num_swarms=2, particles_per_swarm=8, c1=0.8, c2=0.5, c3=0.5, vmax=1.0, norm=True, depth=2,
                local_search=True, migration=False, migration_factor=0.0, migration_period=1, seed=1)
    base.update(kw)
    return base


def oracle_cfg(cfg):
    return {k: v for k, v in cfg.items() if k not in ("engine", "delta_path")}


def make_gpu(q, F, D, cfg):
    return q.Swarm.create(F, D, **cfg)


def oracle_from_state(orc, F, D, cfg, st):
    o = orc.OracleSwarm(F, D, **oracle_cfg(cfg))
    o.load_state(dict(st, V=np.asarray(st["V"], np.float64)))
    return o


def assert_v_close(Vg, Vo, tol=VTOL):
    """Every entry within tol of the oracle's value, relative to that value
    (|Vg - Vo| <= tol |Vo| + VFLOOR).  The message also gives the error
    relative to the column's largest entry, as a diagnostic."""
    Vg = np.asarray(Vg, np.float64)
    Vo = np.asarray(Vo, np.float64)
    err = np.abs(Vg - Vo)
    bad = err > tol * np.abs(Vo) + VFLOOR
    if bad.any():
        colmax = np.abs(Vo).max(axis=-2, keepdims=True)  # per column (facility)
        i = tuple(np.argwhere(bad)[0])
        cm = colmax[i[:-2] + (0, i[-1])]
        raise AssertionError("V mismatch at %s: gpu %r oracle %r (rel %.3g, col max %r, rel to col max %.3g), %d cells"
                             % (i, Vg[i], Vo[i], err[i] / max(abs(Vo[i]), 1e-300), cm, err[i] / max(cm, 1e-300),
                                int(bad.sum())))


def assert_states_equal(g, o, vtol=VTOL, what=""):
    """Everything integer is exact; V within vtol."""
    for k in ("X", "PL", "goal", "goalPL", "PG", "goalPG", "best_perm"):
        a, b = np.asarray(g[k]), np.asarray(o[k])
        if not np.array_equal(a, b):
            idx = np.argwhere(a != b)[0] if a.shape == b.shape else None
            raise AssertionError("%s %s differs (first at %s): gpu %s oracle %s" % (
                what, k, idx, a[tuple(idx[:1])] if idx is not None else a.shape,
                b[tuple(idx[:1])] if idx is not None else b.shape))
    assert int(g["best_goal"]) == int(o["best_goal"]), (what, g["best_goal"], o["best_goal"])
    assert list(np.asarray(g["best_info"])) == list(np.asarray(o["best_info"])), (what, g["best_info"], o["best_info"])
    assert int(g["t"]) == int(o["t"])
    assert_v_close(g["V"], o["V"], vtol)


def announce(*a):
    """Name the GPU case on stdout before it runs (a fault then points at it)."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def oracle_particle_step(orc, F, D, cfg, st, k):
    """One iteration t -> t+1 of particle k alone, from an exported state st,
    by the oracle's per-particle functions (velocity, keys, SecondTarget, local
    search, goal), in the order of the oracle's swarm step.  Returns the
    particle's V, X, goal, P^L and goal of P^L after the iteration (P^G and the
    bests need the whole swarm and are not produced)."""
    S = cfg["particles_per_swarm"]
    g, s = divmod(int(k), S)
    t1 = int(st["t"]) + 1
    seed = cfg["seed"]
    r2 = orc.u01(orc.word(seed, 0, t1, s, g))
    r3 = orc.u01(orc.word(seed, 1, t1, s, g))
    V = np.asarray(st["V"][k], np.float64)
    x = np.asarray(st["X"][k])
    # the coefficients as the library holds them (binary32 parameters), as OracleSwarm takes them
    c1, c2, c3, vmax = (float(np.float32(cfg[key])) for key in ("c1", "c2", "c3", "vmax"))
    Vn = orc.velocity(V, x, st["PL"][k], st["PG"][g], c1, c2, c3, r2, r3, vmax, cfg["norm"])
    xs = orc.second_target(orc.keys(V, x), x, cfg["depth"], seed=seed, t=t1, particle=s, swarm=g)
    if cfg["local_search"]:
        xs, goal, _, _ = orc.local_search(F, D, xs)
    else:
        goal = orc.cost(F, D, xs)
    if goal < int(st["goalPL"][k]):
        pl, gpl = xs.copy(), goal
    else:
        pl, gpl = np.asarray(st["PL"][k]).copy(), int(st["goalPL"][k])
    return Vn, np.asarray(xs), int(goal), np.asarray(pl), int(gpl)
