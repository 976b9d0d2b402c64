"""The headline configuration at full size, in the launch configuration the
benchmark times (n = 128, F and D symmetric U{0..127}, 200 swarms x 50
particles, Norm, depth 2, one pair exchange, fused engine replaying its
captured graph): properties over all 10,000 particles and exact one-step
parity of sampled particles against the oracle.  Then the largest sizes."""
import numpy as np
import pytest

import qap_inputs as gen
from _parity import (VTOL, announce, assert_states_equal, assert_v_close, make_gpu, oracle_from_state,
                     oracle_particle_step, run_cfg)

pytestmark = pytest.mark.gpu

HEADLINE = run_cfg(num_swarms=200, particles_per_swarm=50, c1=0.8, c2=0.5, c3=0.5, vmax=1.0, norm=True, depth=2,
                   local_search=True, seed=1)


def test_headline_size_sampled_parity(q, orc):
    F, D = gen.uniform_instance(128, 0, 127, 104)
    announce("fullsize n128x10k")
    sw = make_gpu(q, F, D, dict(HEADLINE, engine="fused"))
    sw.step(12)
    assert sw.graph_active()
    st = sw.get_state()
    sw.step(1)
    nx = sw.get_state()
    P, n = nx["X"].shape
    assert P == 10000 and n == 128
    # every particle holds a permutation; the iteration counter advanced once
    assert (np.sort(nx["X"], axis=1) == np.arange(n)).all()
    assert (np.sort(nx["PL"], axis=1) == np.arange(n)).all()
    assert nx["t"] == st["t"] + 1 == 13
    # P^L only improves; independent swarms: goal(P^G) = min over members of goal(P^L)
    assert (nx["goalPL"] <= st["goalPL"]).all()
    assert (nx["goalPG"] == nx["goalPL"].reshape(200, 50).min(axis=1)).all()
    rng = np.random.default_rng(2024)
    sample = np.concatenate([[0, 49, 50, 9999], rng.choice(P, 20, replace=False)])
    for k in sample:
        Vn, x, goal, pl, gpl = oracle_particle_step(orc, F, D, HEADLINE, st, k)
        assert np.array_equal(nx["X"][k], x), k
        assert int(nx["goal"][k]) == goal == orc.cost(F, D, nx["X"][k]), k
        assert np.array_equal(nx["PL"][k], pl) and int(nx["goalPL"][k]) == gpl, k
        assert_v_close(nx["V"][k][None], Vn[None], VTOL)
    # swarm bests of sampled swarms: P^G is a permutation with its goal
    for g in (0, 1, 199):
        assert orc.cost(F, D, nx["PG"][g]) == int(nx["goalPG"][g])
    assert orc.cost(F, D, nx["best_perm"]) == int(nx["best_goal"]) == int(nx["goalPG"].min())
    sw.close()


@pytest.mark.parametrize("engine", ["fused", "plain"])
@pytest.mark.parametrize("n", [160, 256])
def test_largest_sizes_one_step_parity(q, orc, engine, n):
    """n = 160 is the largest padded size of the fused kernel; n = 256 the
    largest the library takes (the fused engine steps it with the per-stage
    kernels).  Three re-synchronised one-step comparisons each."""
    F, D = gen.uniform_instance(n, 0, 127, 300 + n)
    cfg = run_cfg(num_swarms=1, particles_per_swarm=6, seed=n)
    announce("largest", engine, n)
    sw = make_gpu(q, F, D, dict(cfg, engine=engine))
    assert sw.path()[0] == ("int8" if engine == "fused" and n <= 160 else "int32")
    for it in range(3):
        st = sw.get_state()
        o = oracle_from_state(orc, F, D, cfg, st)
        o.step()
        sw.step(1)
        assert_states_equal(sw.get_state(), o.state(), what="n=%d iteration %d" % (n, it + 1))
    sw.close()


def _workload_cfg(w, **extra):
    return run_cfg(num_swarms=w["num_swarms"], particles_per_swarm=w["particles_per_swarm"],
                   migration=w["migration"], migration_factor=w.get("migration_factor", 0.0),
                   migration_period=w.get("migration_period", 1), seed=1, **extra)


@pytest.mark.parametrize("name,path,steps", [
    ("n50", "int32", 12),         # 10 x 1000, the int32 path forced as in that workload
    ("n128", "int8", 12),         # 8 x 512
    ("n128wide", "split", 12),    # 8 x 512, D up to 1000: byte-split MFMA
    ("n100mig", "split", 49),     # 20 x 500, migration every 50 iterations: the compared step migrates
])
def test_workload_sizes_sampled_parity(q, orc, name, path, steps):
    """The other workloads at full size on the fused engine: sampled particles
    exactly as the oracle's per-particle step, and the swarm-level invariants
    over the whole population (with migration, P^G holds a member's current
    solution and its goal, not necessarily the swarm's best)."""
    w = gen.WORKLOADS[name]
    F, D = w["gen"]()
    cfg = _workload_cfg(w, delta_path="int32" if path == "int32" else "auto")
    announce("fullsize", name, path)
    sw = make_gpu(q, F, D, dict(cfg, engine="fused"))
    assert sw.path()[0] == path
    sw.step(steps)
    st = sw.get_state()
    sw.step(1)
    nx = sw.get_state()
    m, S = cfg["num_swarms"], cfg["particles_per_swarm"]
    P, n = nx["X"].shape
    assert P == m * S and n == F.shape[0]
    assert nx["t"] == steps + 1
    assert (np.sort(nx["X"], axis=1) == np.arange(n)).all()
    assert (nx["goalPL"] <= st["goalPL"]).all()
    rng = np.random.default_rng(7)
    sample = np.concatenate([[0, S - 1, S, P - 1], rng.choice(P, 12, replace=False)])
    for k in sample:
        Vn, x, goal, pl, gpl = oracle_particle_step(orc, F, D, cfg, st, k)
        assert np.array_equal(nx["X"][k], x), (name, k)
        assert int(nx["goal"][k]) == goal == orc.cost(F, D, nx["X"][k]), (name, k)
        assert np.array_equal(nx["PL"][k], pl) and int(nx["goalPL"][k]) == gpl, (name, k)
        assert_v_close(nx["V"][k][None], Vn[None], VTOL)
    for g in range(m):
        assert orc.cost(F, D, nx["PG"][g]) == int(nx["goalPG"][g]), (name, g)
    if not cfg["migration"]:
        assert (nx["goalPG"] == nx["goalPL"].reshape(m, S).min(axis=1)).all()
    else:
        # Alg. 2 ran after this step: d = floor(0.33 m) recipients took a member's goal
        d = int(cfg["migration_factor"] * m)
        best_now = nx["goal"].reshape(m, S).min(axis=1)
        moved = int((nx["goalPG"] != np.minimum(st["goalPG"], best_now)).sum())
        assert moved <= d, (moved, d)
    assert orc.cost(F, D, nx["best_perm"]) == int(nx["best_goal"]) <= int(nx["goalPG"].min())
    sw.close()
