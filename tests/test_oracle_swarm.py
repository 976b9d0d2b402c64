"""Pins of the oracle's whole-swarm logic: initialisation, best updates,
migration (Alg. 2, Sec. 3.2) and whole runs (invariants, brute-force optima).
"""
import itertools
from collections import Counter

import numpy as np
import pytest

import qap_inputs as gen


def brute_opt(orc, F, D):
    n = F.shape[0]
    return min(orc.cost(F, D, p) for p in itertools.permutations(range(n)))


def test_init_permutations_uniform(orc):
    F, D = gen.uniform_instance(4, 0, 10, 1)
    sw = orc.OracleSwarm(F, D, num_swarms=4, particles_per_swarm=1200, seed=77)
    cnt = Counter(tuple(x) for x in sw.X)
    assert all(sorted(k) == [0, 1, 2, 3] for k in cnt)
    assert len(cnt) == 24
    exp = sw.P / 24
    chi2 = sum((c - exp) ** 2 / exp for c in cnt.values())
    assert chi2 < 49.7  # 23 dof, p ~ 1e-3


def test_init_mean_cost_closed_form(orc):
    n = 9
    F, D = gen.general_instance(n, 0, 20, 3)
    sw = orc.OracleSwarm(F, D, num_swarms=10, particles_per_swarm=600, seed=5)
    offF = float(F.sum() - np.trace(F))
    offD = float(D.sum() - np.trace(D))
    mean = offF * offD / (n * (n - 1)) + float(np.trace(F)) * float(np.trace(D)) / n
    se = sw.goal.std() / np.sqrt(sw.P)
    assert abs(sw.goal.mean() - mean) < 4 * se


@pytest.mark.parametrize("norm", [True, False])
def test_init_state_consistency(orc, norm):
    F, D = gen.uniform_instance(12, 0, 10, 101)
    sw = orc.OracleSwarm(F, D, num_swarms=3, particles_per_swarm=20, norm=norm, vmax=0.75, seed=9)
    for i in range(sw.P):
        assert sw.goal[i] == orc.cost(F, D, sw.X[i])
    assert np.array_equal(sw.PL, sw.X) and np.array_equal(sw.goalPL, sw.goal)
    assert np.abs(sw.V).max() <= 0.75
    if norm:
        assert np.allclose(np.abs(sw.V).sum(1), 1.0, rtol=0, atol=1e-12)
    for g in range(3):
        blk = sw.goal[g * 20:(g + 1) * 20]
        j = int(np.argmin(blk))
        assert sw.goalPG[g] == blk[j] and np.array_equal(sw.PG[g], sw.X[g * 20 + j])
    assert sw.best_goal[0] == sw.goal.min() and list(sw.best_info)[0] == 0


def test_migration_invariants(orc):
    n, m, S, d = 8, 9, 5, 4
    rng = np.random.default_rng(1)
    X = np.stack([rng.permutation(n) for _ in range(m * S)]).astype(np.int32)
    goal = rng.integers(0, 1000, m * S).astype(np.int64)
    PG = np.stack([rng.permutation(n) for _ in range(m)]).astype(np.int32)
    goalPG = rng.integers(0, 1000, m).astype(np.int64)
    goalPG[3] = goalPG[5]  # a tie in the sort
    PG0, gPG0 = PG.copy(), goalPG.copy()
    orc.lib().orc_migrate(n, m, S, d, 42, 50, X, goal, PG, goalPG)
    order = sorted(range(m), key=lambda g: (gPG0[g], g))
    donors, recips = order[:d], order[m - d:]
    assert not set(donors) & set(recips)
    changed = [g for g in range(m) if not np.array_equal(PG[g], PG0[g]) or goalPG[g] != gPG0[g]]
    assert set(changed) <= set(recips)
    for k in range(d):
        rcp, dnr = order[m - 1 - k], order[k]
        j = orc.bounded(orc.word(42, k, 50, 0xFFFFFFFF, 0), S)
        assert np.array_equal(PG[rcp], X[dnr * S + j]) and goalPG[rcp] == goal[dnr * S + j]
    for g in donors + order[d:m - d]:
        assert np.array_equal(PG[g], PG0[g]) and goalPG[g] == gPG0[g]


def check_run_invariants(orc, sw, F, D, independent):
    for i in range(sw.P):
        assert sw.goal[i] == orc.cost(F, D, sw.X[i])
        assert sorted(sw.X[i]) == list(range(sw.n))
        assert sw.goalPL[i] == orc.cost(F, D, sw.PL[i]) and sw.goalPL[i] <= sw.goal[i]
    for g in range(sw.m):
        assert sw.goalPG[g] == orc.cost(F, D, sw.PG[g])
        if independent:
            # without migration P^G holds the best position any member ever had
            assert sw.goalPG[g] == sw.goalPL[g * sw.S:(g + 1) * sw.S].min()
    assert sw.best_goal[0] == orc.cost(F, D, sw.best_perm)
    assert sw.best_goal[0] <= sw.goalPL.min()


@pytest.mark.parametrize("norm,ls,depth", [(True, True, 2), (False, True, 1), (True, False, 3), (False, False, 0)])
def test_run_invariants_independent(orc, norm, ls, depth):
    F, D = gen.uniform_instance(12, 0, 10, 101)
    sw = orc.OracleSwarm(F, D, num_swarms=2, particles_per_swarm=16, norm=norm, local_search=ls,
                         depth=depth, seed=3)
    prev_best = sw.best_goal[0]
    for _ in range(15):
        sw.step()
        assert sw.best_goal[0] <= prev_best
        prev_best = sw.best_goal[0]
    check_run_invariants(orc, sw, F, D, independent=True)
    assert sw.t == 15


def test_run_invariants_migration(orc):
    F, D = gen.euclid_sparse_instance(16, 103)
    sw = orc.OracleSwarm(F, D, num_swarms=6, particles_per_swarm=8, migration=True, migration_factor=0.33,
                         migration_period=3, seed=4)
    assert sw.migr_d == 1
    for _ in range(12):
        sw.step()
    check_run_invariants(orc, sw, F, D, independent=False)


@pytest.mark.parametrize("n,seed", [(5, 203), (6, 204), (7, 205), (8, 206)])
def test_small_instances_reach_brute_force_optimum(orc, n, seed):
    F, D = gen.uniform_instance(n, 0, 10, seed)
    opt = brute_opt(orc, F, D)
    sw = orc.OracleSwarm(F, D, num_swarms=1, particles_per_swarm=64, seed=1)
    for _ in range(30):
        sw.step()
        assert sw.best_goal[0] >= opt
    assert sw.best_goal[0] == opt


def test_linear_sum_family_reaches_sorted_optimum(orc):
    n = 20
    F, D, a = gen.linear_sum_instance(n, 31)
    w = F.sum(1).astype(np.int64) + F.sum(0).astype(np.int64)
    p = np.zeros(n, np.int32)
    p[np.argsort(-w, kind="stable")] = np.argsort(a, kind="stable")
    opt = orc.cost(F, D, p)
    sw = orc.OracleSwarm(F, D, num_swarms=4, particles_per_swarm=32, seed=2)
    for _ in range(60):
        sw.step()
    assert sw.best_goal[0] >= opt
    assert sw.best_goal[0] == opt


def test_step_is_deterministic_and_thread_independent(orc):
    F, D = gen.uniform_instance(20, 0, 50, 7)
    outs = []
    for th in (1, 4):
        orc.set_threads(th)
        sw = orc.OracleSwarm(F, D, num_swarms=3, particles_per_swarm=10, seed=11)
        sw.step(5)
        outs.append(sw.state())
    orc.set_threads(0)
    a, b = outs
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
