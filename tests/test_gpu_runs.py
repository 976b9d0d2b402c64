"""Whole runs on the GPU against whole runs of the oracle.

One-step parity re-synchronises both sides every iteration.  Over a free run
the binary32 velocities of the GPU and the binary64 velocities of the oracle
drift apart by rounding, and a near-tied SecondTarget selection can then go
either way, after which the two trajectories are different samples of the
same random process.  So whole runs are compared by distribution: the n = 12
workload (F and D symmetric U{0..10}, 1 swarm x 64 particles, 100 iterations)
from 20 seeds on both sides, two-sample Kolmogorov-Smirnov tests at the 1 %
level on per-run statistics of the final goals (mean, median, best ever).
The run is the sampling unit: the 64 particles of one run share their swarm
best and end up strongly correlated, so a test on the pooled per-particle
goals treats 1,280 dependent values as independent and rejects even two
independent sets of oracle runs (seeds 1-20 against 21-40, 41-60, ...: p from
1e-37 to 0.01).  Small instances (n = 3..9) must reach the optimum found by
enumerating every permutation, on both sides.
"""
import itertools

import numpy as np
import pytest

import qap_inputs as gen
from _parity import announce, make_gpu, run_cfg

pytestmark = pytest.mark.gpu

SEEDS = range(1, 21)
ALPHA = 0.01


def _c1_runs(q, orc, engine):
    F, D = gen.uniform_instance(12, 0, 10, 101)
    gpu, ora = [], []
    for seed in SEEDS:
        cfg = run_cfg(num_swarms=1, particles_per_swarm=64, seed=seed)
        sw = make_gpu(q, F, D, dict(cfg, engine=engine))
        sw.step(100)
        gpu.append(sw.get_state())
        sw.close()
        o = orc.OracleSwarm(F, D, **cfg)
        o.step(100)
        ora.append(o.state())
    return F, D, gpu, ora


@pytest.mark.parametrize("engine", ["fused", "plain"])
def test_full_run_goal_distributions_agree(q, orc, engine):
    from scipy.stats import ks_2samp
    announce("runs n12 x 20 seeds", engine)
    F, D, gpu, ora = _c1_runs(q, orc, engine)
    for g in gpu:
        assert g["t"] == 100
        assert (np.sort(g["X"], axis=1) == np.arange(12)).all()
        for k in (0, 31, 63):
            assert int(g["goal"][k]) == orc.cost(F, D, g["X"][k])
    # per run: the mean and the median of the final goals, the best goal ever seen
    stats = {}
    for what, f in (("run means", lambda s: s["goal"].mean()), ("run medians", lambda s: np.median(s["goal"])),
                    ("run bests", lambda s: s["best_goal"])):
        stats[what] = (np.array([f(g) for g in gpu]), np.array([f(o) for o in ora]))
    same = sum(np.array_equal(g["X"], o["X"]) for g, o in zip(gpu, ora))
    print("runs with identical final solutions: %d of %d" % (same, len(gpu)))
    for what, (a, b) in stats.items():
        p = ks_2samp(a, b).pvalue
        print("%s: KS p = %.4g" % (what, p))
        assert p > ALPHA, (what, p)


def _brute_force_optimum(F, D):
    n = F.shape[0]
    F = F.astype(np.int64)
    D = D.astype(np.int64)
    perms = np.array(list(itertools.permutations(range(n))), np.int64)
    best = None
    for i in range(0, len(perms), 20000):
        p = perms[i:i + 20000]
        c = (F[None, :, :] * D[p[:, :, None], p[:, None, :]]).sum(axis=(1, 2)).min()
        best = int(c) if best is None else min(best, int(c))
    return best


@pytest.mark.parametrize("engine", ["fused", "plain"])
def test_small_instances_reach_brute_force_optimum(q, orc, engine):
    announce("brute force n3..9", engine)
    for n, seed in zip(range(3, 10), range(201, 208)):
        F, D = gen.uniform_instance(n, 0, 10, seed)
        opt = _brute_force_optimum(F, D)
        cfg = run_cfg(num_swarms=1, particles_per_swarm=64, depth=min(2, n - 1), seed=1)
        sw = make_gpu(q, F, D, dict(cfg, engine=engine))
        sw.step(100)
        g, perm, _ = sw.best()
        sw.close()
        o = orc.OracleSwarm(F, D, **cfg)
        o.step(100)
        assert g == orc.cost(F, D, perm) == opt, (n, g, opt)
        assert o.state()["best_goal"] == opt, (n, o.state()["best_goal"], opt)
