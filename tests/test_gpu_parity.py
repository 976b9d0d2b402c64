"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Goals, pair-exchange deltas and every permutation are compared exactly;
velocities entry by entry within 1e-5 relative (FP32 vs FP64).  One
step is compared from the same state: the GPU's state is exported, loaded into
the oracle, and both advance one iteration.
"""
import sys

import numpy as np
import pytest

import qap_inputs as gen
from _parity import announce, assert_states_equal, assert_v_close, make_gpu, oracle_from_state, run_cfg

pytestmark = pytest.mark.gpu

ENGINES = ["fused", "plain"]


INSTANCES = [
    ("sym8-n2", lambda: gen.uniform_instance(2, 0, 127, 1)),
    ("sym8-n12", lambda: gen.uniform_instance(12, 0, 10, 101)),
    ("sym8-n33", lambda: gen.uniform_instance(33, 0, 127, 5)),
    ("sym-wide-n50", lambda: gen.uniform_instance(50, 0, 99, 102, d_hi=1000)),
    ("gen-neg-n40", lambda: gen.general_instance(40, -128, 127, 7)),
    ("gen-wide-n65", lambda: gen.general_instance(65, -3000, 3000, 8)),
    ("euclid-n100", lambda: gen.euclid_sparse_instance(100, 103)),
    ("sym8-n128", lambda: gen.uniform_instance(128, 0, 127, 104)),
    ("sym8-n150", lambda: gen.uniform_instance(150, 0, 99, 9)),
]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("name,mk", INSTANCES, ids=[i[0] for i in INSTANCES])
def test_eval_goals_and_deltas_exact(q, orc, engine, name, mk):
    F, D = mk()
    n = F.shape[0]
    announce("eval", engine, name)
    sw = make_gpu(q, F, D, run_cfg(num_swarms=1, particles_per_swarm=2, depth=min(2, n - 1), engine=engine))
    perms = gen.random_perms(6, n, 3)
    goals, dl = sw.eval(perms, deltas=True)
    for i, p in enumerate(perms):
        assert goals[i] == orc.cost(F, D, p)
        assert np.array_equal(dl[i], orc.deltas(F, D, p)), (name, i)
    sw.close()


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("norm", [True, False])
@pytest.mark.parametrize("n", [20, 128, 150, 256])
def test_init_parity(q, orc, engine, norm, n):
    """Iteration 0 (random permutations, V(0) through S_v, goals, bests) up to
    the largest size: the column norm of V(0) sums n entries."""
    F, D = gen.uniform_instance(n, 0, 50, 11)
    cfg = run_cfg(num_swarms=3, particles_per_swarm=17, norm=norm, vmax=0.8, seed=99)
    announce("init", engine, norm, n)
    sw = make_gpu(q, F, D, dict(cfg, engine=engine))
    g = sw.get_state()
    o = orc.OracleSwarm(F, D, **cfg).state()
    assert_states_equal(g, o, what="init")
    sw.close()


CASES = [
    dict(n=12, kind="sym", norm=True, depth=2, ls=True),
    dict(n=12, kind="sym", norm=False, depth=1, ls=True),
    dict(n=12, kind="sym", norm=True, depth=0, ls=False),
    dict(n=33, kind="gen", norm=True, depth=3, ls=True),
    dict(n=33, kind="sym", norm=False, depth=32, ls=True),
    dict(n=64, kind="sym", norm=True, depth=2, ls=True),
    dict(n=70, kind="gen", norm=False, depth=2, ls=True),
    dict(n=100, kind="euclid", norm=True, depth=2, ls=True, migration=True),
    dict(n=128, kind="sym", norm=True, depth=2, ls=True),
    dict(n=150, kind="sym", norm=False, depth=5, ls=True),
    dict(n=40, kind="sym", norm=True, depth=2, ls=3),
    dict(n=33, kind="gen", norm=True, depth=2, ls=4),
    dict(n=128, kind="sym", norm=True, depth=2, ls=1000),   # to a pair-exchange local optimum
    # column slots of the velocity pass: one lane in the second slot, no tail
    # batch, a ragged second slot at npad 128, one lane in the third slot
    dict(n=65, kind="sym", norm=True, depth=2, ls=True),
    dict(n=80, kind="gen", norm=True, depth=2, ls=True),
    dict(n=97, kind="sym", norm=True, depth=2, ls=True),
    dict(n=129, kind="sym", norm=False, depth=2, ls=True),
]


def _instance(c):
    if c["kind"] == "sym":
        return gen.uniform_instance(c["n"], 0, 127, 40 + c["n"])
    if c["kind"] == "gen":
        return gen.general_instance(c["n"], -50, 127, 50 + c["n"])
    return gen.euclid_sparse_instance(c["n"], 103)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("c", CASES, ids=["n%d-%s-%s-d%d-ls%d%s" % (c["n"], c["kind"], "norm" if c["norm"] else "raw",
                                                                   c["depth"], c["ls"], "-mig" if c.get("migration") else "")
                                          for c in CASES])
def test_one_step_parity_along_a_run(q, orc, engine, c):
    """Several iterations; before each one the oracle is re-synchronised to
    the GPU's exported state, then both advance one iteration."""
    F, D = _instance(c)
    mig = c.get("migration", False)
    cfg = run_cfg(num_swarms=6 if mig else 2, particles_per_swarm=6, norm=c["norm"], depth=c["depth"],
                  local_search=c["ls"], migration=mig, migration_factor=0.34 if mig else 0.0,
                  migration_period=2, seed=7 + c["n"])
    announce("onestep", engine, c)
    sw = make_gpu(q, F, D, dict(cfg, engine=engine))
    for it in range(4):
        st = sw.get_state()
        o = oracle_from_state(orc, F, D, cfg, st)
        o.step()
        sw.step(1)
        assert_states_equal(sw.get_state(), o.state(), what="iteration %d" % (it + 1))
    sw.close()


@pytest.mark.parametrize("engine", ENGINES)
def test_free_run_matches_oracle_run_n12(q, orc, engine):
    """Both sides from the same seed, no re-synchronisation: the FP32 and FP64
    velocity trajectories drift apart by rounding only, so over a short run
    every integer decision still agrees."""
    F, D = gen.uniform_instance(12, 0, 10, 101)
    cfg = run_cfg(num_swarms=1, particles_per_swarm=64, seed=5)
    announce("freerun", engine)
    sw = make_gpu(q, F, D, dict(cfg, engine=engine))
    o = orc.OracleSwarm(F, D, **cfg)
    sw.step(3)
    o.step(3)
    g = sw.get_state()
    same = (g["X"] == o.X).all(axis=1)
    # a one-ulp key difference can flip a near-tied selection; nearly all agree
    assert same.mean() >= 0.9, same.mean()
    assert np.array_equal(g["goal"][same], o.goal[same])
    for i in range(len(g["goal"])):
        assert g["goal"][i] == orc.cost(F, D, g["X"][i])
    assert_v_close(g["V"][same], o.V[same], 1e-4)
    sw.close()


@pytest.mark.parametrize("engine", ENGINES)
def test_run_invariants_and_brute_force_optimum(q, orc, engine):
    import itertools
    F, D = gen.uniform_instance(7, 0, 10, 205)
    opt = min(orc.cost(F, D, p) for p in itertools.permutations(range(7)))
    announce("bruteforce", engine)
    sw = make_gpu(q, F, D, run_cfg(num_swarms=1, particles_per_swarm=64, seed=1, engine=engine))
    sw.step(30)
    g, perm, it = sw.best()
    assert g == opt == orc.cost(F, D, perm)
    st = sw.get_state()
    for i in range(len(st["goal"])):
        assert st["goal"][i] == orc.cost(F, D, st["X"][i])
    assert st["t"] == 30
    sw.close()


@pytest.mark.parametrize("engine", ENGINES)
def test_determinism_and_checkpoint(q, engine):
    F, D = gen.uniform_instance(30, 0, 99, 3)
    cfg = run_cfg(num_swarms=3, particles_per_swarm=10, seed=21, engine=engine)
    announce("determinism", engine)
    a = make_gpu(q, F, D, cfg)
    a.step(6)
    sa = a.get_state()
    b = make_gpu(q, F, D, cfg)
    b.step(3)
    ck = b.get_state()
    b.close()
    c = make_gpu(q, F, D, cfg)
    c.set_state(ck)
    c.step(3)
    sc = c.get_state()
    for k in sa:
        assert np.array_equal(np.asarray(sa[k]), np.asarray(sc[k])), k
    a.close()
    c.close()


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("n,depth", [(5, 0), (17, 2), (70, 2), (128, 0), (128, 2), (150, 3)])
def test_secondtarget_with_exact_ties(q, orc, engine, n, depth):
    """Quantised velocities make exact key ties frequent; X(t+1) (local search
    off) must equal the oracle's SecondTarget, tie-breaks included."""
    rng = np.random.default_rng(n * 10 + depth)
    F, D = gen.uniform_instance(n, 0, 20, n)
    m, S = 2, 16
    cfg = run_cfg(num_swarms=m, particles_per_swarm=S, norm=False, depth=depth, local_search=False, seed=3)
    announce("ties", engine, n, depth)
    sw = make_gpu(q, F, D, dict(cfg, engine=engine))
    st = sw.get_state()
    V = (rng.integers(-3, 4, size=(m * S, n, n)) / 4.0).astype(np.float32)
    st["V"] = V
    sw.set_state(st)
    sw.step(1)
    g = sw.get_state()
    nties = 0
    for k in range(m * S):
        W = orc.keys(V[k].astype(np.float64), st["X"][k])
        ref, ties = orc.second_target(W, st["X"][k], depth, seed=3, t=st["t"] + 1, particle=k % S, swarm=k // S,
                                      return_ties=True)
        nties += int((ties > 1).sum())
        assert np.array_equal(g["X"][k], ref), (n, depth, k)
    assert nties > 0
    sw.close()


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("mode", ["disjoint", "clash", "pairs", "pairs2"])
@pytest.mark.parametrize("n", [40, 128])
def test_secondtarget_tie_groups(q, orc, engine, mode, n):
    """Large groups of equal maximal keys.  "disjoint": every column's best
    non-Z cell (value 0.5) lies on a permutation pi avoiding the rows of X, so
    after the depth selections the rest of pi is one row/column-disjoint tie
    group, taken whole.  "clash": pi(c) is the X row of column c + 1, whose Z
    key 1 - 0.5 ties at 0.5, so the random order decides which cell of each
    clashing pair survives.  "pairs": the shape of late runs, -0.5 on the X
    row and +0.5 on a random other row of every column (rows repeat across
    columns); "pairs2" adds a second +0.5 cell to some columns.  X(t+1) must
    equal the oracle's SecondTarget."""
    rng = np.random.default_rng(n + (mode == "clash"))
    F, D = gen.uniform_instance(n, 0, 20, n)
    m, S = 1, 8
    cfg = run_cfg(num_swarms=m, particles_per_swarm=S, norm=False, depth=2, local_search=False, seed=11)
    announce("tiegroups", engine, mode, n)
    sw = make_gpu(q, F, D, dict(cfg, engine=engine))
    st = sw.get_state()
    V = np.empty((m * S, n, n), np.float32)
    for k in range(m * S):
        x = st["X"][k].astype(np.int64)
        # distinct small values elsewhere (no accidental ties below the maximum)
        V[k] = (rng.permutation(n * n).reshape(n, n) / (4.0 * n * n) - 0.375).astype(np.float32)
        cols = np.arange(n)
        if mode == "disjoint":
            pi = x[(cols + 1) % n] if n > 1 else x   # a permutation with pi(c) != x(c)
            V[k][x, cols] = -0.75                    # Z keys 0.25, below the group
        elif mode == "clash":
            pi = x[(cols + 1) % n]                   # pi(c) = X row of column c + 1
            V[k][x, cols] = -0.5                     # Z keys 0.5: each clashes with a pi cell
        else:
            pi = (x + rng.integers(1, n, size=n)) % n  # random rows other than X's, with repeats
            V[k][x, cols] = -0.5
            if mode == "pairs2":
                two = rng.random(n) < 0.1
                r2 = (pi + 1) % n
                r2 = np.where(r2 == x, (pi + 2) % n, r2)   # neither the X row nor pi
                V[k][r2[two], cols[two]] = 0.5
        V[k][pi, cols] = 0.5
    st["V"] = V
    sw.set_state(st)
    sw.step(1)
    g = sw.get_state()
    for k in range(m * S):
        W = orc.keys(V[k].astype(np.float64), st["X"][k])
        ref, ties = orc.second_target(W, st["X"][k], 2, seed=11, t=st["t"] + 1, particle=k % S, swarm=k // S,
                                      return_ties=True)
        assert (ties > 1).sum() > 0
        assert np.array_equal(g["X"][k], ref), (mode, n, k)
    sw.close()


@pytest.mark.parametrize("engine", ENGINES)
def test_norm_run_with_column_scales_n128(q, orc, engine):
    """Norm runs keep V as a matrix times per-column scales; near-equal keys
    1 + v arise often at n = 128.  Ten re-synchronised one-step comparisons."""
    F, D = gen.uniform_instance(128, 0, 127, 168)
    cfg = run_cfg(num_swarms=2, particles_per_swarm=8, norm=True, depth=2, local_search=True, seed=135)
    announce("normscale", engine)
    sw = make_gpu(q, F, D, dict(cfg, engine=engine))
    for it in range(10):
        st = sw.get_state()
        o = oracle_from_state(orc, F, D, cfg, st)
        o.step()
        sw.step(1)
        assert_states_equal(sw.get_state(), o.state(), what="iteration %d" % (it + 1))
    sw.close()


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("n", [12, 40, 128, 150])
def test_pick_column_one_step_parity(q, orc, engine, n):
    """S_x = PickColumn (runs on the per-stage kernels for both engines):
    re-synchronised one-step parity, integers exact and V within tolerance."""
    F, D = gen.uniform_instance(n, 0, 127, 600 + n)
    cfg = run_cfg(num_swarms=2, particles_per_swarm=6, seed=n + 1, sx="pick_column")
    announce("pickcolumn", engine, n)
    sw = make_gpu(q, F, D, dict(cfg, engine=engine))
    assert sw.path()[0] == "int32"
    for it in range(3):
        st = sw.get_state()
        o = oracle_from_state(orc, F, D, cfg, st)
        o.step()
        sw.step(1)
        assert_states_equal(sw.get_state(), o.state(), what="pickcolumn n=%d iteration %d" % (n, it + 1))
    sw.close()


def test_pick_column_with_exact_ties(q, orc):
    """Quantised velocities: many equal keys inside the visited columns."""
    n = 40
    F, D = gen.uniform_instance(n, 0, 20, 9)
    cfg = run_cfg(num_swarms=2, particles_per_swarm=8, norm=False, local_search=False, seed=5, sx="pick_column")
    announce("pickcolumn ties")
    sw = make_gpu(q, F, D, dict(cfg, engine="fused"))
    st = sw.get_state()
    rng = np.random.default_rng(3)
    V = (rng.integers(-2, 3, size=(16, n, n)) / 2.0).astype(np.float32)
    st["V"] = V
    sw.set_state(st)
    sw.step(1)
    g = sw.get_state()
    for k in range(16):
        ref = orc.pick_column(orc.keys(V[k].astype(np.float64), st["X"][k]), seed=5, t=st["t"] + 1, particle=k % 8,
                              swarm=k // 8)
        assert np.array_equal(g["X"][k], ref), k
    sw.close()
