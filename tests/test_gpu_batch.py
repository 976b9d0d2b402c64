"""Batched stepping and graph replays.

One handle over several instances steps them with one fused launch per kernel
class, the per-stage kernels for instances outside the int8 path, and batched
bests; it must give exactly the states of the same instances stepped in
handles of their own.  Graph replays must give exactly the states of eager
launches, replay after replay, with the program's own work and waits between
them."""
import numpy as np
import pytest

import qap_inputs as gen
from _parity import announce, run_cfg

pytestmark = pytest.mark.gpu

KEYS = ("V", "X", "PL", "goal", "goalPL", "PG", "goalPG", "best_perm", "best_goal", "best_info", "t")


def assert_same(a, b, what):
    for k in KEYS:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (what, k)


def mixed_cases():
    """Mixed sizes and kinds: symmetric zero-diagonal int8 instances of several
    padded sizes, a symmetric one with non-zero diagonals, a general one, one
    too wide for int8 (byte-split on the fused engine), an asymmetric wide one
    (int32 per-stage kernels), and one in migration mode."""
    cases = []
    for i, (F, D) in enumerate(gen.mixed_batch(count=5, seed=105, lo_n=12, hi_n=150)):
        cases.append((F, D, run_cfg(num_swarms=2 + i % 2, particles_per_swarm=8 + 3 * i, seed=10 + i)))
    rng = np.random.default_rng(77)
    A = rng.integers(0, 30, size=(40, 40)); F = A + A.T
    B = rng.integers(0, 30, size=(40, 40)); D = B + B.T
    cases.append((F, D, run_cfg(seed=21)))                                   # symmetric, non-zero diagonal
    F, D = gen.general_instance(33, -20, 40, 5)
    cases.append((F, D, run_cfg(seed=22)))                                   # general
    F, D = gen.uniform_instance(50, 0, 1000, 9)
    cases.append((F, D, run_cfg(seed=23, depth=1)))                          # byte-split path (fused engine)
    F, D = gen.general_instance(36, -900, 900, 6)
    cases.append((F, D, run_cfg(seed=25)))                                   # int32 path (asymmetric, wide)
    F, D = gen.uniform_instance(64, 0, 99, 11)
    cases.append((F, D, run_cfg(num_swarms=6, particles_per_swarm=5, migration=True, migration_factor=0.34,
                                migration_period=2, seed=24)))              # migration
    return cases


@pytest.mark.parametrize("engine", ["fused", "plain"])
def test_batch_equals_separate_handles(q, engine):
    cases = mixed_cases()
    announce("batch", engine, len(cases))
    params = [q.make_params(engine=engine, **cfg) for _, _, cfg in cases]
    batch = q.Swarm([(F, D) for F, D, _ in cases], params)
    singles = [q.Swarm.create(F, D, engine=engine, **cfg) for F, D, cfg in cases]
    for k, s in enumerate(singles):
        assert_same(batch.get_state(k), s.get_state(), ("init", k))
    for it in range(5):
        batch.step(1)
        for s in singles:
            s.step(1)
        for k, s in enumerate(singles):
            assert_same(batch.get_state(k), s.get_state(), ("iteration", it + 1, "instance", k))
    batch.step(3)
    for s in singles:
        s.step(3)
    for k, s in enumerate(singles):
        assert_same(batch.get_state(k), s.get_state(), ("iteration 8, instance", k))
        assert batch.best(k)[0] == s.best()[0]
        s.close()
    batch.close()


@pytest.mark.parametrize("engine", ["fused", "plain"])
def test_graph_replays_equal_eager(q, engine):
    """Handle a replays its captured graph; handle b launches eagerly (profiling
    on).  Every replay is compared, with exports (device-to-host copies and
    waits) between replays, then a run of replays back to back."""
    cases = mixed_cases()[:3] + mixed_cases()[-2:]
    announce("graph", engine)
    params = [q.make_params(engine=engine, **cfg) for _, _, cfg in cases]
    a = q.Swarm([(F, D) for F, D, _ in cases], params)
    b = q.Swarm([(F, D) for F, D, _ in cases], params)
    b.profile(True)
    for it in range(6):
        a.step(1)
        b.step(1)
        assert a.graph_active() and not b.graph_active()
        for k in range(len(cases)):
            assert_same(a.get_state(k), b.get_state(k), ("replay", it + 1, "instance", k))
    a.step(5)
    b.step(5)
    for k in range(len(cases)):
        assert_same(a.get_state(k), b.get_state(k), ("replays 7-11, instance", k))
    # longer steps replay graphs of several iterations (and single ones for the rest)
    a.step(19)
    b.step(19)
    for k in range(len(cases)):
        assert_same(a.get_state(k), b.get_state(k), ("replays 12-30, instance", k))
    # a state written between replays is picked up by the next replay
    st = b.get_state(0)
    a.set_state(st, 0)
    b.set_state(st, 0)
    a.step(2)
    b.step(2)
    assert_same(a.get_state(0), b.get_state(0), "after set_state")
    a.close()
    b.close()


@pytest.mark.parametrize("migration", [False, True], ids=["independent", "migration"])
def test_stream_groups_bit_identical(q, migration):
    """Swarms stepped as 1, 2 or 3 concurrent stream groups give identical
    states: the groups only partition the swarms.  In migration mode the
    groups join at every iteration where Alg. 2 is due and one launch ranks
    all swarms of the instance (period 10 here: several migrations in the run,
    steps that end on, before and after one); a final long step replays
    graphs of several iterations between the migrations."""
    F, D = gen.uniform_instance(64, 0, 99, 31)
    cfg = run_cfg(num_swarms=7, particles_per_swarm=9, seed=17, migration=migration,
                  migration_factor=0.3 if migration else 0.0, migration_period=10 if migration else 1)
    announce("stream groups", migration)
    hs = [q.Swarm.create(F, D, engine="fused", stream_groups=g, **cfg) for g in (1, 2, 3)]
    assert [h.stream_groups() for h in hs] == [1, 2, 3]
    moved = 0
    for it in range(5):
        before = hs[0].get_state()
        for h in hs:
            h.step(1 + it)
        ref = hs[0].get_state()
        for h in hs[1:]:
            assert_same(h.get_state(), ref, ("groups", h.stream_groups(), "after", it + 1))
            assert h.best()[0] == hs[0].best()[0]
        best_now = ref["goal"].reshape(7, 9).min(axis=1)
        moved += int((ref["goalPG"] != np.minimum(before["goalPG"], best_now)).sum())
    if migration:
        assert moved > 0  # Alg. 2 moved solutions within the run
    for h in hs:
        h.step(31)
    ref = hs[0].get_state()
    assert ref["t"] == 46
    for h in hs[1:]:
        assert_same(h.get_state(), ref, ("groups", h.stream_groups(), "after a long step"))
    for h in hs:
        h.close()
