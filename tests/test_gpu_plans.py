"""Launch plans and the autotuner.

A plan (stream chains; swarms, whole instances or whole kernel classes over
the chains; eager launches or graphs of k iterations) changes only how
iterations are launched: states must be bit-identical under every plan, also
when the plan changes between steps.
The tuner must leave the handle exactly in the state its initialisation made,
on the plan it reports, and record that plan in the cache file named by
QAP_SWARM_TUNE_CACHE, from which a new handle of the same workload starts.
"""
import os

import numpy as np
import pytest

import qap_inputs as gen
from _parity import announce, run_cfg

pytestmark = pytest.mark.gpu

KEYS = ("V", "X", "PL", "goal", "goalPL", "PG", "goalPG", "best_perm", "best_goal", "best_info", "t")


def assert_same(a, b, what):
    for k in KEYS:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (what, k)


def cases():
    """Mixed padded sizes, a byte-split one, an int32 one and a migrating one."""
    out = []
    for i, (F, D) in enumerate(gen.mixed_batch(count=4, seed=106, lo_n=20, hi_n=150)):
        out.append((F, D, run_cfg(num_swarms=3 + i % 2, particles_per_swarm=6 + i, seed=40 + i)))
    F, D = gen.uniform_instance(48, 0, 99, 61, d_hi=900)
    out.append((F, D, run_cfg(num_swarms=4, particles_per_swarm=5, seed=46)))            # byte-split
    F, D = gen.general_instance(30, -500, 500, 62)
    out.append((F, D, run_cfg(num_swarms=2, particles_per_swarm=5, seed=47)))            # int32
    F, D = gen.uniform_instance(40, 0, 99, 63)
    out.append((F, D, run_cfg(num_swarms=7, particles_per_swarm=4, migration=True, migration_factor=0.3,
                              migration_period=5, seed=48)))                            # migration
    return out


def make(q, cs):
    return q.Swarm([(F, D) for F, D, _ in cs], [q.make_params(engine="fused", **c) for _, _, c in cs])


PLANS = [(1, 0, 0), (2, 0, 1), (3, 0, 8), (4, 0, 8), (1, 1, 8), (2, 1, 0), (3, 1, 1), (4, 1, 8), (3, 0, 16),
         (2, 2, 8), (4, 2, 0), (3, 2, 1)]


def test_states_identical_under_every_plan(q):
    cs = cases()
    announce("plans", len(PLANS))
    ref = make(q, cs)
    ref.set_plan(1, 0, 0)
    ref.step(23)
    want = [ref.get_state(k) for k in range(len(cs))]
    ref.close()
    for chains, split, ipg in PLANS:
        h = make(q, cs)
        h.set_plan(chains, split, ipg)
        assert h.plan() == dict(stream_chains=chains, split=split, iters_per_graph=ipg)
        h.step(7)
        h.step(16)
        for k in range(len(cs)):
            assert_same(h.get_state(k), want[k], ("plan", chains, split, ipg, "instance", k))
        h.close()


def test_plan_changes_between_steps(q):
    cs = cases()
    announce("plan changes")
    ref = make(q, cs)
    ref.set_plan(1, 0, 0)
    h = make(q, cs)
    for i, (chains, split, ipg) in enumerate(PLANS):
        ref.step(3 + i)
        h.set_plan(chains, split, ipg)
        h.step(3 + i)
        for k in range(len(cs)):
            assert_same(h.get_state(k), ref.get_state(k), ("after plan", chains, split, ipg, "instance", k))
    ref.close()
    h.close()


def test_tune_returns_to_the_initial_state_and_caches_its_choice(q, tmp_path):
    cs = cases()
    cache = tmp_path / "plans.txt"
    announce("tune")
    old = os.environ.get("QAP_SWARM_TUNE_CACHE")
    os.environ["QAP_SWARM_TUNE_CACHE"] = str(cache)
    try:
        fresh = make(q, cs)  # no cache entry yet: the default plan
        assert fresh.plan() == dict(stream_chains=3, split=0, iters_per_graph=8)
        h = make(q, cs)
        chosen = h.tune(8)
        assert chosen["ms_per_iteration"] > 0
        got = h.plan()
        assert got == {k: chosen[k] for k in got}
        for k in range(len(cs)):
            assert_same(h.get_state(k), fresh.get_state(k), ("after tune", k))
        h.step(11)
        fresh.step(11)
        for k in range(len(cs)):
            assert_same(h.get_state(k), fresh.get_state(k), ("stepped after tune", k))
        with pytest.raises(q.QapError) as e:
            h.tune(8)  # only before the first step
        assert e.value.code == q.QAP_ERR_INVALID_ARG
        lines = cache.read_text().split()
        assert len(lines) == 5
        again = make(q, cs)  # same workload: starts on the cached plan
        assert again.plan() == got
        for s in (fresh, h, again):
            s.close()
    finally:
        if old is None:
            os.environ.pop("QAP_SWARM_TUNE_CACHE", None)
        else:
            os.environ["QAP_SWARM_TUNE_CACHE"] = old
    with pytest.raises(q.QapError) as e:
        bad = make(q, cs)
        try:
            bad.set_plan(q.QAP_MAX_CHAINS + 1, 0, 8)
        finally:
            bad.close()
    assert e.value.code == q.QAP_ERR_INVALID_ARG


def test_tune_keeps_chains_within_the_hardware_queues(q):
    """With GPU_MAX_HW_QUEUES = 2 only one chain fits beside the handle's own
    stream's queue: the tuner then times single-chain plans only."""
    cs = cases()
    announce("tune, queue bound")
    old = os.environ.get("GPU_MAX_HW_QUEUES")
    os.environ["GPU_MAX_HW_QUEUES"] = "2"
    try:
        h = make(q, cs)
        chosen = h.tune(4)
        assert chosen["stream_chains"] == 1
        assert h.plan()["stream_chains"] == 1
        h.close()
    finally:
        if old is None:
            os.environ.pop("GPU_MAX_HW_QUEUES", None)
        else:
            os.environ["GPU_MAX_HW_QUEUES"] = old
