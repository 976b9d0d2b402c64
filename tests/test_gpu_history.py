"""Per-iteration statistics recorded on the device during stepping (the
percentile ranks and PMFs of Sec. 4.2 followed iteration by iteration),
against the oracle's definitions applied to the goals of each iteration:
with several stream chains, in a batch where one instance records, across
the wrap-around of the ring, after a restart, and with migration."""
import numpy as np
import pytest

import qap_inputs as gen
from _parity import announce, run_cfg

pytestmark = pytest.mark.gpu

Q = (10000, 50000, 250000, 500000, 750000, 1000000)


def _check_records(orc, rec, goals_by_t, m, S, bins, lo, hi):
    for r, t in enumerate(rec["iters"]):
        g = goals_by_t[int(t)]
        for s in range(m):
            seg = g[s * S:(s + 1) * S]
            assert np.array_equal(rec["swarm_q"][r][s], orc.nearest_rank_quantiles(seg, Q)), (t, s)
            if bins:
                assert np.array_equal(rec["swarm_hist"][r][s], orc.goal_histogram(seg, bins, lo, hi)), (t, s)
        assert np.array_equal(rec["pop_q"][r], orc.nearest_rank_quantiles(g, Q)), t
        if bins:
            assert np.array_equal(rec["pop_hist"][r], orc.goal_histogram(g, bins, lo, hi)), t


@pytest.mark.parametrize("chains", [1, 3])
def test_history_matches_the_statistics_of_each_iteration(q, orc, chains):
    F, D = gen.uniform_instance(45, 0, 99, 71)
    F2, D2 = gen.uniform_instance(70, 0, 99, 72)
    cfgs = [run_cfg(num_swarms=5, particles_per_swarm=13, seed=8, migration=True, migration_factor=0.2,
                    migration_period=4),
            run_cfg(num_swarms=3, particles_per_swarm=9, seed=9)]
    announce("history", chains)
    h = q.Swarm([(F, D), (F2, D2)], [q.make_params(engine="fused", **c) for c in cfgs])
    h.set_plan(chains, 0, 8)
    g0 = h.get_state(0)["goal"]
    lo, hi, bins = int(g0.min()) - 1000, int(g0.max()) + 1, 24
    h.history_start(6, Q, bins, lo, hi, instance=0)
    goals = {}
    for t in range(1, 11):
        h.step(1)
        goals[t] = h.get_state(0)["goal"]
    rec = h.history_read(instance=0)
    assert list(rec["iters"]) == [5, 6, 7, 8, 9, 10]  # the ring holds the latest 6
    _check_records(orc, rec, goals, 5, 13, bins, lo, hi)
    assert len(h.history_read(max_records=2, instance=0)["iters"]) == 2
    with pytest.raises(q.QapError):
        h.history_read(instance=1)  # not recording
    # a longer step records every iteration as well; a restart drops the old records
    h.step(3)
    rec = h.history_read(instance=0)
    assert list(rec["iters"]) == [8, 9, 10, 11, 12, 13]
    h.history_start(4, Q, 0, 0, 1, instance=0)  # percentiles only
    assert len(h.history_read(instance=0)["iters"]) == 0
    for t in range(14, 17):
        h.step(1)
        goals[t] = h.get_state(0)["goal"]
    rec = h.history_read(instance=0)
    assert list(rec["iters"]) == [14, 15, 16]
    _check_records(orc, rec, goals, 5, 13, 0, 0, 1)
    h.history_stop(instance=0)
    with pytest.raises(q.QapError):
        h.history_read(instance=0)
    h.close()
