"""Population statistics on the device (percentile ranks and PMF counts of
the current goals, per swarm and over the population) against the oracle's
definitions on the exported goals: exact."""
import numpy as np
import pytest

import qap_inputs as gen
from _parity import announce, make_gpu, run_cfg

pytestmark = pytest.mark.gpu

Q = [1, 50000, 250000, 500000, 750000, 999999, 1000000]


def check(q, orc, sw, bins, lo, hi):
    st = sw.get_state()
    m, S = sw.ms[0], sw.Ss[0]
    got = sw.stats(Q, bins, lo, hi)
    goals = st["goal"]
    for g in range(m):
        seg = goals[g * S:(g + 1) * S]
        assert np.array_equal(got["swarm_q"][g], orc.nearest_rank_quantiles(seg, Q)), g
        assert np.array_equal(got["swarm_hist"][g], orc.goal_histogram(seg, bins, lo, hi)), g
    assert np.array_equal(got["pop_q"], orc.nearest_rank_quantiles(goals, Q))
    assert np.array_equal(got["pop_hist"], orc.goal_histogram(goals, bins, lo, hi))


def test_stats_general_instance_negative_goals(q, orc):
    F, D = gen.general_instance(24, -40, 30, 3)
    cfg = run_cfg(num_swarms=5, particles_per_swarm=13, seed=8)
    announce("stats general")
    sw = make_gpu(q, F, D, dict(cfg, engine="fused"))
    for it in range(3):
        sw.step(1)
        goals = sw.get_state()["goal"]
        lo, hi = int(goals.min()) + 3, int(goals.max())  # some goals fall outside [lo, hi)
        check(q, orc, sw, 17, lo, hi)
    sw.close()


def test_stats_headline_size(q, orc):
    F, D = gen.uniform_instance(128, 0, 127, 104)
    cfg = run_cfg(num_swarms=200, particles_per_swarm=50, seed=1)
    announce("stats headline")
    sw = make_gpu(q, F, D, dict(cfg, engine="fused"))
    sw.step(5)
    goals = sw.get_state()["goal"]
    check(q, orc, sw, 64, int(goals.min()), int(goals.max()) + 1)
    sw.close()


def test_stats_single_particle_swarms_and_errors(q, orc):
    F, D = gen.uniform_instance(12, 0, 10, 101)
    cfg = run_cfg(num_swarms=6, particles_per_swarm=1, seed=2)
    announce("stats S=1")
    sw = make_gpu(q, F, D, dict(cfg, engine="plain"))
    sw.step(2)
    check(q, orc, sw, 1, -10**12, 10**12)
    goals = sw.get_state()["goal"]
    got = sw.stats(Q)
    assert (got["swarm_q"] == goals[:, None]).all()
    for bad in (dict(q_ppm=[0]), dict(q_ppm=[1000001]), dict(bins=5, lo=3, hi=3), dict(bins=5000, lo=0, hi=9),
                dict(bins=2, lo=-(2**62), hi=2**62)):
        with pytest.raises(q.QapError):
            sw.stats(**bad)
    sw.close()
