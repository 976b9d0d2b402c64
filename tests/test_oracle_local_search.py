"""The oracle's local search inside a particle-iteration: after S_x, up to L
best-improvement pair exchanges (smallest delta, ties to the smallest a then
b), each made only if it lowers the goal.  Pinned against brute force: every
candidate exchange is evaluated by recomputing the goal of the exchanged
permutation from the definition of the QAP cost (eq. qap), not by the
pair-exchange delta formula the oracle uses."""
import numpy as np
import pytest

import qap_inputs as gen


def brute_cost(F, D, p):
    n = len(p)
    return int(sum(int(F[i, j]) * int(D[p[i], p[j]]) for i in range(n) for j in range(n)))


def brute_exchanges(F, D, p, L):
    p = np.array(p, np.int64)
    c = brute_cost(F, D, p)
    for _ in range(L):
        best = None
        n = len(p)
        for a in range(n):
            for b in range(a + 1, n):
                q = p.copy()
                q[a], q[b] = q[b], q[a]
                d = brute_cost(F, D, q) - c
                if best is None or d < best[0]:
                    best = (d, a, b)
        if best is None or best[0] >= 0:
            break
        d, a, b = best
        p[a], p[b] = p[b], p[a]
        c += d
    return p, c


@pytest.mark.parametrize("L", [1, 2, 5, 10000])
@pytest.mark.parametrize("kind", ["sym", "gen"])
def test_step_makes_up_to_L_best_exchanges(orc, L, kind):
    n = 9
    if kind == "sym":
        F, D = gen.uniform_instance(n, 0, 20, 7)
    else:
        F, D = gen.general_instance(n, -5, 20, 8)
    sw = orc.OracleSwarm(F, D, num_swarms=2, particles_per_swarm=3, local_search=L, seed=4)
    for it in range(3):
        st = sw.state()
        t1 = sw.t + 1
        sw.step()
        for k in range(sw.P):
            g, s = divmod(k, sw.S)
            xs = orc.second_target(orc.keys(st["V"][k], st["X"][k]), st["X"][k], sw.depth, seed=sw.seed, t=t1,
                                   particle=s, swarm=g)
            p, c = brute_exchanges(F, D, xs, L)
            assert np.array_equal(sw.X[k], p), (kind, L, it, k)
            assert int(sw.goal[k]) == c == brute_cost(F, D, sw.X[k])


def test_many_exchanges_end_at_a_local_optimum(orc):
    F, D = gen.uniform_instance(10, 0, 30, 12)
    sw = orc.OracleSwarm(F, D, num_swarms=1, particles_per_swarm=4, local_search=10000, seed=9)
    sw.step(2)
    for k in range(sw.P):
        p = sw.X[k].astype(np.int64)
        c = brute_cost(F, D, p)
        for a in range(10):
            for b in range(a + 1, 10):
                q = p.copy()
                q[a], q[b] = q[b], q[a]
                assert brute_cost(F, D, q) >= c
