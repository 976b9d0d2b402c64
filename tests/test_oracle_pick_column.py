"""PickColumn (Sec. 3.1, the second S_x procedure), as read: columns visited in
a Fisher-Yates order from the particle's stream, each taking its largest key
over the rows left.  Pinned by properties independent of the oracle's code."""
import itertools

import numpy as np
import pytest


def visit_order(orc, n, seed, t, particle, swarm):
    """The column order of the reading, restated: for i = n-1 .. 1 swap
    positions i and bounded(element 4 + n + (n-1-i), i+1) of 0 .. n-1."""
    order = list(range(n))
    for i in range(n - 1, 0, -1):
        j = orc.bounded(orc.word(seed, 4 + n + (n - 1 - i), t, particle, swarm), i + 1)
        order[i], order[j] = order[j], order[i]
    return order


@pytest.mark.parametrize("n", [1, 2, 5, 17, 64])
def test_output_is_a_permutation(orc, n):
    rng = np.random.default_rng(n)
    W = rng.integers(-3, 4, size=(n, n)).astype(np.float32)  # many ties
    for particle in range(6):
        p = orc.pick_column(W, seed=2, t=3, particle=particle, swarm=1)
        assert sorted(p.tolist()) == list(range(n))


def test_unique_column_maxima_in_distinct_rows_fix_the_result(orc):
    """If every column's largest key is unique and the rows of these maxima
    differ, every visit order gives that permutation."""
    n = 12
    rng = np.random.default_rng(5)
    pi = rng.permutation(n)
    W = rng.random((n, n)).astype(np.float32)
    W[pi, np.arange(n)] = 10.0 + np.arange(n)
    for particle in range(20):
        assert np.array_equal(orc.pick_column(W, seed=7, t=1, particle=particle, swarm=0), pi)


def test_each_visited_column_takes_its_largest_remaining_key(orc):
    n = 20
    rng = np.random.default_rng(11)
    W = rng.permutation(n * n).reshape(n, n).astype(np.float32)  # distinct keys
    for particle in range(8):
        p = orc.pick_column(W, seed=3, t=4, particle=particle, swarm=2)
        left = set(range(n))
        for c in visit_order(orc, n, 3, 4, particle, 2):
            best = max(left, key=lambda r: W[r, c])
            assert p[c] == best
            left.remove(best)


def test_all_ties_give_uniform_permutations(orc):
    """All keys equal: the procedure draws a uniformly random permutation."""
    n, N = 3, 6000
    W = np.zeros((n, n), np.float32)
    perms = list(itertools.permutations(range(n)))
    counts = np.zeros(len(perms))
    for particle in range(N):
        p = tuple(orc.pick_column(W, seed=9, t=2, particle=particle, swarm=0).tolist())
        counts[perms.index(p)] += 1
    e = N / len(perms)
    chi2 = float(((counts - e) ** 2 / e).sum())
    assert chi2 < 20.5  # 5 degrees of freedom, p ~ 0.001
