"""Pins of the oracle's position update (S_x = SecondTarget, Alg. 1) and
velocity update (eq. velocity with S_v raw / norm), Sec. 3.1.

SecondTarget is pinned by the paper's 3x3 examples (golden fixture), by a
sort-based greedy matching (a different algorithm with the same result when
keys are distinct), by its invariants, and by the uniformity of its random
tie-break.  The velocity update is pinned by closed forms and a hand example.
"""
import os
from collections import Counter

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def load_example():
    mats = {}
    for line in open(os.path.join(HERE, "golden", "paper_3x3_example.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tag, *vals = line.split()
        mats.setdefault(tag, []).append([int(v) for v in vals])
    return {k: np.array(v) for k, v in mats.items()}


def perm_of(M):
    """p[c] = row of the 1 in column c."""
    M = np.asarray(M)
    assert (M.sum(0) == 1).all() and (M.sum(1) == 1).all()
    return np.argmax(M, axis=0).astype(np.int32)


def test_paper_example_globalmax_stagnates(orc):
    ex = load_example()
    z = perm_of(ex["X"])
    W = (ex["X"] + ex["V"]).astype(np.float32)
    out = orc.second_target(W, z, depth=0)
    assert np.array_equal(out, perm_of(ex["GLOBALMAX"]))
    assert np.array_equal(out, z)  # X(t+1) = X(t): the stagnation of Sec. 3.1


def test_paper_example_depth2_second_variant(orc):
    ex = load_example()
    z = perm_of(ex["X"])
    W = (ex["X"] + ex["V"]).astype(np.float32)
    out, ties = orc.second_target(W, z, depth=2, return_ties=True)
    assert np.array_equal(out, perm_of(ex["DEPTH2"]))
    assert list(ties) == [1, 1, 1]


def test_paper_example_depth1_differs_from_printed(orc):
    """The printed depth-1 matrix takes the cell z = 1 (value 6) first, which
    Alg. 1 excludes from the first selection.  Taking Alg. 1 literally, the
    first pick is 4 at (row 2, col 2) (1-based), then 8, then 2."""
    ex = load_example()
    z = perm_of(ex["X"])
    W = (ex["X"] + ex["V"]).astype(np.float32)
    out = orc.second_target(W, z, depth=1)
    assert np.array_equal(out, [0, 1, 2])
    assert not np.array_equal(out, perm_of(ex["DEPTH1_PRINTED"]))


def greedy_by_sort(W, z, depth):
    """Sequential greedy on cells sorted by key (distinct keys): accept a
    cell whose row and column are free; the first `depth` acceptances skip
    cells of Z, after which the scan restarts from the top over all cells."""
    n = W.shape[0]
    order = np.argsort(-W, axis=None, kind="stable")
    rows_used, cols_used = set(), set()
    out = -np.ones(n, np.int32)
    taken = 0
    for phase in (0, 1):
        for flat in order:
            if phase == 0 and taken >= depth:
                break
            r, c = divmod(int(flat), n)
            if r in rows_used or c in cols_used:
                continue
            if phase == 0 and z[c] == r:
                continue
            out[c] = r
            rows_used.add(r)
            cols_used.add(c)
            taken += 1
    return out


@pytest.mark.parametrize("n,depth,seed", [(5, 0, 1), (8, 2, 2), (16, 3, 3), (33, 2, 4), (64, 7, 5), (128, 2, 6)])
def test_secondtarget_equals_sorted_greedy(orc, n, depth, seed):
    rng = np.random.default_rng(seed)
    z = rng.permutation(n).astype(np.int32)
    V = rng.standard_normal((n, n))
    W = orc.keys(V, z)
    assert len(np.unique(W)) == n * n
    out, ties = orc.second_target(W, z, depth, return_ties=True)
    assert (ties == 1).all()
    assert np.array_equal(out, greedy_by_sort(W, z, depth))


@pytest.mark.parametrize("n,depth", [(6, 0), (6, 5), (20, 3), (50, 49)])
def test_secondtarget_invariants(orc, n, depth):
    rng = np.random.default_rng(n + depth)
    for trial in range(20):
        z = rng.permutation(n).astype(np.int32)
        # quantised keys make exact ties frequent
        V = rng.integers(-2, 3, size=(n, n)).astype(np.float64) / 2
        W = orc.keys(V, z)
        out, ties = orc.second_target(W, z, depth, seed=trial, t=3, particle=1, swarm=2, return_ties=True)
        assert sorted(out) == list(range(n))           # a permutation
        assert (out != z).sum() >= depth               # the first depth picks avoid Z
        assert (ties >= 1).all()


def test_tiebreak_enumeration_order(orc):
    """Two tied maxima (0,1) and (1,0): in column-major order (1,0) comes first;
    the pick is the k-th with k = bounded(word of element 4 + 0, 2)."""
    W = np.array([[0.0, 5.0, 0.0], [5.0, 0.0, 0.0], [0.0, 0.0, 1.0]], np.float32)
    z = np.array([0, 1, 2], np.int32)
    seen = Counter()
    for seed in range(40):
        out, ties = orc.second_target(W, z, depth=0, seed=seed, t=1, return_ties=True)
        assert ties[0] == 2
        k = orc.bounded(orc.word(seed, 4, 1, 0, 0), 2)
        first = (1, 0) if k == 0 else (0, 1)   # (row, col)
        assert out[first[1]] == first[0]
        seen[k] += 1
    assert seen[0] > 5 and seen[1] > 5


def test_all_tied_keys_give_uniform_permutations(orc):
    # with every key equal, sequential uniform picks make every permutation equally likely
    n = 3
    W = np.zeros((n, n), np.float32)
    z = np.arange(n, dtype=np.int32)
    cnt = Counter()
    N = 6000
    for s in range(N):
        cnt[tuple(orc.second_target(W, z, 0, seed=s, t=1))] += 1
    assert len(cnt) == 6
    exp = N / 6
    chi2 = sum((c - exp) ** 2 / exp for c in cnt.values())
    assert chi2 < 20.5  # 5 dof, p ~ 1e-3


def test_keys_add_one_on_z_cells(orc):
    V = np.array([[0.25, -0.5], [1e-9, 0.75]])
    z = np.array([1, 0], np.int32)  # facility 0 at location 1, facility 1 at location 0
    W = orc.keys(V, z)
    assert W.dtype == np.float32
    assert W[1, 0] == np.float32(1.0) + np.float32(1e-9)   # rounds to 1 in binary32
    assert W[0, 1] == np.float32(0.5)
    assert W[0, 0] == np.float32(0.25) and W[1, 1] == np.float32(0.75)


# ---------------------------------------------------------------- velocity
def test_velocity_hand_example(orc):
    V = np.array([[0.5, -0.25], [0.125, 1.0]])
    p = np.array([0, 1], np.int32)    # X = identity
    pl = np.array([1, 1], np.int32)   # P^L: facility 0 at location 1
    pg = np.array([0, 0], np.int32)   # P^G: facility 1 at location 0 (not a permutation; cells only)
    c1, c2, c3, r2, r3 = 0.5, 0.5, 0.25, 0.5, 1.0
    raw = orc.velocity(V, p, pl, pg, c1, c2, c3, r2, r3, vmax=10.0, norm=False)
    # (0,0): 0.25 + 0.25*(0-1) + 0.25*(1-1) = 0 ; (1,0): 0.0625 + 0.25*(1-0) + 0 = 0.3125
    # (0,1): -0.125 + 0 + 0.25*(1-0) = 0.125   ; (1,1): 0.5 + 0.25*(1-1) + 0.25*(0-1) = 0.25
    assert np.array_equal(raw, [[0.0, 0.125], [0.3125, 0.25]])
    clamp = orc.velocity(V, p, pl, pg, c1, c2, c3, r2, r3, vmax=0.2, norm=False)
    assert np.array_equal(clamp, [[0.0, 0.125], [0.2, 0.2]])
    nrm = orc.velocity(V, p, pl, pg, c1, c2, c3, r2, r3, vmax=10.0, norm=True)
    assert np.allclose(nrm, [[0.0, 0.125 / 0.375], [1.0, 0.25 / 0.375]], rtol=0, atol=1e-15)


@pytest.mark.parametrize("norm", [False, True])
def test_velocity_closed_forms(orc, norm):
    rng = np.random.default_rng(3)
    n = 17
    V = rng.uniform(-2, 2, (n, n))
    p, pl, pg = (rng.permutation(n).astype(np.int32) for _ in range(3))

    def sv(T, vmax):
        T = np.clip(T, -vmax, vmax)
        if norm:
            s = np.abs(T).sum(0)
            T = np.where(s > 0, T / np.where(s > 0, s, 1), 0)
        return T

    # c2 = c3 = 0: V' = S_v(c1 V)
    out = orc.velocity(V, p, pl, pg, 0.7, 0.0, 0.0, 0.3, 0.9, 1.5, norm)
    assert np.allclose(out, sv(0.7 * V, 1.5), rtol=0, atol=1e-14)
    # X = P^L = P^G: the attraction terms vanish
    out = orc.velocity(V, p, p, p, 0.7, 0.5, 0.5, 0.3, 0.9, 1.5, norm)
    assert np.allclose(out, sv(0.7 * V, 1.5), rtol=0, atol=1e-14)
    out = orc.velocity(V, p, pl, pg, 0.8, 0.5, 0.5, 0.4, 0.6, 1.0, norm)
    assert np.abs(out).max() <= 1.0
    if norm:
        s = np.abs(out).sum(0)
        assert np.allclose(s[s > 0], 1.0, rtol=0, atol=1e-14)


def test_velocity_zero_column_stays_zero(orc):
    n = 4
    V = np.zeros((n, n))
    p = np.arange(n, dtype=np.int32)
    out = orc.velocity(V, p, p, p, 0.5, 0.5, 0.5, 0.5, 0.5, 1.0, True)
    assert (out == 0).all()
