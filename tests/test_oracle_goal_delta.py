"""Pins of the oracle's goal function (eq. qap) and pair-exchange deltas.

Checked against: eq. (qap) written with the permutation matrix X (x_ki = 1 iff
k = p(i)); brute force over all permutations; relabelling and transposition
invariance; the closed-form mean over random permutations; the D = a_k + a_l
family whose optimum is given by sorting; and recomputed cost differences.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import qap_inputs as gen


def perm_matrix(p):
    n = len(p)
    X = np.zeros((n, n), np.int64)
    X[np.asarray(p), np.arange(n)] = 1  # row = location, column = facility
    return X


def eq_qap(F, D, p):
    """Eq. (qap): sum_ijkl f_ij d_kl x_ki x_lj with the permutation matrix."""
    X = perm_matrix(p)
    return int(np.einsum("ij,kl,ki,lj->", F.astype(np.int64), D.astype(np.int64), X, X))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cost_equals_matrix_form(orc, seed):
    F, D = gen.general_instance(6, -9, 9, seed)
    for p in itertools.islice(itertools.permutations(range(6)), 0, 720, 37):
        assert orc.cost(F, D, p) == eq_qap(F, D, p)


def test_cost_trace_form(orc):
    # C(p) = tr(F X^T D^T X)... written via the location-space matrix X: C = tr(F^T X^T D X)
    F, D = gen.general_instance(9, -50, 50, 11)
    rng = np.random.default_rng(0)
    for _ in range(20):
        p = rng.permutation(9)
        X = perm_matrix(p)
        assert orc.cost(F, D, p) == int(np.trace(F.T.astype(np.int64) @ X.T @ D.astype(np.int64) @ X))


def test_relabel_and_transpose_invariance(orc):
    F, D = gen.general_instance(10, -20, 30, 5)
    rng = np.random.default_rng(1)
    for _ in range(20):
        p = rng.permutation(10)
        c = orc.cost(F, D, p)
        s = rng.permutation(10)   # facility relabelling F'[i][j] = F[s_i][s_j], p' = p o s
        assert orc.cost(F[np.ix_(s, s)], D, p[s]) == c
        tau = rng.permutation(10)  # location relabelling D'[k][l] = D[tau_k][tau_l], p' = tau^-1 o p
        tinv = np.argsort(tau)
        assert orc.cost(F, D[np.ix_(tau, tau)], tinv[p]) == c
        assert orc.cost(F.T.copy(), D.T.copy(), p) == c


def test_mean_over_all_permutations_closed_form(orc):
    n = 6
    F, D = gen.general_instance(n, 0, 9, 8)
    tot = sum(orc.cost(F, D, p) for p in itertools.permutations(range(n)))
    mean = Fraction(tot, 720)
    offF = int(F.sum() - np.trace(F))
    offD = int(D.sum() - np.trace(D))
    closed = Fraction(offF * offD, n * (n - 1)) + Fraction(int(np.trace(F)) * int(np.trace(D)), n)
    assert mean == closed


@pytest.mark.parametrize("n,seed", [(5, 21), (7, 22), (8, 23)])
def test_linear_sum_family_optimum_by_sorting(orc, n, seed):
    F, D, a = gen.linear_sum_instance(n, seed)
    # C(p) = sum_i a_{p_i} (rowsum_i + colsum_i): rearrangement inequality
    w = F.sum(1).astype(np.int64) + F.sum(0).astype(np.int64)
    p = np.zeros(n, np.int32)
    p[np.argsort(-w, kind="stable")] = np.argsort(a, kind="stable")
    best = min(orc.cost(F, D, q) for q in itertools.permutations(range(n)))
    assert orc.cost(F, D, p) == best == int((a[p] * w).sum())


def _swap(p, a, b):
    q = np.array(p, np.int32).copy()
    q[a], q[b] = q[b], q[a]
    return q


@pytest.mark.parametrize("kind,n,seed", [("sym", 12, 1), ("general", 15, 2), ("general", 30, 3),
                                         ("neg", 20, 4), ("sym", 40, 5)])
def test_delta_equals_recomputed_difference(orc, kind, n, seed):
    if kind == "sym":
        F, D = gen.uniform_instance(n, 0, 99, seed)
    elif kind == "neg":
        F, D = gen.general_instance(n, -128, 127, seed)
    else:
        F, D = gen.general_instance(n, 0, 1000, seed)
    p = np.random.default_rng(seed).permutation(n).astype(np.int32)
    c = orc.cost(F, D, p)
    Dm = orc.deltas(F, D, p)
    for a in range(n):
        assert Dm[a, a] == 0
        for b in range(a + 1, n):
            exp = orc.cost(F, D, _swap(p, a, b)) - c
            assert Dm[a, b] == exp and Dm[b, a] == exp
            assert orc.delta(F, D, p, b, a) == exp


def test_delta_sampled_large(orc):
    F, D = gen.general_instance(150, -1000, 1000, 9)
    p = np.random.default_rng(9).permutation(150).astype(np.int32)
    c = orc.cost(F, D, p)
    rng = np.random.default_rng(10)
    for _ in range(60):
        a, b = rng.choice(150, 2, replace=False)
        assert orc.delta(F, D, p, int(a), int(b)) == orc.cost(F, D, _swap(p, a, b)) - c


def test_local_search_picks_first_minimum(orc):
    F, D = gen.uniform_instance(14, 0, 20, 3)
    rng = np.random.default_rng(4)
    for _ in range(10):
        p = rng.permutation(14).astype(np.int32)
        c = orc.cost(F, D, p)
        q, g, (a, b, bd), sw = orc.local_search(F, D, p)
        Dm = orc.deltas(F, D, p)
        iu = np.triu_indices(14, 1)
        m = Dm[iu].min()
        first = [(i, j) for i, j in zip(*iu) if Dm[i, j] == m][0]
        assert (a, b) == first and bd == m
        if m < 0:
            assert sw and g == c + m and g == orc.cost(F, D, q)
            assert np.array_equal(q, _swap(p, a, b))
        else:
            assert not sw and g == c and np.array_equal(q, p)


def test_local_search_at_brute_force_optimum_is_noop(orc):
    F, D = gen.uniform_instance(7, 0, 10, 201)
    perms = list(itertools.permutations(range(7)))
    costs = [orc.cost(F, D, p) for p in perms]
    opt = np.array(perms[int(np.argmin(costs))], np.int32)
    q, g, (_, _, bd), sw = orc.local_search(F, D, opt)
    assert not sw and bd >= 0 and g == min(costs)
