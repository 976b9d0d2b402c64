"""Byte-split MFMA path: symmetric instances whose F or D leave the int8 range.

Each matrix outside [-128, 127] is split into a low plane (M mod 128) and a
high plane (floor(M / 128)); the plane products run on int8 MFMA and are
combined in int32.  Goals and deltas must equal the oracle's exactly, and whole
iterations must match the oracle's as in the other parity tests; the cases
cover F split, D split, both split, non-zero diagonals, negative entries,
ragged sizes over every padded size, and deltas near the int32 bound that makes
an instance eligible.
"""
import numpy as np
import pytest

import qap_inputs as gen
from _parity import announce, assert_states_equal, make_gpu, oracle_from_state, run_cfg

pytestmark = pytest.mark.gpu


def sym(n, f, d, seed, zero_diag=True):
    rng = np.random.default_rng(seed)
    F = gen.symmetric_uniform(n, f[0], f[1], rng, zero_diag=zero_diag)
    D = gen.symmetric_uniform(n, d[0], d[1], rng, zero_diag=zero_diag)
    return F, D


def signs_instance(n, mag, seed):
    """F = mag s s^T, D = mag t t^T for random sign vectors: every product has
    the same size, so goals and deltas reach a large part of the bound
    8 (n + 3) max|F| max|D| < 2^31 that admits the instance."""
    rng = np.random.default_rng(seed)
    s = rng.choice([-1, 1], size=n)
    t = rng.choice([-1, 1], size=n)
    return (mag * np.outer(s, s)).astype(np.int32), (mag * np.outer(t, t)).astype(np.int32)


def aligned_perm(F, D):
    """A permutation putting facility i on a location whose sign in D's first
    column matches i's sign in F's first column, as far as the counts allow:
    for signs_instance this makes |sum_i s_i t_(p_i)| as large as it gets, and
    with it the goal and the deltas."""
    n = F.shape[0]
    s = np.where(F[:, 0] >= 0, 1, -1)
    t = np.where(D[:, 0] >= 0, 1, -1)
    p = np.empty(n, np.int32)
    free = {1: list(np.flatnonzero(t > 0)), -1: list(np.flatnonzero(t < 0))}
    rest = []
    for i in range(n):
        if free[int(s[i])]:
            p[i] = free[int(s[i])].pop()
        else:
            rest.append(i)
    left = free[1] + free[-1]
    for i, loc in zip(rest, left):
        p[i] = loc
    assert sorted(p) == list(range(n))
    return p


def with_entry(FD, i, j, v):
    """F with F[i][j] = F[j][i] = v (still symmetric)."""
    F, D = FD
    F = F.copy()
    F[i, j] = F[j, i] = v
    return F, D


# (name, instance, split pattern: 1 F, 2 D, 3 both)
CASES = [
    ("D-n12", lambda: sym(12, (0, 10), (0, 1000), 1), 2),
    ("F-n37-neg", lambda: sym(37, (-3000, 3000), (0, 127), 2), 1),
    ("FD-n64-diag", lambda: sym(64, (-2000, 2000), (-300, 300), 3, zero_diag=False), 3),
    ("D-n100-diag", lambda: sym(100, (-128, 127), (0, 16383), 4, zero_diag=False), 2),
    ("F-n100-euclid", lambda: gen.euclid_sparse_instance(100, 103), 1),  # D at most 121 at this seed
    ("FD-n128", lambda: sym(128, (0, 2980), (0, 141), 5), 3),
    ("D-n150", lambda: sym(150, (0, 127), (0, 1000), 6), 2),
    ("F-n150-diag", lambda: sym(150, (-16384, 16383), (-20, 20), 7, zero_diag=False), 1),
    ("FD-n60-bound", lambda: signs_instance(60, 2000, 8), 3),
]
IDS = [c[0] for c in CASES]


@pytest.mark.parametrize("name,mk,split", CASES, ids=IDS)
def test_split_path_is_chosen(q, name, mk, split):
    F, D = mk()
    announce("split-path", name)
    sw = make_gpu(q, F, D, run_cfg(num_swarms=1, particles_per_swarm=2, engine="fused"))
    assert sw.path() == ("split", True)
    sw.close()
    sw = make_gpu(q, F, D, run_cfg(num_swarms=1, particles_per_swarm=2, engine="plain"))
    assert sw.path() == ("int32", True)
    sw.close()


@pytest.mark.parametrize("name,mk,split", CASES, ids=IDS)
def test_split_eval_goals_and_deltas_exact(q, orc, name, mk, split):
    F, D = mk()
    n = F.shape[0]
    announce("split-eval", name)
    sw = make_gpu(q, F, D, run_cfg(num_swarms=1, particles_per_swarm=2, engine="fused"))
    perms = list(gen.random_perms(5, n, 11))
    perms.append(np.arange(n, dtype=np.int32))
    perms.append(np.arange(n, dtype=np.int32)[::-1].copy())
    perms.append(aligned_perm(F, D))
    perms = np.stack(perms)
    goals, dl = sw.eval(perms, deltas=True)
    big = 0
    for i, p in enumerate(perms):
        assert goals[i] == orc.cost(F, D, p), (name, i)
        ref = orc.deltas(F, D, p)
        assert np.array_equal(dl[i], ref), (name, i, np.argwhere(dl[i] != ref)[:3])
        big = max(big, int(np.abs(ref).max()))
    if name.endswith("bound"):
        assert big > 2 ** 29, big  # the int32 epilogue is exercised near its range
    sw.close()


@pytest.mark.parametrize("ls", [True, 3])
@pytest.mark.parametrize("name,mk,split", CASES, ids=IDS)
def test_split_one_step_parity(q, orc, name, mk, split, ls):
    F, D = mk()
    n = F.shape[0]
    cfg = run_cfg(num_swarms=2, particles_per_swarm=6, depth=min(2, n - 1), local_search=ls, seed=5 + n)
    announce("split-onestep", name, ls)
    sw = make_gpu(q, F, D, dict(cfg, engine="fused"))
    assert sw.path()[0] == "split"
    for it in range(3):
        st = sw.get_state()
        o = oracle_from_state(orc, F, D, cfg, st)
        o.step()
        sw.step(1)
        assert_states_equal(sw.get_state(), o.state(), what="%s iteration %d" % (name, it + 1))
    sw.close()


def test_split_requested_on_int8_data(q, orc):
    """delta_path='split' on data that fits int8: F is split all the same
    (its high plane holds 0 or -1, negative entries included) and the result
    is exact."""
    F, D = gen.general_instance(30, -128, 127, 9)
    F = (F + F.T) // 2
    D = (D + D.T) // 2
    cfg = run_cfg(num_swarms=2, particles_per_swarm=5, seed=4)
    announce("split-int8-data")
    sw = make_gpu(q, F, D, dict(cfg, engine="fused", delta_path="split"))
    assert sw.path() == ("split", True)
    perms = gen.random_perms(4, 30, 2)
    goals, dl = sw.eval(perms, deltas=True)
    for i, p in enumerate(perms):
        assert goals[i] == orc.cost(F, D, p)
        assert np.array_equal(dl[i], orc.deltas(F, D, p))
    st = sw.get_state()
    o = oracle_from_state(orc, F, D, cfg, st)
    o.step()
    sw.step(1)
    assert_states_equal(sw.get_state(), o.state(), what="split on int8 data")
    sw.close()


@pytest.mark.parametrize("what,mk", [
    ("asymmetric", lambda: gen.general_instance(40, -3000, 3000, 10)),
    ("beyond-15-bits", lambda: with_entry(sym(40, (0, 16383), (0, 10), 11), 0, 1, 16384)),
    ("both-split-npad160", lambda: sym(150, (0, 1000), (0, 1000), 12)),
    ("over-the-delta-bound", lambda: signs_instance(60, 2100, 13)),
])
def test_ineligible_instances_take_int32(q, what, mk):
    F, D = mk()
    announce("split-ineligible", what)
    sw = make_gpu(q, F, D, run_cfg(num_swarms=1, particles_per_swarm=2, engine="fused"))
    assert sw.path()[0] == "int32"
    sw.close()
    with pytest.raises(q.QapError) as e:
        make_gpu(q, F, D, run_cfg(num_swarms=1, particles_per_swarm=2, engine="fused", delta_path="split"))
    assert e.value.code == q.QAP_ERR_RANGE


def test_split_batch_equals_separate_handles(q):
    """One handle over int8 and byte-split instances (both kinds of split, two
    padded sizes) gives exactly the states of separate handles."""
    cases = [
        (sym(40, (0, 127), (0, 127), 20), run_cfg(seed=31)),
        (sym(40, (0, 127), (0, 900), 21), run_cfg(seed=32)),
        (sym(70, (-2000, 2000), (0, 200), 22, zero_diag=False), run_cfg(seed=33, particles_per_swarm=7)),
        (sym(100, (0, 3000), (0, 127), 23), run_cfg(seed=34, num_swarms=3)),
    ]
    announce("split-batch", len(cases))
    params = [q.make_params(engine="fused", **cfg) for _, cfg in cases]
    batch = q.Swarm([fd for fd, _ in cases], params)
    singles = [q.Swarm.create(F, D, engine="fused", **cfg) for (F, D), cfg in cases]
    assert [batch.path(k)[0] for k in range(len(cases))] == ["int8", "split", "split", "split"]
    keys = ("V", "X", "PL", "goal", "goalPL", "PG", "goalPG", "best_perm", "best_goal", "best_info", "t")
    for it in range(4):
        batch.step(1)
        for s in singles:
            s.step(1)
        for k, s in enumerate(singles):
            a, b = batch.get_state(k), s.get_state()
            for key in keys:
                assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), (it, k, key)
    batch.close()
    for s in singles:
        s.close()
