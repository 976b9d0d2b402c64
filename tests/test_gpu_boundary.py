"""Boundary entry points beyond stepping, through the C ABI.

qap_swarm_deltas: the pair-exchange delta matrix of a particle's S_x output
in the last step (before its exchanges) equals the oracle's for the same
state, the permutation equals the oracle's S_x output, and the step's own
result follows from them (the first minimum pair exchanged if it improves).

Allocation failures: every device allocation of an init, a batch init, an
evaluation, a statistics call and a deltas call is made to fail in turn;
the call returns QAP_ERR_NOMEM, the library holds exactly the allocations it
held before, and a handle that existed stays usable.
"""
import numpy as np
import pytest

import qap_inputs as gen
from _parity import announce, make_gpu, oracle_from_state, run_cfg

pytestmark = pytest.mark.gpu


def _wide_asym(n, seed):
    return gen.general_instance(n, -900, 900, seed)


DELTA_CASES = [
    ("int8-sym", lambda: gen.uniform_instance(40, 0, 127, 3), dict(), "fused"),
    ("int8-gen", lambda: gen.general_instance(33, -50, 127, 4), dict(depth=3), "fused"),
    ("split-D", lambda: gen.uniform_instance(50, 0, 99, 5, d_hi=1000), dict(), "fused"),
    ("int32-asym", lambda: _wide_asym(36, 6), dict(), "fused"),
    ("plain-n70", lambda: gen.uniform_instance(70, 0, 127, 7), dict(depth=1), "plain"),
    ("pick-column", lambda: gen.uniform_instance(30, 0, 127, 8), dict(sx="pick_column"), "fused"),
    ("int8-n150", lambda: gen.uniform_instance(150, 0, 99, 9), dict(), "fused"),
]


@pytest.mark.parametrize("name,mk,extra,engine", DELTA_CASES, ids=[c[0] for c in DELTA_CASES])
def test_deltas_of_the_last_step(q, orc, name, mk, extra, engine):
    F, D = mk()
    n = F.shape[0]
    cfg = run_cfg(num_swarms=2, particles_per_swarm=5, seed=31, **extra)
    ocfg = {k: v for k, v in cfg.items() if k != "sx"}
    announce("deltas", name, engine)
    sw = make_gpu(q, F, D, dict(cfg, engine=engine))
    with pytest.raises(q.QapError) as e:
        sw.deltas(0)  # no step yet
    assert e.value.code == q.QAP_ERR_INVALID_ARG
    sw.step(2)
    st = sw.get_state()
    sw.step(1)
    nx = sw.get_state()
    o = orc.OracleSwarm(F, D, sx=cfg.get("sx", "second_target"), **ocfg)
    o.load_state(dict(st, V=np.asarray(st["V"], np.float64)))
    dl_o = np.zeros((10, n, n), np.int64)
    o.step(deltas_out=dl_o)
    S = cfg["particles_per_swarm"]
    for k in range(10):
        dl, perm = sw.deltas(k)
        g, s = divmod(k, S)
        W = orc.keys(np.asarray(st["V"][k], np.float64), st["X"][k])
        if cfg.get("sx") == "pick_column":
            xs = orc.pick_column(W, seed=cfg["seed"], t=3, particle=s, swarm=g)
        else:
            xs = orc.second_target(W, st["X"][k], cfg["depth"], seed=cfg["seed"], t=3, particle=s, swarm=g)
        assert np.array_equal(perm, xs), (name, k)
        assert np.array_equal(dl, dl_o[k]), (name, k)
        assert np.array_equal(dl, orc.deltas(F, D, perm)), (name, k)
        # the step's own exchange: the first minimum pair, made if it improves
        iu = np.triu_indices(n, 1)
        j = int(np.argmin(dl[iu]))
        a, b, best = int(iu[0][j]), int(iu[1][j]), int(dl[iu][j])
        want = perm.copy()
        if best < 0:
            want[a], want[b] = perm[b], perm[a]
        assert np.array_equal(nx["X"][k], want), (name, k)
        assert int(nx["goal"][k]) == orc.cost(F, D, perm) + min(best, 0), (name, k)
    with pytest.raises(q.QapError) as e:
        sw.deltas(10)
    assert e.value.code == q.QAP_ERR_INVALID_ARG
    sw.set_state(nx)
    with pytest.raises(q.QapError) as e:
        sw.deltas(0)  # the previous-state buffers do not belong to the state just written
    assert e.value.code == q.QAP_ERR_INVALID_ARG
    sw.close()


def _expect_nomem(q, fn):
    try:
        fn()
    except q.QapError as e:
        assert e.code == q.QAP_ERR_NOMEM, e
        return True
    return False


def test_allocation_failures_release_everything(q):
    L = q.load_library()
    F, D = gen.uniform_instance(40, 0, 99, 12)
    Fw, Dw = gen.uniform_instance(30, 0, 99, 13, d_hi=900)
    Fa, Da = _wide_asym(20, 14)
    cfg = run_cfg(num_swarms=3, particles_per_swarm=4, seed=5)
    announce("allocation failures")
    base = L.qap_swarm_live_allocations()
    try:
        # single and batched inits: every allocation in turn
        for what, mk in (("init", lambda: q.Swarm.create(F, D, engine="fused", **cfg)),
                         ("batch", lambda: q.Swarm([(F, D), (Fw, Dw), (Fa, Da)],
                                                   [q.make_params(engine="fused", **cfg)] * 3))):
            failed = 0
            for k in range(1, 400):
                assert L.qap_swarm_fail_alloc(k) == 0
                made = []
                if not _expect_nomem(q, lambda: made.append(mk())):
                    assert L.qap_swarm_fail_alloc(0) == 0
                    made[0].close()
                    break
                failed += 1
                assert L.qap_swarm_live_allocations() == base, (what, k)
            assert failed >= 10, (what, failed)  # device buffers, plans, tables: many allocations
            assert L.qap_swarm_live_allocations() == base
        # per-call allocations of an existing handle: the handle stays usable
        sw = q.Swarm.create(F, D, engine="fused", **cfg)
        held = L.qap_swarm_live_allocations()
        sw.step(2)
        perms = gen.random_perms(3, 40, 1)
        ref_goals, ref_dl = sw.eval(perms, deltas=True)
        ref_stats = sw.stats(bins=8, lo=0, hi=10 ** 6)
        ref_d, _ = sw.deltas(3)
        calls = (("eval", lambda: sw.eval(perms, deltas=True), 3),
                 ("stats", lambda: sw.stats(bins=8, lo=0, hi=10 ** 6), 1),
                 ("deltas", lambda: sw.deltas(3), 3))
        for what, fn, count in calls:
            for k in range(1, count + 1):
                assert L.qap_swarm_fail_alloc(k) == 0
                assert _expect_nomem(q, fn), (what, k)
                assert L.qap_swarm_live_allocations() == held, (what, k)
        assert L.qap_swarm_fail_alloc(0) == 0
        g2, dl2 = sw.eval(perms, deltas=True)
        assert np.array_equal(g2, ref_goals) and np.array_equal(dl2, ref_dl)
        st2 = sw.stats(bins=8, lo=0, hi=10 ** 6)
        assert all(np.array_equal(st2[k], ref_stats[k]) for k in ref_stats)
        assert np.array_equal(sw.deltas(3)[0], ref_d)
        sw.step(1)
        assert sw.get_state()["t"] == 3
        sw.close()
        assert L.qap_swarm_live_allocations() == base
    finally:
        L.qap_swarm_fail_alloc(0)
