"""Batched stepping against the oracle.

A handle over several instances steps every fused-kernel class (padded size,
contraction kind, symmetry, zero diagonals) with one launch.  A class of one
instance passes its descriptor as a kernel argument; a class of several reads
the descriptors and the workgroup map from device tables (the table form).
Here every class holds at least three instances in every stream group, so
each class runs in the table form, for the int8 kernels (symmetric with and
without zero diagonals, general) and both byte-split kernels (one matrix
split, both split); each instance is checked by re-synchronised one-step
parity against the oracle.  Then the 64-instance mixed-size batch (n uniform
in 20..150, 4 swarms x 64 particles each, 16,384 particles) in the launch
configuration the benchmark times: sampled particles of every instance
against the oracle's per-particle step, and the swarm invariants over all
particles.
"""
import numpy as np
import pytest

import qap_inputs as gen
from _parity import (VTOL, announce, assert_states_equal, assert_v_close, oracle_from_state, oracle_particle_step,
                     run_cfg)

pytestmark = pytest.mark.gpu


def _sym_nonzero_diag(n, hi, seed):
    rng = np.random.default_rng(seed)
    F = gen.symmetric_uniform(n, 0, hi, rng, zero_diag=False)
    D = gen.symmetric_uniform(n, 0, hi, rng, zero_diag=False)
    return F, D


def table_classes():
    """(kind, F, D) with three or more instances per fused-kernel class."""
    out = []
    for i, n in enumerate((20, 26, 32)):                  # npad 32, int8 symmetric zero diagonal
        out.append(("i8-sym-zd-32", *gen.uniform_instance(n, 0, 127, 600 + i)))
    for i, n in enumerate((97, 110, 128)):                # npad 128, int8 symmetric zero diagonal
        out.append(("i8-sym-zd-128", *gen.uniform_instance(n, 0, 127, 610 + i)))
    for i, n in enumerate((40, 52, 64)):                  # npad 64, int8 symmetric, non-zero diagonals
        out.append(("i8-sym-64", *_sym_nonzero_diag(n, 60, 620 + i)))
    for i, n in enumerate((35, 47, 60)):                  # npad 64, int8 general (asymmetric, negative)
        out.append(("i8-gen-64", *gen.general_instance(n, -60, 100, 630 + i)))
    for i, n in enumerate((33, 45, 64)):                  # npad 64, byte-split, D split
        out.append(("split-D-64", *gen.uniform_instance(n, 0, 99, 640 + i, d_hi=1000)))
    for i, n in enumerate((70, 81, 96)):                  # npad 96, byte-split, F split
        F, D = gen.uniform_instance(n, 0, 99, 650 + i)
        out.append(("split-F-96", D * 7 + 1 - np.eye(n, dtype=np.int32), F))
    for i, n in enumerate((21, 27, 30)):                  # npad 32, byte-split, both split
        out.append(("split-FD-32", *gen.uniform_instance(n, 0, 600, 660 + i)))
    return out


def test_table_form_classes_one_step_parity(q, orc):
    cases = table_classes()
    cfgs = [run_cfg(num_swarms=3, particles_per_swarm=5, depth=1 + k % 3, seed=700 + k) for k in range(len(cases))]
    announce("batch table classes", len(cases))
    params = [q.make_params(engine="fused", **c) for c in cfgs]
    h = q.Swarm([(F, D) for _, F, D in cases], params)
    want = {"i8": "int8", "split": "split"}
    for k, (kind, F, D) in enumerate(cases):
        assert h.path(k)[0] == want[kind.split("-")[0]], (k, kind)
    assert h.stream_groups() == 3  # three swarms each: every class appears in every group
    h.step(2)
    for it in range(3):
        olds = [h.get_state(k) for k in range(len(cases))]
        h.step(1)
        for k, (kind, F, D) in enumerate(cases):
            o = oracle_from_state(orc, F, D, cfgs[k], olds[k])
            o.step()
            assert_states_equal(h.get_state(k), o.state(), what="%s instance %d iteration %d" % (kind, k, it + 3))
    h.close()


def test_mixed_64_instance_batch_sampled_parity(q, orc):
    insts = gen.mixed_batch(64, 105)
    cfgs = [run_cfg(num_swarms=4, particles_per_swarm=64, seed=1 + k) for k in range(len(insts))]
    announce("mixed batch 64 x (4 x 64)")
    params = [q.make_params(engine="fused", **c) for c in cfgs]
    h = q.Swarm(insts, params)
    assert all(h.path(k)[0] == "int8" for k in range(len(insts)))
    h.step(3)
    assert h.graph_active()
    olds = [h.get_state(k) for k in range(len(insts))]
    h.step(1)
    rng = np.random.default_rng(105)
    for k, (F, D) in enumerate(insts):
        st, nx = olds[k], h.get_state(k)
        n = F.shape[0]
        P = 256
        assert nx["X"].shape == (P, n) and nx["t"] == 4
        assert (np.sort(nx["X"], axis=1) == np.arange(n)).all(), k
        assert (nx["goalPL"] <= st["goalPL"]).all(), k
        assert (nx["goalPG"] == nx["goalPL"].reshape(4, 64).min(axis=1)).all(), k
        for p in (0, 63, 64, P - 1, int(rng.integers(0, P))):
            Vn, x, goal, pl, gpl = oracle_particle_step(orc, F, D, cfgs[k], st, p)
            assert np.array_equal(nx["X"][p], x), (k, n, p)
            assert int(nx["goal"][p]) == goal, (k, n, p)
            assert np.array_equal(nx["PL"][p], pl) and int(nx["goalPL"][p]) == gpl, (k, n, p)
            assert_v_close(nx["V"][p][None], Vn[None], VTOL)
        for g in range(4):
            assert orc.cost(F, D, nx["PG"][g]) == int(nx["goalPG"][g]), (k, g)
        assert orc.cost(F, D, nx["best_perm"]) == int(nx["best_goal"]) == int(nx["goalPG"].min()), k
    h.close()
