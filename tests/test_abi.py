"""C-ABI library checks that need no GPU: it loads, exports every entry point
the header declares, and rejects invalid requests before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qap_swarm.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int64_t|int|void|const char\*)\s+(qap_swarm_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def L():
    import paper_1504_05158_amd as q
    return q.load_library()


def test_header_declares_the_boundary():
    names = declared()
    for must in ["qap_swarm_init", "qap_swarm_step", "qap_swarm_best", "qap_swarm_destroy", "qap_swarm_strerror"]:
        assert must in names


def test_library_exports_every_declared_symbol(L):
    import paper_1504_05158_amd as q
    for name in declared():
        assert hasattr(L, name), name
        assert name in q.EXPORTS
    assert sorted(q.EXPORTS) == declared()


def test_binding_constants_match_the_header():
    import paper_1504_05158_amd as q
    src = open(HEADER).read()
    for name in ("QAP_MAX_CHAINS", "QAP_SPLIT_SWARMS", "QAP_SPLIT_INSTANCES", "QAP_SPLIT_CLASSES",
                 "QAP_PATH_SPLIT_MFMA", "QAP_ENGINE_PLAIN"):
        m = re.search(r"\b%s\s*=\s*(\d+)" % name, src)
        assert m and int(m.group(1)) == getattr(q, name), name


def test_strerror_and_null_safety(L):
    assert L.qap_swarm_strerror(0) == b"ok"
    assert b"range" in L.qap_swarm_strerror(-2)
    L.qap_swarm_destroy(None)  # NULL is a no-op


def _init(L, F, D, **kw):
    import paper_1504_05158_amd as q
    F = np.ascontiguousarray(F, np.int32)
    D = np.ascontiguousarray(D, np.int32)
    inst = q.qap_instance(F.shape[0], F.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          D.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    base = dict(num_swarms=2, particles_per_swarm=4)
    base.update(kw)
    prm = q.make_params(**base)
    h = ctypes.c_void_p()
    rc = L.qap_swarm_init(ctypes.byref(inst), ctypes.byref(prm), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("kw", [
    dict(num_swarms=0), dict(particles_per_swarm=0), dict(c1=1.5), dict(c2=-0.1), dict(c3=float("nan")),
    dict(vmax=0.0), dict(depth=-1), dict(depth=5), dict(migration=True, migration_factor=0.5, num_swarms=4),
    dict(migration=True, migration_factor=0.25, num_swarms=4, migration_period=0), dict(delta_path=7),
    dict(engine=9),
])
def test_invalid_params_rejected_on_host(L, kw):
    F = np.ones((5, 5), np.int32)
    rc, h = _init(L, F, F, **kw)
    assert rc == -1 and not h.value


def test_invalid_sizes_rejected(L):
    rc, h = _init(L, np.ones((1, 1)), np.ones((1, 1)))
    assert rc == -1 and not h.value
    big = np.ones((257, 257))
    rc, h = _init(L, big, big)
    assert rc == -1


def test_range_errors_on_host(L):
    F = np.full((8, 8), 200, np.int32)
    D = np.full((8, 8), 3, np.int32)
    rc, h = _init(L, F, D, delta_path="int8")
    assert rc == -2 and not h.value
    # no exact int32 contraction: n * max|F| * max|D| >= 2^31
    F = np.full((8, 8), 1 << 14, np.int32)
    D = np.full((8, 8), 1 << 14, np.int32)
    rc, h = _init(L, F, D, delta_path="int32")
    assert rc == -2 and not h.value


def test_header_enums_match_the_binding():
    import paper_1504_05158_amd as q
    src = open(HEADER).read()
    vals = dict((k, int(v)) for k, v in re.findall(r"\b(QAP_(?:PATH|SX|ENGINE|SV|ERR)_\w+)\s*=\s*(-?\d+)", src))
    for name in ("QAP_PATH_AUTO", "QAP_PATH_INT8_MFMA", "QAP_PATH_INT32", "QAP_PATH_SPLIT_MFMA", "QAP_ERR_RANGE"):
        assert name in vals, name
    for name, v in vals.items():
        if hasattr(q, name):
            assert getattr(q, name) == v, name


def test_split_path_range_errors_on_host(L):
    import paper_1504_05158_amd as q
    # asymmetric data outside int8: no byte-split path
    F = np.arange(64, dtype=np.int32).reshape(8, 8) * 5
    D = np.full((8, 8), 3, np.int32)
    rc, h = _init(L, F, D, delta_path="split")
    assert rc == q.QAP_ERR_RANGE and not h.value
    # symmetric, but an entry beyond 15 bits
    F = np.full((8, 8), 16384, np.int32)
    rc, h = _init(L, F, D, delta_path="split")
    assert rc == q.QAP_ERR_RANGE and not h.value
    # symmetric and 15-bit, but 8 (n + 3) max|F| max|D| >= 2^31
    F = np.full((8, 8), 16383, np.int32)
    D = np.full((8, 8), 1500, np.int32)
    rc, h = _init(L, F, D, delta_path="split")
    assert rc == q.QAP_ERR_RANGE and not h.value
    # an unknown path value
    rc, h = _init(L, F, F, delta_path=4)
    assert rc == q.QAP_ERR_INVALID_ARG and not h.value
