"""qap_swarm_stats_noalloc against qap_swarm_stats, through the C ABI.

The allocation-free variant keeps its scratch in a fixed device array shared
by every call on the GPU; two calls in a row (the second on a smaller request,
so stale contents of the first would show) must give exactly what the
allocating entry point gives.  An armed allocation failure is not consumed by
it, and the library's allocation count does not change."""
import numpy as np
import pytest

import qap_inputs as gen
from _parity import announce, run_cfg

pytestmark = pytest.mark.gpu

KEYS = ("swarm_q", "pop_q", "swarm_hist", "pop_hist")


def _same(a, b, what):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (what, k)


def test_stats_noalloc_equals_stats(q):
    L = q.load_library()
    F, D = gen.uniform_instance(60, 0, 99, 41)
    F2, D2 = gen.uniform_instance(25, 0, 50, 42)
    announce("stats noalloc")
    big = q.Swarm.create(F, D, engine="fused", **run_cfg(num_swarms=40, particles_per_swarm=25, seed=3))
    small = q.Swarm.create(F2, D2, engine="plain", **run_cfg(num_swarms=3, particles_per_swarm=7, seed=4))
    big.step(4)
    small.step(2)
    gbig = big.get_state()["goal"]
    gsmall = small.get_state()["goal"]
    reqs = [
        (big, dict(q_ppm=(10000, 50000, 250000, 500000, 750000, 950000, 1000000), bins=256,
                   lo=int(gbig.min()), hi=int(gbig.max()) + 1)),
        (small, dict(q_ppm=(500000,), bins=4, lo=int(gsmall.min()), hi=int(gsmall.max()) + 1)),
        (big, dict(q_ppm=(1, 999999), bins=0)),
        (small, dict(q_ppm=(), bins=3, lo=int(gsmall.min()) - 5, hi=int(gsmall.min()) + 40)),
    ]
    try:
        for i, (h, kw) in enumerate(reqs):
            ref = h.stats(**kw)
            before = L.qap_swarm_live_allocations()
            assert L.qap_swarm_fail_alloc(1) == 0  # an allocation now would fail
            got = h.stats(noalloc=True, **kw)
            assert L.qap_swarm_fail_alloc(0) == 0
            assert L.qap_swarm_live_allocations() == before
            _same(got, ref, ("request", i))
    finally:
        L.qap_swarm_fail_alloc(0)
    # a request beyond the fixed scratch is refused, the allocating one serves it
    wide = q.Swarm.create(F2, D2, engine="plain", **run_cfg(num_swarms=1100, particles_per_swarm=1, seed=5))
    with pytest.raises(q.QapError) as e:
        wide.stats(q_ppm=(500000,), bins=4096, lo=0, hi=10 ** 8, noalloc=True)
    assert e.value.code == q.QAP_ERR_UNSUPPORTED
    assert wide.stats(q_ppm=(500000,), bins=4096, lo=0, hi=10 ** 8)["pop_hist"].sum() == 1100
    for h in (big, small, wide):
        h.close()
