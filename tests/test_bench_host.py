"""Host-side logic of bench.py, no GPU: the algorithmic byte counts the
roofline uses, the per-iteration span read from a kernel trace, the traffic
summary's source-hash check, and the single-GPU guard.

bench is imported inside the tests: importing it raises GPU_MAX_HW_QUEUES for
the process, which must not leak into the GPU tests' collection."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    return bench


def test_algorithmic_bytes():
    b = _bench()
    # V(t) read and V(t+1) written (8 n^2), X read and written and P^L read (3 n), two goals (24)
    assert b.algorithmic_bytes("fused", 128) == 8 * 128 * 128 + 3 * 128 + 24 == 131480
    assert b.workload_bytes(b.workload_setup("n128x10k")) == 10000 * 131480
    mixed = b.workload_setup("mixed64")
    assert len(mixed) == 64
    assert b.workload_bytes(mixed) == sum(256 * (8 * F.shape[0] ** 2 + 3 * F.shape[0] + 24) for F, _, _ in mixed)


def _write_trace(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for r in rows:
            w.writerow(r)


def test_trace_span_takes_the_last_iterations(tmp_path):
    """Two chains, 3 warm-up iterations then 2 timed ones: the span runs from
    the first dispatch after the last finish of the warm-up to the last end."""
    b = _bench()
    us = 1000  # timestamps in ns
    rows, t = [], 0
    for it in range(5):
        for chain in range(2):
            s = t + 10 * us * chain
            rows.append(("void qap::k_fused_step<128, true, true, false, 4>(qap::InstDesc)", s, s + 100 * us))
            rows.append(("qap::k_swarm_best(qap::InstDesc const*)", s + 100 * us, s + 110 * us))
            rows.append(("qap::k_finish(qap::InstDesc const*, int)", s + 110 * us, s + 120 * us))
        t += 1000 * us
    path = tmp_path / "t_kernel_trace.csv"
    _write_trace(path, rows)

    class A:
        steps, groups, workload = 2, 2, "n128x10k"

    r = b.trace_span(str(path), A)
    # the timed iterations start at 3000 us and end at 4000 + 10 + 120 us
    assert r["span_ms_per_iteration"] == pytest.approx((4130 - 3000) / 1e3 / 2)
    assert r["fused_dispatches"] == 4
    assert r["dispatches_in_timed_region"] == 12


def test_measured_traffic_needs_the_current_sources(tmp_path, monkeypatch):
    b = _bench()
    f = tmp_path / "fused_w_traffic.md"
    monkeypatch.setattr(b, "traffic_file", lambda w: str(f))
    f.write_text("source hash: `%s`\n\nscaled HBM bytes per step: 1.2345e+09\n" % b.kernel_hash())
    assert b.measured_traffic("w") == pytest.approx(1.2345e9)
    f.write_text("source hash: `0000000000000000`\n\nscaled HBM bytes per step: 1.2345e+09\n")
    assert b.measured_traffic("w") is None
    monkeypatch.setattr(b, "traffic_file", lambda w: str(tmp_path / "absent.md"))
    assert b.measured_traffic("w") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
