#!/usr/bin/env python
"""Throughput of the multi-swarm PSO hot path for the QAP on one MI355X.

Workload (the headline configuration): n = 128, F and D symmetric integers
uniform in [0, 127] with zero diagonal (seeded, synthetic -- stands in for the
paper's QAPLIB instances), 200 swarms x 50 particles = 10,000 particles,
S_v = Norm, c1 = 0.8, c2 = c3 = 0.5, vmax = 1, SecondTarget depth 2, one
pair-exchange improvement per particle-iteration, independent swarms.

A step is one iteration of every particle (S_x, velocity, goal, pair-exchange
deltas and exchange, P^L, swarm bests).  Inputs are resident in HBM before
the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

# Concurrent stream chains overlap only on hardware queues of their own: HIP
# gives a process 4 by default, shared by every stream it creates (the default
# stream and the caller's included), and kernels of two streams on one queue
# run one after the other.  Ask for at least 8 (set before HIP starts).
HW_QUEUES = 8
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < HW_QUEUES:
    os.environ["GPU_MAX_HW_QUEUES"] = str(HW_QUEUES)

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
VALU_INT_PEAK_TOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 ops per multiply-add

WORKLOAD = dict(name="n128x10k", n=128, seed_inst=104, num_swarms=200, particles_per_swarm=50)
RUN = dict(c1=0.8, c2=0.5, c3=0.5, vmax=1.0, norm=True, depth=2, local_search=True, migration=False, seed=1)


def algorithmic_bytes(stage: str, n: int) -> int:
    """HBM bytes per particle-iteration the stage cannot avoid."""
    if stage == "fused":      # V(t) read + V(t+1) write, X read+write, P^L read, goal + P^L goal
        return 8 * n * n + 3 * n + 24
    if stage == "sx":         # V(t) read, X(t) read, X' write
        return 4 * n * n + 2 * n
    if stage == "velocity":   # V(t) read + V(t+1) write, X, P^L, P^G reads
        return 8 * n * n + 3 * n
    if stage == "goal_delta":  # X' read, X write, P^L read, goal, P^L goal
        return 3 * n + 24
    return 0


def traffic_file(workload: str) -> str:
    """The committed HBM-traffic summary of the fused kernel on a workload."""
    return os.path.join(ROOT, "profiles", "fused_%s_traffic.md" % workload)
KERNEL_SOURCES = ["common.hpp", "philox.hpp", "dword.hpp", "second_target.hpp", "kernels.hpp", "kernels_fused.hip"]


def kernel_hash() -> str:
    """Hash of the device sources the fused step kernel is built from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1504_05158_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per step of the fused kernel (all its launches of one
    iteration) from the committed counter summary of the workload (FETCH_SIZE +
    WRITE_SIZE, each scaled by the same counter on a copy of known size), or
    None if absent or taken on other kernel sources."""
    try:
        text = open(traffic_file(workload)).read()
    except OSError:
        return None
    m = re.search(r"source hash:\s*`?([0-9a-f]+)", text)
    t = re.search(r"scaled HBM bytes per step:\s*([0-9.e+]+)", text)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def traffic_calibration(size_mib: int = 1024, reps: int = 3) -> None:
    """A plain device copy of known size (size_mib read + written per
    launch) for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = size_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": size_mib * (1 << 20), "launches": reps}))


def contraction_ops(n: int, sym: bool) -> int:
    """Integer operations of the pair-exchange contraction per particle (2 per multiply-add)."""
    return 2 * n ** 3 * (1 if sym else 2)


MIXED = dict(name="mixed64", count=64, seed=105, num_swarms=4, particles_per_swarm=64)
WORKLOAD_NAMES = ["n128x10k", "n12", "n50", "n100mig", "n128", "n128wide", "mixed64"]


def workload_setup(name: str):
    """Instances and run parameters of a named workload: a list of
    (F, D, params) -- the headline one (n128x10k), another of
    qap_inputs.WORKLOADS, or the 64-instance mixed-size batch (mixed64: n
    uniform in 20..150, F and D U{0..99} symmetric, 4 swarms x 64 particles
    each, one seed per instance)."""
    import qap_inputs as gen
    if name == MIXED["name"]:
        out = []
        for k, (F, D) in enumerate(gen.mixed_batch(MIXED["count"], MIXED["seed"])):
            out.append((F, D, dict(RUN, num_swarms=MIXED["num_swarms"],
                                   particles_per_swarm=MIXED["particles_per_swarm"], seed=1 + k)))
        return out
    w = gen.WORKLOADS[name]
    F, D = w["gen"]()
    run = dict(RUN, migration=w["migration"], migration_factor=w.get("migration_factor", 0.0),
               migration_period=w.get("migration_period", 1), num_swarms=w["num_swarms"],
               particles_per_swarm=w["particles_per_swarm"])
    if name == "n50":
        run["delta_path"] = "int32"  # that workload is defined on the plain int32 cost and delta path
    return [(F, D, run)]


def workload_bytes(insts, stage: str = "fused") -> int:
    """Algorithmic HBM bytes of one step of the workload."""
    return sum(algorithmic_bytes(stage, F.shape[0]) * p["num_swarms"] * p["particles_per_swarm"]
               for F, D, p in insts)


def run_gpu(args, engine: str):
    import numpy as np
    import torch
    import paper_1504_05158_amd as q

    insts = workload_setup(args.workload)
    if args.local_search is not None:
        insts = [(A, B, dict(p, local_search=args.local_search)) for A, B, p in insts]
    F, D = insts[0][0], insts[0][1]
    n = F.shape[0]
    stream = torch.cuda.Stream()
    P = sum(p["num_swarms"] * p["particles_per_swarm"] for _, _, p in insts)

    plan = None

    def make():
        nonlocal plan
        prms = [q.make_params(stream=stream.cuda_stream, engine=engine, **p) for _, _, p in insts]
        h = q.Swarm([(A, B) for A, B, _ in insts], prms)
        if args.plan:
            c, s_, i = (int(x) for x in args.plan.split(","))
            h.set_plan(c, s_, i)
            plan = h.plan()
        elif not args.no_tune:
            # the launch plan is chosen on the handle's own work and the handle
            # returned to iteration 0: set-up, before the timed region
            if plan is None:
                plan = h.tune(32)
            else:
                h.set_plan(plan["stream_chains"], plan["split"], plan["iters_per_graph"])
        else:
            plan = h.plan()
        return h

    sw = make()
    paths = sorted(set(sw.path(k)[0] for k in range(len(insts))))
    path = paths[0] if len(paths) == 1 else "+".join(paths)
    sym = all(sw.path(k)[1] for k in range(len(insts)))
    groups = sw.stream_groups()
    sw.step(args.warmup)
    sw.sync()
    torch.cuda.synchronize()
    # HIP events on the handle's stream bracket the timed region: the library's
    # stream groups fork from it and join back within every step call
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    sw.step(args.steps)
    ev1.record(stream)
    sw.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sw.close()
    secs = t1 - t0
    region_ms = ev0.elapsed_time(ev1) / args.steps
    value = P * args.steps / secs
    # per-kernel durations from HIP events on the streams the kernels run on: a
    # second run from the same seed replays exactly the timed iterations (events
    # stay out of the timed run, where they would add a few percent)
    if args.no_profile_pass:
        # the fused engine's iteration is its fused kernel (and the small bests
        # kernels); the per-stage engine's is reported as a whole
        key = "fused" if engine == "fused" else "iteration"
        stage_ms, iters = {key: region_ms * args.steps * groups}, args.steps
    else:
        sw = make()
        sw.step(args.warmup)
        sw.profile(True)
        sw.step(args.steps)
        stage_ms, iters = sw.profile(False)
        sw.close()
    dom = max(stage_ms, key=stage_ms.get)
    launches = groups if dom == "fused" else 1
    avg_ms = stage_ms[dom] / max(iters, 1) / launches
    if dom == "goal_delta" and path == "int32":
        achieved = sum(contraction_ops(A.shape[0], sym) * p["num_swarms"] * p["particles_per_swarm"]
                       for A, _, p in insts) / (avg_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 3), peak=VALU_INT_PEAK_TOPS, unit="TOP/s",
                    frac=round(achieved / VALU_INT_PEAK_TOPS, 4), traffic=None)
    else:
        bps = workload_bytes(insts, "fused" if dom == "iteration" else dom)  # per step, over the `launches` launches
        if launches > 1:
            # concurrent launches overlap: the aggregate rate is the step's bytes over the
            # event-timed region per step (which also holds the small bests kernels)
            achieved = bps / (region_ms * 1e-3) / 1e9
        else:
            achieved = bps / (avg_ms * 1e-3) / 1e9
        traffic = (measured_traffic(args.workload)
                   if (dom == "fused" and engine == "fused" and args.local_search is None) else None)
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=None if traffic is None else round(traffic / 1e9, 4))
        roof["algorithmic_gb_per_step"] = round(bps / 1e9, 4)
        roof["traffic_unit"] = "GB per step"
        roof["launches_per_step"] = launches
        roof["region_ms_per_step"] = round(region_ms, 4)
        roof["achieved_per_launch"] = round(bps / launches / (avg_ms * 1e-3) / 1e9, 1)
    roof["kernel"] = dom
    roof["avg_ms"] = round(avg_ms, 4)  # per launch
    return dict(value=value, ms=secs * 1e3 / args.steps, path=path, sym=sym, P=P, n=n, roofline=roof,
                stage_ms={k: round(v / max(iters, 1) / groups, 4) for k, v in stage_ms.items()},
                groups=groups, instances=len(insts), plan=plan)


ORACLE_KEYS = ("c1", "c2", "c3", "vmax", "norm", "depth", "local_search", "migration", "migration_factor",
               "migration_period", "seed")


def cpu_baseline(workload: str, target_s: float = 15.0, max_steps: int = 2000, threads: int = 16,
                 swarms: int | None = None, per: int | None = None):
    """The oracle, as it stands, stepping the workload (or a sample of it: at
    most `swarms` swarms of each instance, `per` particles each -- the same
    instances and per-particle work) until about target_s seconds have passed,
    on `threads` OpenMP threads (at most the host's cores)."""
    import oracle as orc

    insts = workload_setup(workload)
    orc.set_threads(max(1, min(threads, os.cpu_count() or 1)))
    used = orc.get_threads()
    sws = []
    for F, D, p in insts:
        S = p["num_swarms"] if swarms is None else min(swarms, p["num_swarms"])
        Sp = p["particles_per_swarm"] if per is None else min(per, p["particles_per_swarm"])
        sws.append(orc.OracleSwarm(F, D, num_swarms=S, particles_per_swarm=Sp,
                                   **{k: p[k] for k in ORACLE_KEYS if k in p}))
    parts = sum(sw.P for sw in sws)
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps:
        for sw in sws:
            sw.step(1)
        steps += 1
        if time.perf_counter() - t0 >= target_s:
            break
    secs = time.perf_counter() - t0
    total = sum(p["num_swarms"] * p["particles_per_swarm"] for _, _, p in insts)
    if len(insts) == 1:
        F, _, p = insts[0]
        what = ("the whole workload" if parts == total else "the first %d of its %d swarms" % (sws[0].m, p["num_swarms"]))
        what += " (%d swarms x %d particles, n=%d)" % (sws[0].m, sws[0].S, F.shape[0])
    else:
        what = ("the whole workload" if parts == total else "every instance with %d swarm(s) x %d particles"
                % (sws[0].m, sws[0].S)) + " (%d instances, %d particles)" % (len(insts), parts)
    return dict(value=round(parts * steps / secs, 2), unit="particle-iterations/s", cores=used,
                kind="oracle",
                sample="%s, iterations 1-%d, %d OpenMP thread%s, %.1f s"
                       % (what, steps, used, "" if used == 1 else "s", secs))


def trace_span(path: str, args) -> dict:
    """Per-iteration span of the timed region in a rocprofv3 kernel trace
    (csv) of `bench.py --no-compare --no-cpu-baseline --no-profile-pass`,
    whose timed iterations are the last work it launches: the k_finish
    dispatches (one per stream chain per iteration) of the timed iterations
    are the last steps x chains of them by end time; the region is every
    dispatch that starts after the k_finish before those, from the first
    start to the last end, divided by the timed iterations."""
    import csv
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            rows.append((r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    fin = sorted(e for name, b, e in rows if "k_finish" in name)
    groups = args.groups
    cut = fin[-args.steps * groups - 1]  # end of the last iteration before the timed ones
    timed = [(name, b, e) for name, b, e in rows if b > cut]
    span_ns = max(e for _, _, e in timed) - min(b for _, b, _ in timed)
    per_iter_ms = span_ns / 1e6 / args.steps
    byts = workload_bytes(workload_setup(args.workload))
    fused = [e - b for name, b, e in timed if "k_fused" in name]
    return {"trace": os.path.basename(path), "workload": args.workload, "timed_iterations": args.steps,
            "finish_dispatches_per_iteration": groups, "dispatches_in_timed_region": len(timed),
            "k_finish_total": len(fin), "span_ms_per_iteration": round(per_iter_ms, 5),
            "fused_dispatches": len(fused), "fused_mean_ms": round(sum(fused) / max(len(fused), 1) / 1e6, 5),
            "algorithmic_gb_per_step": round(byts / 1e9, 4),
            "achieved_gbs": round(byts / (per_iter_ms * 1e-3) / 1e9, 1),
            "frac": round(byts / (per_iter_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--engine", default="fused", choices=["fused", "plain"])
    ap.add_argument("--workload", default=WORKLOAD["name"], choices=WORKLOAD_NAMES,
                    help="n128x10k (the headline, default), a workload of qap_inputs.WORKLOADS, or mixed64 "
                         "(64 instances, n 20..150); the CPU baseline runs with the headline only")
    ap.add_argument("--no-compare", action="store_true", help="skip timing the per-stage (plain int32) engine")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch plan instead of the tuned one")
    ap.add_argument("--plan", metavar="C,S,I", default=None,
                    help="launch plan to use instead of tuning: stream chains, split (0 swarms, 1 instances, "
                         "2 kernel classes), iterations per graph (0 = eager)")
    ap.add_argument("--local-search", type=int, default=None,
                    help="pair exchanges per particle-iteration instead of the workload's (1)")
    ap.add_argument("--no-profile-pass", action="store_true",
                    help="skip the second, event-timed run (for kernel traces of the timed region alone)")
    ap.add_argument("--traffic-calibration", action="store_true",
                    help="run only a 1 GiB device copy (for scaling HBM byte counters)")
    ap.add_argument("--trace-span", metavar="CSV",
                    help="no GPU run: the per-iteration span of the timed region in a rocprofv3 kernel trace")
    ap.add_argument("--groups", type=int, default=3,
                    help="with --trace-span: stream chains of the traced run (its JSON line's stream_groups)")
    args = ap.parse_args()
    if args.trace_span:
        print(json.dumps(trace_span(args.trace_span, args)))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs the hot path on a single MI355X "
              "(the swarms would shard by swarm across GPUs, which is not built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.traffic_calibration:
        traffic_calibration()
        return
    res = run_gpu(args, args.engine)
    other = None
    if not args.no_compare:
        oth = "plain" if args.engine == "fused" else "fused"
        try:
            other = run_gpu(args, oth)
        except Exception as e:  # the other engine may be unavailable for this build
            other = dict(error=str(e))
    headline = args.workload == WORKLOAD["name"]
    line = {
        "metric": ("particle-iterations/sec at n=128, 10k particles (batched int8 vs plain path)" if headline
                   else "particle-iterations/sec, workload %s" % args.workload),
        "value": round(res["value"], 1),
        "unit": "particle-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"int8": "f32+i8", "split": "f32+i8 byte-split"}.get(res["path"], "f32+i32"),
        "data": "synthetic",
        "config": {"workload": ("n128x10k: n=128 QAP, F and D symmetric U{0..127}, 200 swarms x 50 particles, "
                                "Norm, c=(0.8,0.5,0.5), depth 2, one pair exchange") if headline else args.workload,
                   "n": res["n"], "particles": res["P"], "engine": args.engine, "delta_path": res["path"],
                   "parallelism": "single GPU"},
        "roofline": res["roofline"],
        "stage_ms": res["stage_ms"],
        "stream_groups": res["groups"],
        "plan": res["plan"],
        "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"]),
    }
    if res["instances"] > 1:
        line["config"]["instances"] = res["instances"]
    if args.local_search is not None:
        line["config"]["local_search"] = args.local_search
    if other is not None:
        line["compare"] = {("plain" if args.engine == "fused" else "fused"):
                           (round(other["value"], 1) if "value" in other else other)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload)
        # one core on a sample whose iteration takes about a second or two: the
        # headline's first 8 swarms (400 particles), one swarm of the other
        # single-instance workloads, 8 particles of every instance of the batch
        sample = (dict(swarms=8) if headline else dict(swarms=1, per=8) if args.workload == MIXED["name"]
                  else dict(swarms=1))
        line["cpu_baseline"]["one_core"] = cpu_baseline(args.workload, target_s=10.0, threads=1, **sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
