#!/usr/bin/env python3
"""Benchmark of the exact divergence estimator on one MI355X.

Workload (one "step"): one batched call that certifies the canonical optimum
of every window of a batch of synthetic ventral-descent windows on a 346x260
sensor (100k events per 0.25 s window, 2000 textured surface points, 20%
uniform noise, 0.5 px jitter, true D ~ U(0.05, 0.8)), searching D in
[0, 1.5] with eps = 1e-5 (grid depth 18).  The step runs the whole hot path:
event binning, point and interval evaluations, and the device frontier.
Inputs are resident in HBM before the timed region starts.

Printed: one JSON line with event-hypothesis evaluations per second (value),
certified windows per second (batched; batched and seeded by the learned
proposal when its weights are present; plain one-window calls), the roofline
of the hypothesis-evaluation kernel and the CPU oracle timed on a bounded
sample of the same windows on this host.
"""

from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "event-hypothesis evals/sec; BnB windows/sec (plain vs batched+learned) at fixed eps"
WORKLOADS = {
    "c2": "{B} windows of the 346x260 config per step: 100k events/0.25 s window, D in [0,1.5], eps 1e-5 (L=18), "
          "batched certified BnB",
    "c3": "{B} windows of the 640x480 config per step: 50k-1M events (log-uniform) per 0.25 s window, D drifting "
          "0.1 to 0.6, D in [0,1.5], eps 1e-5 (L=18), batched certified BnB",
    "c5": "{B} windows of the 1280x720 config per step: 100k-5M events (log-uniform) per 0.25 s window plus hot "
          "pixels, D in [0,2], eps 1e-5 (L=18), batched certified BnB",
}

# Algorithmic VALU lane-operations of the fp32 statement per unit of work:
OPS_POINT = 8      # per event and point hypothesis: 2 fma, 2 floor, 2 range tests, 1 index, 1 accumulate
OPS_INTERVAL = 16  # per event and interval: 2 endpoint warps (4 fma, 4 floor), 4 range tests, 4 walk set-up
OPS_PIXEL = 12     # per upper-bound pixel increment: corner test (7 fp64), 1 step, 2 range tests, 1 index, 1 acc
# Peak lane-operation rate: 256 CUs x 64 lanes per clock (4 SIMDs x 16) x 2.4 GHz.
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# The library's default frontier batch (nodes expanded together per window and step).
DEFAULT_F = 96
# Bytes of one prepared event record read by the evaluation kernel (x, y, ax, ay as fp32).
EVENT_RECORD_BYTES = 16

# HBM traffic of the evaluation kernel per launch, from two rocprofv3 --pmc
# passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean over the
# dispatches) of `bench.py --steps 2 --warmup 1 --plain-windows 0
# --no-cpu-baseline --no-plan --no-autotune` on the default workload, each scaled by bytes/KiB that
# the same counter reads for a plain copy of 1 GiB (`bench.py
# --calibrate-copy`).  The figures hold only for the kernel sources and the
# workload they were taken on; for anything else `traffic` is null.
TRAFFIC = {
    "sources_sha256": "8e1785769dc120bbf3b11ffb6ffeb316920b40a8dd1689b3bd98a6fc171f5aa7",
    "workload": {"config": "c2", "windows": 32, "frontier_batch": 96},
    "fetch_kib": 24453.7,
    "write_kib": 1039.7,
    "fetch_bytes_per_kib": 1073741824 / 524304.9,
    "write_bytes_per_kib": 1073741824 / 1048576.0,
}
KERNEL_SOURCES = ("paper_2209_13168_amd/csrc/ecmd_kernels.hip", "paper_2209_13168_amd/csrc/ecmd_internal.hpp",
                  "paper_2209_13168_amd/csrc/ecmd_api.hip")


def sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_per_launch(workload: dict):
    """HBM bytes per evaluation launch from the recorded counters, or None."""
    if TRAFFIC["sources_sha256"] != sources_sha256() or TRAFFIC["workload"] != workload:
        return None
    return round(TRAFFIC["fetch_kib"] * TRAFFIC["fetch_bytes_per_kib"]
                 + TRAFFIC["write_kib"] * TRAFFIC["write_bytes_per_kib"])


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 20; 3 for c3 and c5)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up steps (default 3; 1 for c3 and c5)")
    ap.add_argument("--config", choices=["c2", "c3", "c5"], default="c2",
                    help="c2: 32 windows of 346x260 (the default workload); c3: the 64-window 640x480 batch; "
                         "c5: the 256-window 1280x720 batch with hot pixels")
    ap.add_argument("--windows", type=int, default=32, help="windows per step (c2)")
    ap.add_argument("--frontier-batch", type=int, default=0)
    ap.add_argument("--plain-windows", type=int, default=None,
                    help="windows timed one call each (default 8 for c2, all windows of the batch for c3 and c5)")
    ap.add_argument("--cpu-windows", type=int, default=8, help="oracle sample size (windows)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2209_13168_amd", "weights", "cnn_c2.npz"),
                    help="trained proposal network (the step seeds the search with it when present)")
    ap.add_argument("--plain", action="store_true", help="time the search without the learned seeds")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuned leg")
    ap.add_argument("--no-plan", action="store_true",
                    help="skip the asynchronous plan legs (their finished steps launch empty kernels, which a "
                         "kernel trace would average in)")
    ap.add_argument("--print-sources-sha", action="store_true", help="print the kernel sources hash and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB buffer three times (to scale HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.print_sources_sha:
        print(sources_sha256())
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the estimator has no multi-GPU path in this build "
              "(windows would shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2209_13168_amd import ecmd
    from synth import config_windows, pack_batch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel() * 4, "launches": 3}))
        return
    big = args.config != "c2"
    if args.steps is None:
        args.steps = 3 if big else 20
    if args.warmup is None:
        args.warmup = 1 if big else 3
    if args.plain_windows is None:
        args.plain_windows = 10**9 if big else 8
    if big:
        from paper_2209_13168_amd.learned import windows_chunks
        from synth.ventral import config_specs

        B = {"c3": 64, "c5": 256}[args.config]
        parts = list(windows_chunks(list(range(B)), cfg=args.config, chunk=32))
        x, y, t = (np.concatenate([p[k] for p in parts]) for k in range(3))
        tau = np.concatenate([p[4] for p in parts])
        off = np.zeros(B + 1, np.int64)
        off[1:] = np.cumsum(np.concatenate([np.diff(p[3]) for p in parts]))
        s = config_specs(args.config, 0)
        win = lambda k: config_windows(args.config, [k])[0]  # noqa: E731
    else:
        B = args.windows
        wins = config_windows("c2", range(B))
        s = wins[0].spec
        x, y, t, off, tau = pack_batch(wins)
        win = lambda k: wins[k]  # noqa: E731
    dx, dy, dt, doff, dtau = (torch.from_numpy(a).to(dev) for a in (x, y, t, off, tau))
    sensor = ecmd.sensor(s.width, s.height, s.foe)
    ctx = ecmd.Context(0)
    kw = dict(frontier_batch=args.frontier_batch)
    net = None
    if not args.plain and os.path.exists(args.weights):
        from paper_2209_13168_amd import learned

        net, net_meta = learned.load(ctx, args.weights)

    def step_plain():
        return ctx.estimate_batched(sensor, dx, dy, dt, doff, dtau, s.d_lo, s.d_hi, s.eps, **kw)

    def step_learned():
        return ctx.estimate_learned(net, sensor, dx, dy, dt, doff, dtau, s.d_lo, s.d_hi, s.eps, **kw)

    step = step_plain

    ref = None
    for _ in range(args.warmup):
        ref = step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    ctx.profile(reset=True)
    # no Python garbage-collection pass inside the timed region (a full pass
    # over torch's objects takes tens of milliseconds of host time)
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    res = []
    for _ in range(args.steps):
        res.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    prof = ctx.profile(reset=True)
    ctx.set_profiling(False)
    sec = (t1 - t0) / args.steps
    for r in res:  # deterministic results on every step
        assert [(a.j_star, a.K) for a in r] == [(a.j_star, a.K) for a in (ref or res[0])]
    last = res[-1]
    assert all(r.status == 0 for r in last), [r.status for r in last]
    ev_hyp = sum(r.event_hyp_evals for r in last)
    n_w = np.array([r.n_events for r in last], np.int64)
    pt_ev = sum(r.point_evals * r.n_events for r in last)
    bd_ev = sum(r.bound_evals * r.n_events for r in last)
    pix = sum(r.pixel_updates for r in last)
    value = ev_hyp / sec

    # batched and seeded by the learned proposal (same timing method, fewer steps)
    learned_ws = nodes_learned = None
    if net is not None:
        step_learned()
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        reps = max(3, args.steps // 4)
        for _ in range(reps):
            rl = step_learned()
        torch.cuda.synchronize()
        learned_ws = B * reps / (time.perf_counter() - a0)
        assert [(r.j_star, r.K) for r in rl] == [(r.j_star, r.K) for r in last]
        nodes_learned = float(np.mean([r.nodes_expanded for r in rl]))

    # batched + learned with the launch tuning the autotuner picks for this
    # batch (346x260 only: on the large batches one tuning pass takes minutes)
    tuned_ws = tuned = None
    if net is not None and not big and not args.no_autotune:
        tuned = ctx.autotune(sensor, dx, dy, dt, doff, dtau, s.d_lo, s.d_hi, s.eps)
        step_learned()
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        reps = max(3, args.steps // 4)
        for _ in range(reps):
            rt = step_learned()
        torch.cuda.synchronize()
        tuned_ws = B * reps / (time.perf_counter() - a0)
        assert [(r.j_star, r.K) for r in rt] == [(r.j_star, r.K) for r in last]
        ctx.set_tuning()  # back to the default rule for the legs below

    # the same batch handed over in host memory (the library stages it to
    # the device: PCIe-inclusive rate)
    ctx.estimate_batched(sensor, x, y, t, off, tau, s.d_lo, s.d_hi, s.eps, **kw)
    torch.cuda.synchronize()
    a0 = time.perf_counter()
    reps = max(3, args.steps // 4)
    for _ in range(reps):
        rh = ctx.estimate_batched(sensor, x, y, t, off, tau, s.d_lo, s.d_hi, s.eps, **kw)
    torch.cuda.synchronize()
    host_ws = B * reps / (time.perf_counter() - a0)
    assert [(r.j_star, r.K) for r in rh] == [(r.j_star, r.K) for r in last]

    # the asynchronous plan, captured once into a graph and replayed: no host
    # synchronisation inside the search.  Steps: the default 256, and the
    # multiple of four that this batch needs (a caller who knows its workload)
    gstream = torch.cuda.Stream()
    gctx = ecmd.Context(0, stream=gstream.cuda_stream)
    need = int(max(r.steps for r in last)) + 1
    plan_ws = {}
    legs = () if args.no_plan else (("plan_graph_256_steps", 0), (f"plan_graph_{-(-need // 4) * 4}_steps", need))
    for label, msteps in legs:
        plan = gctx.batch_plan(sensor, s.d_lo, s.d_hi, s.eps, max_windows=B, max_events=int(off[-1]),
                               max_steps=msteps, **kw)
        obuf = plan.result_buffer(B)
        torch.cuda.synchronize()
        with torch.cuda.stream(gstream):
            plan.launch(dx, dy, dt, doff, dtau, obuf)  # eager, outside the graph
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gstream):
            plan.launch(dx, dy, dt, doff, dtau, obuf)
        graph.replay()
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        for _ in range(reps):
            graph.replay()
        torch.cuda.synchronize()
        plan_ws[label] = round(B * reps / (time.perf_counter() - a0), 2)
        rpl = plan.results(obuf, B)
        assert [(r.status, r.j_star, r.K) for r in rpl] == [(0, r.j_star, r.K) for r in last]
        del graph
        plan.close()
    gctx.close()

    # plain: one window per call, no batching
    P = min(args.plain_windows, B)
    plain_t = []
    for k in range(P):
        w = win(k)
        px, py, pt, po, ptau = (torch.from_numpy(a).to(dev) for a in pack_batch([w]))
        ctx.estimate_batched(sensor, px, py, pt, po, ptau, s.d_lo, s.d_hi, s.eps)  # warm
        torch.cuda.synchronize()
        a = time.perf_counter()
        rp = ctx.estimate_batched(sensor, px, py, pt, po, ptau, s.d_lo, s.d_hi, s.eps)[0]
        torch.cuda.synchronize()
        plain_t.append(time.perf_counter() - a)
        assert (rp.j_star, rp.K) == (last[k].j_star, last[k].K)

    # measured denominators: conflict-free LDS atomic adds (no return), HBM stream read
    peaks = ctx.measure_peaks()

    # roofline of the evaluation kernel (all its launches in the timed region)
    ops_step = OPS_POINT * pt_ev + OPS_INTERVAL * bd_ev + OPS_PIXEL * pix
    launches = max(prof["eval_launches"], 1)
    avg_launch_s = prof["eval_ms"] / 1e3 / launches
    ops_launch = ops_step * args.steps / launches
    achieved = ops_launch / avg_launch_s if avg_launch_s > 0 else 0.0
    # each launch must read every event of every window still searching once
    alg_bytes = EVENT_RECORD_BYTES * sum(r.steps * r.n_events for r in last) * args.steps / launches
    tkey = {"config": args.config, "windows": B, "frontier_batch": args.frontier_batch or DEFAULT_F}
    roof = {
        "bound": "alu",
        "achieved": round(achieved / 1e9, 1),
        "peak": round(PEAK_LANE_OPS / 1e9, 1),
        "unit": "Gop/s (VALU lane-ops)",
        "frac": round(achieved / PEAK_LANE_OPS, 4),
        "traffic": traffic_per_launch(tkey),
        "traffic_unit": "HBM bytes per launch",
        "algorithmic_bytes": round(alg_bytes),
        "kernel": "k_eval",
        "avg_launch_us": round(avg_launch_s * 1e6, 2),
        "launches_per_step": round(launches / args.steps, 2),
        "eval_share_of_step": round(prof["eval_ms"] / 1e3 / args.steps / sec, 3),
        # one LDS atomic add per event and hypothesis (walk steps add more)
        "lds_atomics_per_s_at_least": round((pt_ev + bd_ev) * args.steps / (prof["eval_ms"] / 1e3), 1)
        if prof["eval_ms"] > 0 else None,
        "lds_atomic_peak_measured": round(peaks["lds_atomics_per_s"], 1),
        "hbm_read_peak_measured_GBps": round(peaks["hbm_read_bytes_per_s"] / 1e9, 1),
    }

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "event-hypothesis evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.config].format(B=B),
            "windows_per_step": B,
            "events_per_window": int(n_w.mean()),
            "eps": s.eps,
            "frontier_batch": args.frontier_batch or DEFAULT_F,
        },
        "windows_per_s": {
            "batched": round(B / sec, 2),
            "batched_learned": round(learned_ws, 2) if learned_ws else None,
            "batched_learned_autotuned": round(tuned_ws, 2) if tuned_ws else None,
            "batched_from_host_buffers": round(host_ws, 2),
            "plain_one_window_per_call": round(P / sum(plain_t), 2) if plain_t else None,
            **plan_ws,
        },
        "search": {
            "nodes_expanded_mean": float(np.mean([r.nodes_expanded for r in last])),
            "nodes_expanded_mean_learned_seeds": nodes_learned,
            "steps_max": int(max(r.steps for r in last)),
            "point_event_evals": int(pt_ev),
            "interval_event_evals": int(bd_ev),
            "pixel_updates": int(pix),
            "autotuned": {k: v for k, v in tuned.items() if k in ("frontier_batch", "tile_px", "graph", "group",
                                                                   "eval_threads")} if tuned else None,
        },
        # per step time, and per time in the evaluation kernel (its HIP-event total over the timed steps)
        "rates_per_s": {
            "point_event_evals": round(pt_ev / sec, 1),
            "interval_event_evals": round(bd_ev / sec, 1),
            "pixel_updates": round(pix / sec, 1),
            "event_hyp_evals_kernel_time": round(ev_hyp * args.steps / (prof["eval_ms"] / 1e3), 1)
            if prof["eval_ms"] > 0 else None,
        },
        "roofline": roof,
    }

    if not args.no_cpu_baseline:
        from oracle import oracle as O

        # the smallest windows of the batch (all c2 windows have 100k events)
        order = np.argsort(np.diff(off), kind="stable")
        nc = max(1, min(args.cpu_windows, B))
        t_cpu = 0.0
        ev_cpu = 0
        dev64 = []
        for k in (int(v) for v in order[:nc]):
            w = win(k)
            a = time.perf_counter()
            o = O.bnb(O.Events.of_window(w), s.d_lo, s.d_hi, s.eps)
            t_cpu += time.perf_counter() - a
            ev_cpu += (o.point_evals + o.bound_evals) * w.n
            assert (o.j_star, o.K) == (last[k].j_star, last[k].K), "GPU and oracle optima differ"
            if len(dev64) < 2:  # the same method in fp64 arithmetic, for |D_gpu - D_fp64|
                _, d64 = O.bnb64(O.Events.of_window(w), s.d_lo, s.d_hi, s.eps)
                dev64.append(abs(float(last[k].d_hat) - d64))
        out["cpu_baseline"] = {
            "value": round(ev_cpu / t_cpu, 1),
            "unit": "event-hypothesis evals/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"{nc} of the step's windows (the smallest), canonical BnB, single thread "
                      f"({t_cpu:.1f} s, {nc / t_cpu:.3f} windows/s)",
            "windows_per_s": round(nc / t_cpu, 4),
        }
        out["fp64_check"] = {"windows": len(dev64), "max_abs_d_gpu_minus_d_fp64": max(dev64),
                             "eps": s.eps}
    print(json.dumps(out), flush=True)
    if net is not None:
        net.close()
    ctx.close()


if __name__ == "__main__":
    main()
