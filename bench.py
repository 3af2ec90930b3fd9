#!/usr/bin/env python3
"""Benchmark of the exact divergence estimator on one MI355X.

Workload (one "step", default): one batched call that certifies the
canonical optimum of every window of the 256-window 1280x720 stress batch:
synthetic ventral-descent windows of 100k-5M events (log-uniform) per 0.25 s
plus 0.1% hot pixels firing at 1 kHz, 20,490 textured surface points, 30%
uniform noise, 0.5 px jitter, true D ~ U(0.05, 1.5), searching D in [0, 2]
with eps = 1e-5 (grid depth 18).  The step runs the whole hot path: event
binning, point and interval evaluations and the device frontier.  Inputs are
resident in HBM before the timed region starts.

Printed: one JSON line with event-hypothesis evaluations per second (value),
certified windows per second (batched; batched and seeded by the learned
proposal; every child bounded exactly, without the endpoint certificates;
Algorithm 1's gamma stop with and without the seeds; the batch
handed over in host memory; the asynchronous plan replayed as a graph; plain
one-window calls), the roofline of the hypothesis-evaluation kernel, the CPU
oracle timed over the host cores on a bounded sample of the same windows,
and shorter lines of the 346x260 and 640x480 batches.  Progress goes to
stderr.
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
    "c2": "{B} windows of the 346x260 config per step: 100k events/0.25 s window, 2000 textured points, 20% noise, "
          "D ~ U(0.05,0.8), search D in [0,1.5], eps 1e-5 (L=18), batched certified BnB",
    "c3": "{B} windows of the 640x480 config per step: 50k-1M events (log-uniform) per 0.25 s window, D drifting "
          "0.1 to 0.6, 20% noise, search D in [0,1.5], eps 1e-5 (L=18), batched certified BnB",
    "c5": "{B} windows of the 1280x720 stress config per step: 100k-5M events (log-uniform) per 0.25 s window plus "
          "0.1% hot pixels at 1 kHz, 30% noise, D ~ U(0.05,1.5), search D in [0,2], eps 1e-5 (L=18), batched "
          "certified BnB",
}
BATCH = {"c2": 32, "c3": 64, "c5": 256}
# (timed steps, warm-up steps) of the shorter lines of the other batches
EXTRA_STEPS = {"c2": (20, 3), "c3": (5, 2), "c5": (3, 1)}
# oracle sample per batch: the smallest windows, spread over the host cores
CPU_WINDOWS = {"c2": 32, "c3": 32, "c5": 64}

# Algorithmic VALU lane-operations of the fp32 statement per unit of work
# (what the method must compute, not what the kernel issues):
OPS_POINT = 11     # per event and point hypothesis: 2 fma, 4 range compares, 2 floor, 1 index mad, 1 add, 1 increment
OPS_INTERVAL = 22  # per event and interval: two endpoint warps as above, N_low test, start pixel
OPS_WALK = 6       # per walk step of the upper-bound image: step, fp64 corner compare, index, increment
# Peak lane-operation rate: 256 CUs x 64 lanes per clock (4 SIMDs x 16) x 2.4 GHz.
PEAK_LANE_OPS = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12  # bytes/s, MI355X specification
# The library's default frontier batch (nodes expanded together per window and step).
DEFAULT_F = 96
# Bytes of one prepared event record read by the evaluation kernel (x, y, ax, ay as fp32).
EVENT_RECORD_BYTES = 16

# HBM traffic of the evaluation kernel per launch, from two rocprofv3 --pmc
# passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean over the
# dispatches) of `bench.py --steps 1 --warmup 0 --legs main --extra none
# --no-cpu-baseline` on the default workload, each scaled by bytes/KiB that
# the same counter reads for a plain copy of 1 GiB (`bench.py
# --calibrate-copy`).  The figures hold only for the kernel sources and the
# workload they were taken on; for anything else `traffic` is null.
TRAFFIC = {
    "sources_sha256": "fdc6d8b0e93706e4a3455bfc52efb26aef555c542fff6116ae86563e543558f0",
    "workload": {"config": "c5", "windows": 256, "frontier_batch": 96},
    "fetch_kib": 5342178.8,
    "write_kib": 7266.1,
    "fetch_bytes_per_kib": 1073741824 / 524304.8,
    "write_bytes_per_kib": 1073741824 / 1048576.0,
}
KERNEL_SOURCES = ("paper_2209_13168_amd/csrc/ecmd_kernels.hip", "paper_2209_13168_amd/csrc/ecmd_internal.hpp",
                  "paper_2209_13168_amd/csrc/ecmd_api.hip")
LEGS = ("main", "learned", "exact", "gamma", "host", "plan", "plain", "autotune")


def log(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


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
    ap.add_argument("--steps", type=int, default=20, help="timed steps of the main batch")
    ap.add_argument("--warmup", type=int, default=3, help="warm-up steps of the main batch")
    ap.add_argument("--config", choices=sorted(BATCH), default="c5",
                    help="main batch: c5 = 256 windows of 1280x720 with hot pixels (default); c3 = 64 windows of "
                         "640x480; c2 = 32 windows of 346x260")
    ap.add_argument("--extra", default="c2,c3",
                    help="other batches measured with a shorter line (comma list, 'none' for none)")
    ap.add_argument("--legs", default=",".join(LEGS[:-1]),
                    help=f"legs of the main batch besides the timed steps (comma list of {', '.join(LEGS)}; "
                         "autotune takes minutes on the large batches)")
    ap.add_argument("--frontier-batch", type=int, default=0)
    ap.add_argument("--gamma", type=float, default=0.025,
                    help="Algorithm 1's stop gap (contrast units) of the gamma legs (Sec. 6 uses 0.025)")
    ap.add_argument("--cpu-windows", type=int, default=None, help="oracle sample size (smallest windows)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--weights", default=None,
                    help="trained proposal network of the learned legs (default: the one trained for the main "
                         "batch's sensor, paper_2209_13168_amd/weights/cnn_c2.npz for 346x260 and 640x480, "
                         "cnn_c5.npz for 1280x720)")
    ap.add_argument("--print-sources-sha", action="store_true", help="print the kernel sources hash and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB buffer three times (to scale HBM byte counters)")
    return ap.parse_args()


class Batch:
    """A synthetic batch in the CSR layout, on the host and on the device."""

    def __init__(self, cfg: str, dev):
        import numpy as np
        import torch

        from synth import config_windows, pack_batch
        from synth.ventral import config_specs

        self.cfg = cfg
        self.B = BATCH[cfg]
        a = time.perf_counter()
        if cfg == "c2":
            x, y, t, off, tau = pack_batch(config_windows(cfg, range(self.B)))
        else:
            from paper_2209_13168_amd.learned import windows_chunks

            parts = list(windows_chunks(list(range(self.B)), cfg=cfg, chunk=32))
            x, y, t = (np.concatenate([p[k] for p in parts]) for k in range(3))
            tau = np.concatenate([p[4] for p in parts])
            off = np.zeros(self.B + 1, np.int64)
            off[1:] = np.cumsum(np.concatenate([np.diff(p[3]) for p in parts]))
        self.spec = config_specs(cfg, 0)
        self.host = (x, y, t, off, tau)
        self.dev = tuple(torch.from_numpy(v).to(dev) for v in self.host)
        torch.cuda.synchronize()
        log(f"{cfg}: {self.B} windows, {int(off[-1])} events generated and resident in "
            f"{time.perf_counter() - a:.1f} s")

    def window(self, k: int):
        """Window k's arrays (views of the packed host arrays)."""
        x, y, t, off, tau = self.host
        a, b = int(off[k]), int(off[k + 1])
        return x[a:b], y[a:b], t[a:b], float(tau[k])


def timed(fn, reps: int):
    import torch

    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - a) / reps, r


def roofline(ctx, prof, steps: int, sec: float, last, tkey: dict, peaks=None) -> dict:
    pt_ev = sum(r.point_evals * r.n_events for r in last)
    bd_ev = sum(r.bound_evals * r.n_events for r in last)
    pix = sum(r.pixel_updates for r in last)
    walk = max(0, pix - bd_ev)  # increments beyond each interval event's start pixel
    ops_step = OPS_POINT * pt_ev + OPS_INTERVAL * bd_ev + OPS_WALK * walk
    launches = max(prof["eval_launches"], 1)
    eval_s = prof["eval_ms"] / 1e3
    avg_launch_s = eval_s / launches
    ops_launch = ops_step * steps / launches
    achieved = ops_launch / avg_launch_s if avg_launch_s > 0 else 0.0
    # each launch must read every event of every window still searching once
    alg_bytes = EVENT_RECORD_BYTES * sum(r.steps * r.n_events for r in last) * steps / launches
    traffic = traffic_per_launch(tkey)
    out = {
        "bound": "alu",
        "achieved": round(achieved / 1e9, 1),
        "peak": round(PEAK_LANE_OPS / 1e9, 1),
        "unit": "Gop/s (VALU lane-ops)",
        "frac": round(achieved / PEAK_LANE_OPS, 4),
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch",
        "algorithmic_bytes": round(alg_bytes),
        "kernel": "k_eval",
        "avg_launch_us": round(avg_launch_s * 1e6, 2),
        "launches_per_step": round(launches / steps, 2),
        "eval_share_of_step": round(eval_s / steps / sec, 3),
        "ops_per_unit": {"point_event": OPS_POINT, "interval_event": OPS_INTERVAL, "walk_step": OPS_WALK},
        "units_per_step": {"point_events": int(pt_ev), "interval_events": int(bd_ev), "walk_steps": int(walk),
                           "pixel_updates": int(pix)},
        "ops_per_launch": round(ops_launch),
    }
    if peaks is not None and eval_s > 0:
        # one LDS atomic add per point event and per upper-bound pixel
        lds = (pt_ev + pix) * steps / eval_s
        out["lds_atomics"] = {"achieved_per_s": round(lds, 1), "peak_measured_per_s": round(peaks["lds_atomics_per_s"], 1),
                              "frac": round(lds / peaks["lds_atomics_per_s"], 4)}
        hb = {"algorithmic_GBps": round(alg_bytes / avg_launch_s / 1e9, 2), "peak_GBps": HBM_PEAK / 1e9,
              "peak_measured_read_GBps": round(peaks["hbm_read_bytes_per_s"] / 1e9, 1)}
        if traffic is not None:
            hb["traffic_GBps"] = round(traffic / avg_launch_s / 1e9, 2)
            hb["frac"] = round(traffic / avg_launch_s / HBM_PEAK, 4)
        out["hbm"] = hb
    return out


def search_stats(res) -> dict:
    import numpy as np

    return {"nodes_expanded_mean": round(float(np.mean([r.nodes_expanded for r in res])), 2),
            "steps_max": int(max(r.steps for r in res)), "steps_mean": round(float(np.mean([r.steps for r in res])), 2),
            "exact_bounds_mean": round(float(np.mean([r.bound_evals for r in res])), 2),
            "bound_certs_mean": round(float(np.mean([r.bound_certs for r in res])), 2)}


def cpu_baseline(batch: Batch, last, nc: int) -> dict:
    """The C oracle's canonical BnB on the nc smallest windows, over the host cores."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O

    s = batch.spec
    off = batch.host[3]
    order = [int(v) for v in np.argsort(np.diff(off), kind="stable")[:nc]]
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        avail = os.cpu_count() or 1
    cores = max(1, min(16, avail, nc))

    def events(k):
        x, y, t, tau = batch.window(k)
        return O.Events(x, y, t, tau, s.width, s.height, s.foe)

    def one(k):
        a = time.perf_counter()
        o = O.bnb(events(k), s.d_lo, s.d_hi, s.eps)
        return k, o, time.perf_counter() - a

    O.lib()  # load before the threads start
    a = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        outs = list(ex.map(one, order))
    wall = time.perf_counter() - a
    ev = 0
    for k, o, _ in outs:
        assert (o.j_star, o.K) == (last[k].j_star, last[k].K), f"GPU and oracle optima differ on window {k}"
        ev += (o.point_evals + o.bound_evals) * int(off[k + 1] - off[k])
    single = float(np.mean([dt for _, _, dt in outs]))
    dev64 = []
    for k in order[:2]:  # the same method in fp64 arithmetic, for |D_gpu - D_fp64|
        _, d64 = O.bnb64(events(k), s.d_lo, s.d_hi, s.eps)
        dev64.append(abs(float(last[k].d_hat) - d64))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:  # pragma: no cover
        pass
    n_ev = [int(off[k + 1] - off[k]) for k in order]
    return {
        "value": round(ev / wall, 1),
        "unit": "event-hypothesis evals/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"the {nc} smallest windows of the step ({min(n_ev)}-{max(n_ev)} events), canonical BnB, "
                  f"one window per thread on {cores} threads: {wall:.1f} s wall, {nc / wall:.3f} windows/s; "
                  f"single-thread mean {single:.2f} s per window",
        "windows_per_s": round(nc / wall, 4),
        "single_thread_s_per_window": round(single, 3),
        "host_cores_available": avail,
        "cpu_model": model,
        "oracle_build": "cc " + " ".join(O.CFLAGS),
        "fp64_check": {"windows": len(dev64), "max_abs_d_gpu_minus_d_fp64": max(dev64), "eps": s.eps},
    }


def run_batch(ctx, batch: Batch, steps: int, warmup: int, fb: int, net=None, legs=(), gamma=0.025, dev=None):
    """Times the batched certified search of one batch; returns the report and the last results."""
    import numpy as np
    import torch

    from paper_2209_13168_amd import ecmd

    s = batch.spec
    B = batch.B
    dx, dy, dt, doff, dtau = batch.dev
    sensor = ecmd.sensor(s.width, s.height, s.foe)
    kw = dict(frontier_batch=fb)

    def step_plain(**extra):
        return ctx.estimate_batched(sensor, dx, dy, dt, doff, dtau, s.d_lo, s.d_hi, s.eps, **kw, **extra)

    def step_learned(**extra):
        return ctx.estimate_learned(net, sensor, dx, dy, dt, doff, dtau, s.d_lo, s.d_hi, s.eps, **kw, **extra)

    ref = None
    for _ in range(warmup):
        ref = step_plain()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    ctx.profile(reset=True)
    # no Python garbage-collection pass inside the timed region
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    res = []
    for _ in range(steps):
        res.append(step_plain())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    prof = ctx.profile(reset=True)
    ctx.set_profiling(False)
    sec = (t1 - t0) / steps
    for r in res:  # deterministic results on every step
        assert [(a.j_star, a.K) for a in r] == [(a.j_star, a.K) for a in (ref or res[0])]
    last = res[-1]
    assert all(r.status == 0 for r in last), [r.status for r in last]
    log(f"{batch.cfg}: {steps} timed steps, {sec * 1e3:.1f} ms per step")
    key = [(r.j_star, r.K) for r in last]
    ev_hyp = sum(r.event_hyp_evals for r in last)
    rep = {
        "value": ev_hyp / sec,
        "ms_per_step": sec * 1e3,
        "prof": prof,
        "events_per_window": int(np.mean([r.n_events for r in last])),
        "windows_per_s": {"batched": round(B / sec, 2)},
        "search": search_stats(last),
        "rates_per_s": {
            "point_event_evals": round(sum(r.point_evals * r.n_events for r in last) / sec, 1),
            "interval_event_evals": round(sum(r.bound_evals * r.n_events for r in last) / sec, 1),
            "pixel_updates": round(sum(r.pixel_updates for r in last) / sec, 1),
            "event_hyp_evals_kernel_time": round(ev_hyp * steps / (prof["eval_ms"] / 1e3), 1)
            if prof["eval_ms"] > 0 else None,
        },
    }
    reps = max(3, steps // 4)
    if "learned" in legs and net is not None:
        step_learned()
        t_l, rl = timed(step_learned, reps)
        assert [(r.j_star, r.K) for r in rl] == key
        rep["windows_per_s"]["batched_learned"] = round(B / t_l, 2)
        rep["search"]["learned_seeds"] = search_stats(rl)
        log(f"{batch.cfg}: learned leg {t_l * 1e3:.1f} ms per step")
    if "exact" in legs:
        # every child bounded exactly (no endpoint certificates): the same
        # nodes and result, the cost of computing every bound of Algorithm 1
        step_plain(exact_bounds=True)
        t_e, re_ = timed(lambda: step_plain(exact_bounds=True), max(2, reps // 2))
        for r, a in zip(re_, last):
            assert (r.j_star, r.K, r.nodes_expanded) == (a.j_star, a.K, a.nodes_expanded), (r, a)
        rep["windows_per_s"]["batched_all_bounds_exact"] = round(B / t_e, 2)
        rep["search"]["all_bounds_exact"] = search_stats(re_)
        log(f"{batch.cfg}: all-exact leg {t_e * 1e3:.1f} ms per step")
    if "gamma" in legs:
        # Algorithm 1's stop at a gap of gamma contrast units (Sec. 6): the
        # result is within gamma of the optimum, no longer the canonical one
        g = {}
        for label, fn in (("plain", step_plain), ("learned", step_learned if net is not None else None)):
            if fn is None:
                continue
            fn(gamma=gamma)
            t_g, rg = timed(lambda: fn(gamma=gamma), max(2, reps // 2))
            for r, a in zip(rg, last):
                assert r.status == 0 and a.contrast - r.contrast <= gamma + 1e-12, (r, a)
            g[label] = {"windows_per_s": round(B / t_g, 2), **search_stats(rg)}
        rep["gamma_stop"] = {"gamma": gamma, **g}
        log(f"{batch.cfg}: gamma legs done")
    if "autotune" in legs and net is not None:
        tuned = ctx.autotune(sensor, dx, dy, dt, doff, dtau, s.d_lo, s.d_hi, s.eps)
        step_learned()
        t_a, rt = timed(step_learned, reps)
        assert [(r.j_star, r.K) for r in rt] == key
        rep["windows_per_s"]["batched_learned_autotuned"] = round(B / t_a, 2)
        rep["search"]["autotuned"] = {k: v for k, v in tuned.items()
                                      if k in ("frontier_batch", "tile_px", "graph", "group", "eval_threads")}
        ctx.set_tuning()  # back to the default rule
    if "host" in legs:
        # the batch handed over in host memory (the library stages it: PCIe-inclusive rate)
        x, y, t, off, tau = batch.host
        hstep = lambda: ctx.estimate_batched(sensor, x, y, t, off, tau, s.d_lo, s.d_hi, s.eps, **kw)  # noqa: E731
        hstep()
        t_h, rh = timed(hstep, reps)
        assert [(r.j_star, r.K) for r in rh] == key
        rep["windows_per_s"]["batched_from_host_buffers"] = round(B / t_h, 2)
        log(f"{batch.cfg}: host-buffer leg done")
    if "plan" in legs:
        # the asynchronous plan (default step count), captured once into a
        # graph and replayed: no host synchronisation inside the search
        gstream = torch.cuda.Stream()
        gctx = ecmd.Context(0, stream=gstream.cuda_stream)
        plan = gctx.batch_plan(sensor, s.d_lo, s.d_hi, s.eps, max_windows=B, max_events=int(batch.host[3][-1]), **kw)
        obuf = plan.result_buffer(B)
        torch.cuda.synchronize()
        with torch.cuda.stream(gstream):
            plan.launch(dx, dy, dt, doff, dtau, obuf)  # eager, outside the graph
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gstream):
            plan.launch(dx, dy, dt, doff, dtau, obuf)
        graph.replay()
        t_p, _ = timed(graph.replay, reps)
        rpl = plan.results(obuf, B)
        assert [(r.status, r.j_star, r.K) for r in rpl] == [(0, j, K) for j, K in key]
        rep["windows_per_s"]["plan_graph_%d_steps" % plan.limits["max_steps"]] = round(B / t_p, 2)
        del graph
        plan.close()
        gctx.close()
        log(f"{batch.cfg}: plan leg done")
    if "plain" in legs:
        # plain: one window per call, no batching, no seed
        x, y, t, off, tau = batch.host
        one = []
        for k in range(B):
            a, b = int(off[k]), int(off[k + 1])
            o = np.array([0, b - a], np.int64)
            one.append(tuple(torch.from_numpy(v).to(dev) for v in (x[a:b], y[a:b], t[a:b], o, tau[k:k + 1])))
        big = int(np.argmax(np.diff(off)))
        ctx.estimate_batched(sensor, *one[big], s.d_lo, s.d_hi, s.eps)  # warm, largest buffers
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        rp = [ctx.estimate_batched(sensor, *one[k], s.d_lo, s.d_hi, s.eps)[0] for k in range(B)]
        torch.cuda.synchronize()
        t_p = time.perf_counter() - a0
        assert [(r.j_star, r.K) for r in rp] == key
        rep["windows_per_s"]["plain_one_window_per_call"] = round(B / t_p, 2)
        del one
        log(f"{batch.cfg}: plain leg done")
    return rep, last


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

    import torch

    from paper_2209_13168_amd import ecmd

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
    legs = tuple(v for v in args.legs.split(",") if v)
    unknown = set(legs) - set(LEGS)
    if unknown:
        raise SystemExit(f"unknown legs {sorted(unknown)}")
    extra = [c for c in args.extra.split(",") if c and c != "none" and c != args.config]
    fb = args.frontier_batch or DEFAULT_F

    ctx = ecmd.Context(0)
    net = None
    if args.weights is None:
        args.weights = os.path.join(ROOT, "paper_2209_13168_amd", "weights",
                                    "cnn_c5.npz" if args.config == "c5" else "cnn_c2.npz")
    if os.path.exists(args.weights) and ({"learned", "gamma", "autotune"} & set(legs)):
        from paper_2209_13168_amd import learned

        net, _ = learned.load(ctx, args.weights)

    batch = Batch(args.config, dev)
    rep, last = run_batch(ctx, batch, args.steps, args.warmup, args.frontier_batch, net, legs, args.gamma, dev)
    peaks = ctx.measure_peaks()
    tkey = {"config": args.config, "windows": batch.B, "frontier_batch": fb}
    roof = roofline(ctx, rep["prof"], args.steps, rep["ms_per_step"] / 1e3, last, tkey, peaks)
    out = {
        "metric": METRIC,
        "value": round(rep["value"], 1),
        "unit": "event-hypothesis evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(rep["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.config].format(B=batch.B),
            "windows_per_step": batch.B,
            "events_per_window": rep["events_per_window"],
            "events_per_step": int(batch.host[3][-1]),
            "eps": batch.spec.eps,
            "frontier_batch": fb,
        },
        "windows_per_s": rep["windows_per_s"],
        "search": rep["search"],
        "rates_per_s": rep["rates_per_s"],
        "roofline": roof,
    }
    if "gamma_stop" in rep:
        out["gamma_stop"] = rep["gamma_stop"]
    if not args.no_cpu_baseline:
        nc = min(batch.B, args.cpu_windows or CPU_WINDOWS[args.config])
        log(f"cpu baseline: oracle on {nc} windows")
        out["cpu_baseline"] = cpu_baseline(batch, last, nc)
    del batch
    torch.cuda.empty_cache()

    others = {}
    for cfg in extra:
        b = Batch(cfg, dev)
        st, wu = EXTRA_STEPS[cfg]
        r, lst = run_batch(ctx, b, st, wu, args.frontier_batch, dev=dev)
        rf = roofline(ctx, r["prof"], st, r["ms_per_step"] / 1e3, lst,
                      {"config": cfg, "windows": b.B, "frontier_batch": fb})
        others[cfg] = {"workload": WORKLOADS[cfg].format(B=b.B), "steps": st, "warmup": wu,
                       "value": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 3),
                       "windows_per_s": r["windows_per_s"], "search": r["search"],
                       "roofline": {k: rf[k] for k in ("achieved", "frac", "avg_launch_us", "eval_share_of_step")}}
        del b
        torch.cuda.empty_cache()
    if others:
        out["other_batches"] = others
    print(json.dumps(out), flush=True)
    if net is not None:
        net.close()
    ctx.close()


if __name__ == "__main__":
    main()
