"""Served request stream: replays seeded Poisson arrivals against the
continuous-batching server and reports latency percentiles and throughput.

The workload is the served stream of the benchmark suite (see
`workloads.c4_requests`): Poisson arrivals, lognormal trajectory counts, N in
{1024, 2048}, per-request random-walk temperature tables.  `rate_scale`
stretches the inter-arrival times so that the offered load can be set as a
fraction of the device's capacity; `steps_cap` optionally shortens every
request's time evolution (stated in the report).
"""
from __future__ import annotations

import threading
import time

import numpy as np

from paper_2107_06147_amd import qtraj as qt
from paper_2107_06147_amd import workloads as W


def replay(ctx, requests, precision=qt.QT_FP32_BULK, segment_steps=500, rate_scale=1.0,
           steps_cap=None, hbm_budget_bytes=0, progress_s=None, max_occupancy=0.0):
    """Submits `requests` [(arrival_s, cfg)] at their (scaled) arrival times,
    waits for all, returns per-request latencies and the server's stats.
    progress_s: print a progress line every that many seconds."""
    srv = qt.Server(ctx, precision=precision, segment_steps=segment_steps,
                    hbm_budget_bytes=hbm_budget_bytes, max_occupancy=max_occupancy)
    ids = []
    t_submit = {}
    t_done = {}
    lock = threading.Lock()
    submitted = threading.Event()

    last_print = [time.perf_counter()]

    def watch():
        # completion times, taken while requests are still being submitted
        while True:
            with lock:
                open_ids = [r for r in ids if r not in t_done]
                finished_submitting = submitted.is_set()
                n_sub, n_done = len(ids), len(t_done)
            if finished_submitting and not open_ids:
                return
            now = time.perf_counter()
            if progress_s and now - last_print[0] >= progress_s:
                last_print[0] = now
                st = srv.stats()
                print("serve: %.0f s, %d submitted, %d done, %d running, %d queued, %.3g traj-steps/s busy"
                      % (now - start, n_sub, n_done, st["running"], st["queued"],
                         st["traj_steps_per_s"]), flush=True)
            for r in open_ids:
                if srv.poll(r):
                    now = time.perf_counter()
                    with lock:
                        t_done[r] = now
            time.sleep(0.001)

    start = time.perf_counter()
    watcher = threading.Thread(target=watch, daemon=True)
    watcher.start()
    offered = 0
    for (t_arr, cfg) in requests:
        if steps_cap is not None:
            cfg = dict(cfg, max_steps=int(steps_cap))
        delay = start + t_arr * rate_scale - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        t0 = time.perf_counter()
        rid = srv.submit(cfg)
        with lock:
            t_submit[rid] = t0
            ids.append(rid)
        offered += int(cfg["n_traj"])
    submitted.set()
    watcher.join()
    results = {rid: srv.wait(rid) for rid in ids}
    lat = {rid: t_done[rid] - t_submit[rid] for rid in ids}
    wall = time.perf_counter() - start
    stats = srv.stats()
    srv.close()
    v = np.array(sorted(lat.values()))
    order = sorted(ids, key=lambda r: t_submit[r])
    return {
        "latency_by_arrival_decile_s": [float(np.median([lat[r] for r in part]))
                                        for part in np.array_split(np.array(order), 10) if len(part)],
        "requests": len(ids),
        "trajectories": offered,
        "p50_latency_s": float(np.percentile(v, 50)) if len(v) else None,
        "p99_latency_s": float(np.percentile(v, 99)) if len(v) else None,
        "server_p50_latency_s": stats["p50_latency_s"],
        "server_p99_latency_s": stats["p99_latency_s"],
        "traj_steps": stats["traj_steps"],
        "traj_steps_per_s_busy": stats["traj_steps_per_s"],
        "traj_steps_per_s_wall": stats["traj_steps"] / wall if wall > 0 else None,
        "wall_s": wall,
    }, results


def offered_load(duration_s=30.0, rate=20.0):
    """Trajectory-steps per second that the stream offers at `rate`
    requests/s (mean over `duration_s` seconds of arrivals).  Every request
    runs its whole temperature table, (tau_end - tau_start)/dt steps."""
    reqs = W.c4_requests(duration_s=duration_s, rate=rate)
    total = 0.0
    for (_, cfg) in reqs:
        total += int(cfg["n_traj"]) * (float(cfg["tau"][-1]) - float(cfg["tau_start"])) / float(cfg["dt"])
    return total / duration_s


def bench_stream(ctx, duration_s=6.0, rate_scale=1.0, steps_cap=None, segment_steps=500):
    reqs = W.c4_requests(duration_s=duration_s)
    rep, _ = replay(ctx, reqs, rate_scale=rate_scale, steps_cap=steps_cap,
                    segment_steps=segment_steps)
    rep.update({"arrival_rate_per_s": 20.0 / rate_scale, "duration_s": duration_s,
                "steps_cap": steps_cap, "segment_steps": segment_steps})
    return rep


if __name__ == "__main__":
    # the served stream over its whole duration: python -m
    # paper_2107_06147_amd.serve [--duration 120] [--rate-scale 1]
    import argparse
    import json

    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--duration", type=float, default=120.0)
    ap.add_argument("--rate-scale", type=float, default=1.0)
    ap.add_argument("--segment-steps", type=int, default=500)
    ap.add_argument("--max-occupancy", type=float, default=0.0,
                    help="admitted trajectories per resident slot (0: the server's default)")
    a = ap.parse_args()
    torch.cuda.set_device(0)
    c = qt.Context(0)
    for n in (1024, 2048):
        c.plan(n, qt.QT_FP32_BULK, tune=True)
    reqs = W.c4_requests(duration_s=a.duration)
    off = offered_load(duration_s=a.duration) / a.rate_scale
    print("serve: %d requests over %.0f s, offered %.3g traj-steps/s" % (len(reqs), a.duration * a.rate_scale, off),
          flush=True)
    rep, _ = replay(c, reqs, rate_scale=a.rate_scale, segment_steps=a.segment_steps, progress_s=10.0,
                    max_occupancy=a.max_occupancy)
    rep.update({"arrival_rate_per_s": 20.0 / a.rate_scale, "duration_s": a.duration,
                "offered_load_traj_steps_per_s": off, "segment_steps": a.segment_steps,
                "max_occupancy": a.max_occupancy})
    print(json.dumps(rep))
    c.close()
