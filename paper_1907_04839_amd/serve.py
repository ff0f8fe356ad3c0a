"""Serving driver: a stream of registrations arriving over time.

``run_batched`` submits each job to a continuous-batching ``lddmm.Server``
at its arrival time (real time) and collects completions; ``run_sequential``
serves the same arrivals first come first served with one plain
``lddmm_solve`` at a time on the same GPU.  Latency is completion time minus
arrival time; throughput is jobs / (last completion - first arrival).
"""
from __future__ import annotations

import time

import numpy as np

from . import lddmm, synth


def latency_stats(arrive: np.ndarray, done: np.ndarray) -> dict:
    lat = done - arrive
    span = float(done.max() - arrive.min())
    return {"jobs": int(len(lat)), "solves_per_s": len(lat) / span, "makespan_s": span,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean())}


def make_stream(n_jobs: int, rate: float = 200.0, iters: int = 100):
    """The first n_jobs registrations of the seeded serving stream."""
    jobs = [synth.serving_job(j) for j in range(n_jobs)]
    for jb in jobs:
        jb.iters = iters
    return jobs, synth.arrivals(n_jobs, rate)


def run_batched(jobs, arrivals, precision="fp32c", max_slots: int = 32, max_n: int = 8192,
                hbm_budget_bytes: int = 1 << 30, T: int = 40, timeout: float = 600.0) -> dict:
    srv = lddmm.Server(T, precision, max_slots=max_slots, max_n=max_n,
                       hbm_budget_bytes=hbm_budget_bytes)
    try:
        ids, t_arr = [], []
        start = time.perf_counter()
        srv_zero = None
        for jb, ta in zip(jobs, arrivals):
            delay = ta - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            jid = srv.submit(jb.q0, jb.target, jb.sigma, jb.lam, max_iter=jb.iters)
            ids.append(jid)
            t_arr.append(ta)
        results = []
        deadline = time.perf_counter() + timeout
        for jid in ids:
            r = srv.result(jid, timeout=max(1.0, deadline - time.perf_counter()))
            results.append(r)
        stats = srv.stats()
    finally:
        srv.close()
    # server clock: submission happens at arrival, so shift by the first submit
    sub = np.array([r["submit_s"] for r in results])
    done = np.array([r["done_s"] for r in results])
    arr = np.asarray(t_arr)
    srv_zero = sub[0] - arr[0]
    out = latency_stats(arr, done - srv_zero)
    out["submit_lag_max_s"] = float(np.max(sub - srv_zero - arr))
    out["rounds"] = stats["rounds"]
    out["job_evaluations"] = stats["job_evaluations"]
    out["results"] = results
    return out


def run_sequential(jobs, arrivals, precision="fp32c", ctx: lddmm.Context | None = None) -> dict:
    """One lddmm_solve at a time in arrival order; job k starts when both it
    has arrived and job k-1 has finished (times measured per solve)."""
    import torch
    ctx = ctx or lddmm.Context(0)
    t_free = float(arrivals[0])
    done, results = [], []
    for jb, ta in zip(jobs, arrivals):
        q0 = torch.from_numpy(jb.q0).cuda()
        x = torch.from_numpy(jb.target).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.solve(q0, x, jb.T, jb.sigma, jb.lam, precision=precision, max_iter=jb.iters)
        dt = time.perf_counter() - t0
        start = max(t_free, float(ta))
        t_free = start + dt
        done.append(t_free)
        r["p0"] = r["p0"].cpu().numpy()
        results.append(r)
    out = latency_stats(np.asarray(arrivals, dtype=float), np.asarray(done))
    out["results"] = results
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serve the seeded registration stream")
    ap.add_argument("--jobs", type=int, default=32)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--mode", choices=["batched", "sequential", "both"], default="both")
    ap.add_argument("--max-slots", type=int, default=32)
    ap.add_argument("--hbm-budget-mb", type=int, default=1024,
                    help="the server's arena: jobs wait until their footprint fits")
    a = ap.parse_args(argv)
    jobs, arrivals = make_stream(a.jobs, a.rate, a.iters)
    out = {}
    if a.mode in ("batched", "both"):
        r = run_batched(jobs, arrivals, max_slots=a.max_slots,
                        hbm_budget_bytes=a.hbm_budget_mb << 20)
        r.pop("results")
        out["batched"] = r
        print("batched", json.dumps(r), flush=True)
    if a.mode in ("sequential", "both"):
        r = run_sequential(jobs, arrivals)
        r.pop("results")
        out["sequential"] = r
        print("sequential", json.dumps(r), flush=True)
    return out


if __name__ == "__main__":
    main()
