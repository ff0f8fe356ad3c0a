#!/usr/bin/env python3
"""Throughput of landmark geodesic shooting on one MI355X.

A step is one loss+gradient evaluation through the C ABI (lddmm_shoot_grad):
staging, T forward Euler steps of pair sums, the loss, and T adjoint steps of
pair sums (Alg. 1 ComputeGradient).  It counts 2 T N^2 pair interactions
(T N^2 forward + T N^2 adjoint); checkpoint recompute is not counted.

Headline workload (`value`): the largest single-GPU configuration, 65536
landmarks in two Gaussian blobs (centres 50 apart, sd 15), sigma 5, lambda 1,
T = 50, FP32 pair sums with 72-pair tiles folded into FP64 (FP64 state, loss
and adjoint state).  The same line carries the other precision modes at that
size, the 4096-landmark ellipsoid registration (T = 40) with its full solve,
the 16384-landmark sphere with checkpoints, the point flow, planar and
Runge-Kutta legs, the serving stream, and the oracle timed on the host.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work per ordered pair, in FP32 flops (an FMA counts 2, the one
# exp2 counts 1): forward 26 + 1, adjoint 61 + 1 (see the pair kernels).
FLOPS_PER_PAIR = {"fwd": 27, "adj": 62}
# Planar problems (dim 2, z terms left out): forward 18, adjoint 42.
FLOPS_PER_PAIR_PLANAR = {"fwd": 18, "adj": 42}
# VALU instructions per pair (one exp2 is one instruction).
VALU_PER_PAIR = {"fwd": 17, "adj": 38}
# Point flow (eq. 4), per point-landmark pair: 3 sub, |d|^2 (1 mul + 2 FMA),
# one exp2, 3 FMA = 15 flops in 10 VALU instructions.
FLOW_FLOPS_PER_PAIR = 15
FLOW_VALU_PER_PAIR = 10
# MI355X's published vector peaks: FP32 157.3 TFLOP/s (256 CUs x 128 FMA
# lanes per cycle x 2 flops x 2.4 GHz), FP64 78.6 TFLOP/s.  The FP32 figure is
# the ceiling even though this build emits no packed FP32 instructions: on
# gfx950 FP32 VALU instructions whose operands are all VGPRs issue faster than
# one wave64 instruction per SIMD every 4 cycles (measured: v_mul_f32 at 1.57x,
# v_fmac_f32 at 1.14x of that rate; with an SGPR operand 0.89-0.94x).
PEAK_TFLOPS = {"fp32": 157.3, "fp32c": 157.3, "fp64": 78.6}
# VALU lane-instructions per second at which the FP32 peak counts its FMAs.
PEAK_VALU_INSTR_PER_S = 157.3e12 / 2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    from paper_1907_04839_amd import synth
    if name == "ellipsoid4096":
        pb = synth.ellipsoid_warp()
    elif name == "sphere16384":
        pb = synth.sphere_autograd()
    elif name == "blobs65536":
        pb = synth.two_blobs()
    elif name == "ellipsoid1847":
        pb = synth.ellipsoid_warp(n=1847, T=40, iters=400)
    else:
        raise SystemExit(f"unknown workload {name}")
    return pb


def momentum(pb):
    import numpy as np
    # a momentum that moves the cloud: the pair work is the same for any p0
    if not pb.p0.any():
        return np.ascontiguousarray(0.5 * (pb.target - pb.q0))
    return pb.p0


def time_steps(ctx, dev, pb, precision, steps, warmup, ckpt_every=0, dim=3, integrator="euler"):
    import torch
    q0, x, p0 = dev["q0"], dev["x"], dev["p0"]
    out = dict(grad=torch.empty_like(q0), out3=torch.empty(3, dtype=torch.float64, device=q0.device))
    run = lambda: ctx.shoot_grad(q0, p0, x, pb.T, pb.sigma, pb.lam, precision=precision,  # noqa: E731
                                 ckpt_every=ckpt_every, want_q1=False, out=out, dim=dim,
                                 integrator=integrator)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, float(out["out3"][0])


def step_event_times(ctx, dev, pb, precision, steps, ckpt_every=0):
    """Each evaluation bracketed by its own pair of events on the launch stream:
    per-step median and minimum in ms."""
    import statistics
    import torch
    q0, x, p0 = dev["q0"], dev["x"], dev["p0"]
    out = dict(grad=torch.empty_like(q0), out3=torch.empty(3, dtype=torch.float64, device=q0.device))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        a.record()
        ctx.shoot_grad(q0, p0, x, pb.T, pb.sigma, pb.lam, precision=precision, want_q1=False,
                       out=out, ckpt_every=ckpt_every)
        b.record()
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in evs]
    return statistics.median(ms), min(ms)


def kernel_times(ctx, dev, pb, precision, steps, ckpt_every=0, dim=3, integrator="euler"):
    """Average pair-kernel durations from HIP events recorded on the launch stream."""
    ctx.timing(reset=True)
    ctx.set_timing(True)
    try:
        time_steps(ctx, dev, pb, precision, steps, 0, ckpt_every, dim, integrator)
    finally:
        ctx.set_timing(False)
    t = ctx.timing(reset=True)
    return dict(fwd_us=1e3 * t["fwd_ms"] / max(t["fwd_launches"], 1),
                adj_us=1e3 * t["adj_ms"] / max(t["adj_launches"], 1),
                fwd_launches=t["fwd_launches"], adj_launches=t["adj_launches"])


# Issue rates measured on the chip by the probes of librate_probe.so (filled by
# measured_ceilings(); empty when the probes did not run).
CEILINGS: dict = {}


def measured_ceilings(iters: int = 40000, reps: int = 5) -> dict:
    """Lane-operations per second of plain instructions, 8 waves per SIMD of the
    chip (2048 workgroups of 256 threads, 8 independent chains per lane): FP32 FMA
    with VGPR operands and with one SGPR operand, v_exp_f32, FP64 FMA, FP32
    multiply.  FMA rates are also given in TFLOP/s (2 flops each)."""
    import ctypes
    path = os.path.join(ROOT, "paper_1907_04839_amd", "librate_probe.so")
    lib = ctypes.CDLL(path)
    lib.rate_probe_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_double)]
    lib.rate_probe_run.restype = ctypes.c_int
    names = ["fp32_fma_vgpr", "fp32_fma_sgpr", "exp_f32", "fp64_fma", "fp32_mul_vgpr"]
    out = {}
    for kind, name in enumerate(names):
        r = ctypes.c_double(0.0)
        rc = lib.rate_probe_run(kind, 2048, iters, reps, ctypes.byref(r))
        if rc != 0:
            raise RuntimeError(f"rate probe {name} failed: hipError {rc}")
        out[name + "_per_s"] = round(r.value, 1)
    # FP32 MFMA (16x16x4: 16 FMAs per lane) alone, and 4 MFMAs interleaved with
    # 28 VALU FMAs per round: whether the matrix cores' work overlaps the VALU's
    mf, mix = ctypes.c_double(0.0), ctypes.c_double(0.0)
    for kind, r in ((5, mf), (6, mix)):
        rc = lib.rate_probe_run(kind, 2048, iters // 4, reps, ctypes.byref(r))
        if rc != 0:
            raise RuntimeError(f"rate probe {kind} failed: hipError {rc}")
    out["mfma_f32_tflops"] = round(mf.value * 16 * 2 / 1e12, 2)
    t_alone = 4 / mf.value + 28 / out["fp32_fma_vgpr_per_s"]
    out["mfma_valu_mix"] = {"round_time_vs_sum_of_alone": round((1 / mix.value) / t_alone, 3),
                            "mfma_tflops": round(mix.value * 4 * 16 * 2 / 1e12, 2),
                            "valu_fma_tflops": round(mix.value * 28 * 2 / 1e12, 2)}
    for name in ("fp32_fma_vgpr", "fp32_fma_sgpr", "fp64_fma"):
        out[name + "_tflops"] = round(2 * out[name + "_per_s"] / 1e12, 2)
    # in units of one wave64 instruction per SIMD every 4 cycles (256 CUs, 2.4 GHz)
    unit = 256 * 4 * 64 / 4 * 2.4e9
    out["per_quad_cycle"] = {n: round(out[n + "_per_s"] / unit, 3) for n in names}
    log("[bench] measured rates (per SIMD quad-cycle): " +
        " ".join(f"{k}={v}" for k, v in out["per_quad_cycle"].items()))
    return out


def roofline(n, kt, traffic=None, precision="fp32c", flops=FLOPS_PER_PAIR):
    kind = "adj" if kt["adj_us"] >= kt["fwd_us"] else "fwd"
    dur = kt[f"{kind}_us"] * 1e-6
    pairs = float(n) * n
    achieved = flops[kind] * pairs / dur / 1e12
    issue_frac = VALU_PER_PAIR[kind] * pairs / dur / PEAK_VALU_INSTR_PER_S
    out = {"bound": "alu", "kernel": f"{kind}_pair", "achieved": round(achieved, 3),
           "peak": PEAK_TFLOPS[precision], "unit": "TFLOP/s",
           "frac": round(achieved / PEAK_TFLOPS[precision], 4), "traffic": traffic,
           "avg_launch_us": round(kt[f"{kind}_us"], 2),
           "valu_issue_frac": round(issue_frac, 4)}
    if CEILINGS:
        # beside the published (packed) peak: the measured rate of plain FMAs with
        # VGPR operands, and the kernel's one exp per pair against the measured
        # v_exp_f32 rate
        key = "fp64_fma_tflops" if precision == "fp64" else "fp32_fma_vgpr_tflops"
        out["measured_fma_tflops"] = CEILINGS[key]
        out["frac_of_measured_fma"] = round(achieved / CEILINGS[key], 4)
        if precision != "fp64":
            out["trans_frac"] = round(pairs / dur / CEILINGS["exp_f32_per_s"], 4)
    return out


def issue_ceiling(pairs_per_s: float, precision: str):
    """The evaluation's ceiling in pair-interactions/s from the rates measured on
    the chip and the pair loops' instruction counts: every VALU instruction at
    the measured rate of FP32 FMAs with VGPR operands (multiplies issue a little
    faster, instructions with an SGPR operand much slower, so the bound is high)
    and the one v_exp_f32 per pair at its measured rate, not overlapped.  FP32
    modes only (the FP64 loops compute their own 2^x)."""
    if precision == "fp64" or not CEILINGS:
        return None
    valu = CEILINGS["fp32_fma_vgpr_per_s"]
    exp = CEILINGS["exp_f32_per_s"]
    t = sum((VALU_PER_PAIR[k] - 1) / valu + 1 / exp for k in ("fwd", "adj"))
    ceiling = 2 / t
    return {"pairs_per_s": round(ceiling, 1), "frac": round(pairs_per_s / ceiling, 4),
            "valu_per_pair": {k: VALU_PER_PAIR[k] - 1 for k in ("fwd", "adj")},
            "exp_per_pair": 1}


def measure(ctx, name: str, precision: str, steps: int, warmup: int, ckpt_every: int = 0,
            events: bool = True):
    """pair-interactions/s of one workload (steps timed after warmup), per-step
    event times, the pair kernels' average launch times, the roofline of the
    dominant kernel and the whole evaluation's algorithmic ALU fraction."""
    import torch
    pb = workload(name)
    dev = {k: torch.from_numpy(v).cuda() for k, v in
           (("q0", pb.q0), ("x", pb.target), ("p0", momentum(pb)))}
    pairs = 2 * pb.T * pb.n ** 2
    dt, loss = time_steps(ctx, dev, pb, precision, steps, warmup, ckpt_every)
    ms = 1e3 * dt / steps
    out = {"workload": f"{pb.name}: N={pb.n} landmarks, T={pb.T} Euler steps, sigma={pb.sigma:g}, "
                       f"lambda={pb.lam:g}" + (f", checkpoints every {ckpt_every}" if ckpt_every else ""),
           "n": pb.n, "T": pb.T, "ckpt_every": ckpt_every, "precision": precision,
           "pairs_per_step": pairs, "pairs_per_s": round(pairs * steps / dt, 1),
           "ms_per_step": round(ms, 4), "loss": loss}
    if events:
        med, mn = step_event_times(ctx, dev, pb, precision, steps, ckpt_every)
        out["ms_per_step_events"] = {"median": round(med, 4), "min": round(mn, 4)}
    kt = kernel_times(ctx, dev, pb, precision, max(1, min(steps, 20)), ckpt_every)
    out["kernel_us"] = {"fwd": round(kt["fwd_us"], 2), "adj": round(kt["adj_us"], 2)}
    out["roofline"] = roofline(pb.n, kt, measured_traffic(name, precision), precision)
    # the whole evaluation against the same peak: every forward and adjoint pair's
    # algorithmic flops (recompute launches not counted) over the step time
    flops = (FLOPS_PER_PAIR["fwd"] + FLOPS_PER_PAIR["adj"]) * pb.T * float(pb.n) ** 2
    out["whole_eval_alu_frac"] = round(flops / (ms * 1e-3) / (PEAK_TFLOPS[precision] * 1e12), 4)
    out["issue_ceiling"] = issue_ceiling(out["pairs_per_s"], precision)
    log(f"[bench] {pb.name} {precision}: {out['pairs_per_s']:.4g} pair-interactions/s, "
        f"{ms:.3f} ms/step; adj {kt['adj_us']:.2f} us, fwd {kt['fwd_us']:.2f} us per launch; "
        f"frac {out['roofline']['frac']}, whole evaluation {out['whole_eval_alu_frac']}")
    del dev
    return out


def flow_leg(ctx, precision: str, k: int = 64, reps: int = 3):
    """Deformation of a k^3 grid by the ellipsoid registration (lddmm_flow):
    the landmark forward pass plus every grid point carried through the T steps."""
    import torch
    from paper_1907_04839_amd import synth
    pb, grid = synth.ellipsoid_grid(k)
    q0, p0, x0 = (torch.from_numpy(a).cuda() for a in (pb.q0, pb.p0, grid))
    x1 = torch.empty_like(x0)
    run = lambda: ctx.flow(q0, p0, x0, pb.T, pb.sigma, precision=precision, out=x1)  # noqa: E731
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ctx.timing(reset=True)
    ctx.set_timing(True)
    try:
        run()
    finally:
        ctx.set_timing(False)
    t = ctx.timing(reset=True)
    m, n, T = len(grid), pb.n, pb.T
    pairs = float(m) * n * T
    kern = 1e-3 * t["flow_ms"] / max(t["flow_launches"], 1)
    achieved = FLOW_FLOPS_PER_PAIR * pairs / kern / 1e12
    out = {"workload": f"{pb.name}: {m} grid points, N={n}, T={T}", "points": m,
           "ms_per_call": round(1e3 * dt, 3),
           "point_pairs_per_s": round(pairs / dt, 1),
           "flow_kernel_ms": round(1e3 * kern, 3),
           "roofline": {"bound": "alu", "kernel": "flow", "achieved": round(achieved, 3),
                        "peak": PEAK_TFLOPS[precision], "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_TFLOPS[precision], 4),
                        "valu_issue_frac": round(FLOW_VALU_PER_PAIR * pairs / kern
                                                 / PEAK_VALU_INSTR_PER_S, 4)}}
    log(f"[bench] flow {m} points: {1e3 * dt:.2f} ms/call, kernel {1e3 * kern:.2f} ms, "
        f"{pairs / dt:.4g} point-landmark pairs/s, frac {out['roofline']['frac']}")
    return out


COPY_BYTES = 256 << 20


def traffic_probe(name: str, precision: str):
    """Kernels for the HBM-counter passes: a plain device copy of COPY_BYTES
    (reads and writes COPY_BYTES: the calibration of FETCH_SIZE and
    WRITE_SIZE) and two evaluations of the workload."""
    import torch
    from paper_1907_04839_amd import lddmm
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    pb = workload(name)
    dev = {k: torch.from_numpy(v).cuda() for k, v in
           (("q0", pb.q0), ("x", pb.target), ("p0", momentum(pb)))}
    with lddmm.Context(0) as ctx:
        time_steps(ctx, dev, pb, precision, 2, 0)
    log("[bench] traffic probe done")


def kernel_source_hash() -> str:
    """SHA-256 (first 16 hex digits) of the pair-kernel source with its comments
    and blank space removed: an edit to the code invalidates recorded counters,
    an edit to a comment does not."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1907_04839_amd", "csrc", "shoot_kernels.hip")
    with open(src, encoding="utf-8") as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = " ".join(text.split())
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def measured_traffic(name: str, precision: str):
    """HBM bytes per launch of the adjoint pair kernel, from the committed
    counter summary; None when there is none or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_adj_pair_{name}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith(" "):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash() or \
            vals.get("precision") != precision:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu() -> dict:
    """The host the oracle runs on: logical CPUs, the ones this process may
    use, and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def oracle_threads() -> int:
    """All the cores this process is given: the CPU share the job runs with
    (OMP_NUM_THREADS when the launcher sets it), else every CPU of the
    affinity mask."""
    aff = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(aff, int(env))) if env.isdigit() and int(env) > 0 else aff


def cpu_baseline(pb, target_s=12.0, budget_s=25.0):
    """The FP64 oracle on the host's cores: repeated loss+gradient evaluations
    of the same problem, about target_s seconds of work in all (fewer Euler
    steps than the workload's T when one evaluation would exceed budget_s)."""
    import oracle
    threads = oracle_threads()
    oracle.set_threads(threads)
    p0 = momentum(pb)
    # probe the rate on 2 steps, then size the sample
    t0 = time.perf_counter()
    oracle.shoot_grad(pb.q0, p0, pb.target, pb.sigma, pb.lam, 2)
    rate = 2 * 2 * pb.n ** 2 / (time.perf_counter() - t0)
    T = max(2, min(pb.T, int(budget_s * rate / (2 * pb.n ** 2))))
    evals = max(1, int(round(target_s * rate / (2 * T * pb.n ** 2))))
    t0 = time.perf_counter()
    for _ in range(evals):
        oracle.shoot_grad(pb.q0, p0, pb.target, pb.sigma, pb.lam, T)
    dt = time.perf_counter() - t0
    # one thread, for the paper's single-CPU framing: a 2-step evaluation of a
    # seeded 4096-landmark subsample (the rate per pair does not depend on N)
    from paper_1907_04839_amd import synth
    sub = synth.subsample(pb, min(pb.n, 4096))
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.shoot_grad(sub.q0, momentum(sub), sub.target, sub.sigma, sub.lam, 2)
    one = 2 * 2 * sub.n ** 2 / (time.perf_counter() - t1)
    oracle.set_threads(threads)
    return {"value": round(evals * 2 * T * pb.n ** 2 / dt, 1), "unit": "pair-interactions/s",
            "cores": threads, "kind": "oracle", "seconds": round(dt, 2),
            "value_1_thread": round(one, 1), "host": host_cpu(),
            "sample": f"{evals} FP64 loss+gradient evaluation(s) of the N={pb.n} workload with "
                      f"T={T} of its {pb.T} Euler steps ({evals * 2 * T * pb.n ** 2:.3g} pairs)"}


def full_solve(ctx, dev, pb, precision):
    """One complete registration of the workload (Alg. 1): on-device L-BFGS
    from p0 = 0 for the workload's iteration count."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.solve(dev["q0"], dev["x"], pb.T, pb.sigma, pb.lam, precision=precision,
                  max_iter=pb.iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pairs = 2 * pb.T * pb.n ** 2 * r["fevals"]
    out = {"seconds": round(dt, 4), "iters": r["iters"], "fevals": r["fevals"],
           "status": r["status"], "loss": r["loss"], "avg_dist": r["avg_dist"],
           "max_dist": r["max_dist"], "pair_interactions_per_s": round(pairs / dt, 1)}
    log(f"[bench] full solve: {dt:.3f} s for {r['iters']} iterations / {r['fevals']} "
        f"evaluations, {pairs / dt:.4g} pair-interactions/s, AverageDist {r['avg_dist']:.4g}")
    return out


def planar_leg(ctx, precision, steps=10):
    """The planar ellipse workload (4096 landmarks in the plane z = 0, T = 40)
    through the 2D-specialised pair loops and, for comparison, the 3D ones."""
    import torch
    from paper_1907_04839_amd import synth
    pb = synth.ellipse_warp()
    dev = {k: torch.from_numpy(v).cuda() for k, v in
           (("q0", pb.q0), ("x", pb.target), ("p0", momentum(pb)))}
    pairs = 2 * pb.T * pb.n ** 2
    d2, _ = time_steps(ctx, dev, pb, precision, steps, 2, dim=2)
    d3, _ = time_steps(ctx, dev, pb, precision, steps, 2, dim=3)
    kt = kernel_times(ctx, dev, pb, precision, 2, dim=2)
    out = {"workload": f"{pb.name}: N={pb.n} planar landmarks, T={pb.T}",
           "pairs_per_s": round(pairs * steps / d2, 1),
           "pairs_per_s_3d_loops": round(pairs * steps / d3, 1),
           "speedup": round(d3 / d2, 3),
           "roofline": roofline(pb.n, kt, precision=precision, flops=FLOPS_PER_PAIR_PLANAR)}
    log(f"[bench] planar: {out['pairs_per_s']:.4g} pair-interactions/s "
        f"({out['speedup']:.2f}x the 3D loops)")
    return out


def rk4_leg(ctx, precision, steps=10):
    """Classical Runge-Kutta steps on the ellipsoid workload.  T = 10 RK4 steps
    take as many pair-sum launches (40 forward, 40 adjoint) and pair terms as the
    workload's T = 40 Euler steps; both are timed, and both flows' q(1) are
    compared in FP64 with a fine RK4 reference (T = 160)."""
    import dataclasses
    import torch
    pb = workload("ellipsoid4096")
    p0 = momentum(pb)
    dev = {k: torch.from_numpy(v).cuda() for k, v in (("q0", pb.q0), ("x", pb.target), ("p0", p0))}
    rk = dataclasses.replace(pb, T=10)
    pairs = 2 * 4 * rk.T * pb.n ** 2
    d_rk, _ = time_steps(ctx, dev, rk, precision, steps, 2, integrator="rk4")
    d_eu, _ = time_steps(ctx, dev, pb, precision, steps, 2)
    kt = kernel_times(ctx, dev, rk, precision, 2, integrator="rk4")

    def q1(T, integ, prec="fp64"):
        r = ctx.shoot_forward(dev["q0"], dev["p0"], T, pb.sigma, precision=prec, integrator=integ)
        torch.cuda.synchronize()
        return r[0].cpu().numpy()
    import numpy as np
    ref = q1(160, "rk4")
    err = lambda a: float(np.linalg.norm(a - ref) / np.linalg.norm(ref))  # noqa: E731
    out = {"workload": f"{pb.name} with T=10 Runge-Kutta steps (N={pb.n})",
           "pairs_per_s": round(pairs * steps / d_rk, 1),
           "ms_per_eval": round(1e3 * d_rk / steps, 3),
           "euler_T40_ms_per_eval": round(1e3 * d_eu / steps, 3),
           "q1_rel_err_vs_rk4_T160": {"rk4_T10_fp64": err(q1(10, "rk4")),
                                      "euler_T40_fp64": err(q1(40, "euler")),
                                      "rk4_T10_" + precision: err(q1(10, "rk4", precision)),
                                      "euler_T40_" + precision: err(q1(40, "euler", precision))},
           "roofline": roofline(pb.n, kt, precision=precision)}
    e = out["q1_rel_err_vs_rk4_T160"]
    log(f"[bench] rk4: {out['pairs_per_s']:.4g} pair-interactions/s, {out['ms_per_eval']} ms per "
        f"evaluation (Euler T=40: {out['euler_T40_ms_per_eval']} ms); q(1) error RK4 T=10 "
        f"{e['rk4_T10_fp64']:.2e} vs Euler T=40 {e['euler_T40_fp64']:.2e}")
    return out


def paper_scale_solve(ctx, precision):
    """A registration at the scale of the paper's own experiment (1847 landmarks,
    T = 40, up to 400 L-BFGS iterations), on the synthetic ellipsoid recipe: the
    paper's 32 s on a GTX 980 Ti is for its private data, so this is context only."""
    import torch
    from paper_1907_04839_amd import synth
    pb = synth.ellipsoid_warp(n=1847, T=40, iters=400)
    dev = {"q0": torch.from_numpy(pb.q0).cuda(), "x": torch.from_numpy(pb.target).cuda()}
    out = full_solve(ctx, dev, pb, precision)
    out["workload"] = f"{pb.name}: N=1847, T=40, max 400 iterations, sigma={pb.sigma:g}"
    return out


def alg3_leg(ctx, n: int, reps: int = 10):
    """Sec. 2.4's materialised-matrix forward step (Alg. 3: six N x N FP32 term
    matrices, rows summed by rocBLAS sgemv) beside liblddmm's fused forward step,
    on the same landmarks and momentum (the ellipsoid recipe at N landmarks).
    Context for the paper's 25-30x (Alg. 3) vs 60-70x (shared memory) framing."""
    import torch
    from paper_1907_04839_amd import alg3, synth
    pb = synth.ellipsoid_warp(n=n, T=40, iters=1)
    q0 = torch.from_numpy(pb.q0).cuda()
    p0 = torch.from_numpy(momentum(pb)).cuda()
    wsb = alg3.workspace_bytes(n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    with alg3.Alg3(0) as a3:
        out = (torch.empty_like(q0), torch.empty_like(q0))
        mat = timed(lambda: a3.pair_forward(q0, p0, pb.sigma, ws=ws, out=out))
        mat_alloc = timed(lambda: a3.pair_forward(q0, p0, pb.sigma, out=out))
    fused_T = timed(lambda: ctx.shoot_forward(q0, p0, pb.T, pb.sigma, precision="fp32c"))
    ctx.timing(reset=True)
    ctx.set_timing(True)
    try:
        ctx.shoot_forward(q0, p0, pb.T, pb.sigma, precision="fp32c")
    finally:
        ctx.set_timing(False)
    t = ctx.timing(reset=True)
    fused_us = 1e3 * t["fwd_ms"] / max(t["fwd_launches"], 1)
    del ws
    out = {"workload": f"{pb.name}: one forward step, N={n}",
           "materialised_ms": round(mat, 4), "materialised_with_alloc_ms": round(mat_alloc, 4),
           "fused_step_ms": round(fused_T / pb.T, 4), "fused_pair_kernel_us": round(fused_us, 2),
           "materialised_over_fused": round(mat / (fused_T / pb.T), 2),
           "materialised_workspace_bytes": wsb}
    log(f"[bench] alg3 N={n}: materialised {mat:.3f} ms ({mat_alloc:.3f} with alloc/free), fused "
        f"{fused_T / pb.T:.4f} ms per step ({out['materialised_over_fused']}x), "
        f"{wsb / 2**20:.0f} MiB of term matrices")
    return out


def serving(n_jobs: int, rate: float = 200.0):
    """Registrations of uneven N (log-uniform in [500, 8000], T 40, 100
    L-BFGS iterations, FP32 sums) arriving as Poisson(rate): continuous
    batching vs one plain solve at a time, on the same arrivals."""
    from paper_1907_04839_amd import serve
    jobs, arrivals = serve.make_stream(n_jobs, rate)
    log(f"[bench] serving {n_jobs} jobs (batched) ...")
    b = serve.run_batched(jobs, arrivals)
    log(f"[bench] batched: {b['solves_per_s']:.3g} solves/s, p50 {b['p50_s']:.3f} s, "
        f"p99 {b['p99_s']:.3f} s")
    log(f"[bench] serving {n_jobs} jobs (sequential) ...")
    q = serve.run_sequential(jobs, arrivals)
    log(f"[bench] sequential: {q['solves_per_s']:.3g} solves/s, p50 {q['p50_s']:.3f} s, "
        f"p99 {q['p99_s']:.3f} s")
    keep = ("jobs", "solves_per_s", "p50_s", "p99_s", "mean_s", "makespan_s")
    return {"workload": f"{n_jobs} registrations, N log-uniform in [500, 8000], T=40, 100 "
                        f"iterations, Poisson arrivals at {rate:g}/s, fp32c",
            "batched": {k: round(b[k], 4) for k in keep},
            "sequential": {k: round(q[k], 4) for k in keep},
            "speedup_solves_per_s": round(b["solves_per_s"] / q["solves_per_s"], 3),
            "batched_rounds": b["rounds"], "batched_job_evaluations": b["job_evaluations"]}


def admission(n_jobs: int = 64, budget_mb: int = 64, rate: float = 200.0):
    """The same stream through a server whose arena is only budget_mb: jobs wait
    until their HBM footprint fits, so admission, not compute, limits the batch."""
    from paper_1907_04839_amd import lddmm, serve
    jobs, arrivals = serve.make_stream(n_jobs, rate)
    cfg = lddmm.server_config(40, "fp32c", max_slots=32, max_n=8192)
    fps = [lddmm.job_footprint(cfg, jb.n) for jb in jobs]
    log(f"[bench] admission: {n_jobs} jobs through a {budget_mb} MB arena ...")
    b = serve.run_batched(jobs, arrivals, hbm_budget_bytes=budget_mb << 20)
    keep = ("jobs", "solves_per_s", "p50_s", "p99_s", "mean_s", "makespan_s")
    out = {"workload": f"first {n_jobs} jobs of the serving stream, arena {budget_mb} MB",
           "hbm_budget_bytes": budget_mb << 20, "job_footprint_bytes_max": max(fps),
           "job_footprint_bytes_mean": round(sum(fps) / len(fps)),
           "batched": {k: round(b[k], 4) for k in keep}, "batched_rounds": b["rounds"]}
    log(f"[bench] admission-limited: {b['solves_per_s']:.3g} solves/s, p99 {b['p99_s']:.3f} s")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="blobs65536",
                    choices=["blobs65536", "ellipsoid4096", "sphere16384", "ellipsoid1847"])
    ap.add_argument("--precision", default="fp32c", choices=["fp32", "fp32c", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="only the headline workload")
    ap.add_argument("--serve-jobs", type=int, default=512,
                    help="registrations of the seeded Poisson stream for the serving leg (0: skip)")
    ap.add_argument("--admission-jobs", type=int, default=64,
                    help="jobs through a 64 MB arena for the admission leg (0: skip)")
    ap.add_argument("--flow-only", action="store_true",
                    help="time only the grid deformation (lddmm_flow) and print its record")
    ap.add_argument("--rk4-only", action="store_true",
                    help="time only the Runge-Kutta leg and print its record")
    ap.add_argument("--alg3-only", action="store_true",
                    help="time only the materialised-matrix (Alg. 3) ablation and print it")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for rocprofv3 --pmc passes: a 256 MiB copy (calibration) and 2 steps")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the landmark problem is solved on a "
              "single MI355X); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1907_04839_amd import lddmm

    torch.cuda.set_device(0)
    if args.traffic_probe:
        traffic_probe(args.workload, args.precision)
        return
    if args.flow_only:
        with lddmm.Context(0) as ctx:
            print(json.dumps(flow_leg(ctx, args.precision)), flush=True)
        return
    if args.rk4_only:
        with lddmm.Context(0) as ctx:
            print(json.dumps(rk4_leg(ctx, args.precision)), flush=True)
        return
    if args.alg3_only:
        with lddmm.Context(0) as ctx:
            print(json.dumps({f"n{n}": alg3_leg(ctx, n) for n in (1847, 4096)}), flush=True)
        return
    pb = workload(args.workload)
    ckpt = pb.ckpt_every

    extra = {}
    try:
        CEILINGS.update(measured_ceilings())
        extra["measured_ceilings"] = dict(CEILINGS)
    except (OSError, RuntimeError) as e:
        log(f"[bench] rate probes unavailable: {e}")
    with lddmm.Context(0) as ctx:
        log(f"[bench] {pb.name} N={pb.n} T={pb.T} {args.precision}: warmup {args.warmup}, "
            f"timing {args.steps} steps")
        head = measure(ctx, args.workload, args.precision, args.steps, args.warmup, ckpt)
        ctx.check()
        if not args.quick:
            # the other precision modes at the headline size
            modes = {}
            for prec in ("fp32", "fp32c", "fp64"):
                if prec == args.precision:
                    modes[prec] = {k: head[k] for k in ("pairs_per_s", "ms_per_step",
                                                        "whole_eval_alu_frac", "issue_ceiling",
                                                        "roofline")}
                    continue
                k = max(2, min(args.steps, 3 if pb.n >= 65536 else 10))
                m = measure(ctx, args.workload, prec, k, 1, ckpt, events=False)
                modes[prec] = {k2: m[k2] for k2 in ("pairs_per_s", "ms_per_step",
                                                     "whole_eval_alu_frac", "issue_ceiling",
                                                     "roofline")}
            extra["modes"] = modes
            # the 4096-landmark ellipsoid registration: evaluation rate, modes, full solve
            if args.workload != "ellipsoid4096":
                e = measure(ctx, "ellipsoid4096", args.precision, max(args.steps, 40), 5)
                e["modes_pairs_per_s"] = {args.precision: e["pairs_per_s"]}
                for prec in ("fp32", "fp32c", "fp64"):
                    if prec != args.precision:
                        e["modes_pairs_per_s"][prec] = measure(
                            ctx, "ellipsoid4096", prec, 10, 1, events=False)["pairs_per_s"]
                epb = workload("ellipsoid4096")
                edev = {"q0": torch.from_numpy(epb.q0).cuda(),
                        "x": torch.from_numpy(epb.target).cuda()}
                e["solve"] = full_solve(ctx, edev, epb, args.precision)
                extra["ellipsoid4096"] = e
            if args.workload != "sphere16384":
                extra["sphere16384"] = measure(ctx, "sphere16384", args.precision, 3, 1, 10,
                                               events=False)
            extra["flow"] = flow_leg(ctx, args.precision)
            extra["paper_scale_solve"] = paper_scale_solve(ctx, args.precision)
            extra["planar"] = planar_leg(ctx, args.precision)
            extra["rk4"] = rk4_leg(ctx, args.precision)
            extra["alg3_ablation"] = {f"n{n}": alg3_leg(ctx, n) for n in (1847, 4096)}

    if not args.quick:
        if args.serve_jobs > 0:
            extra["serving"] = serving(args.serve_jobs)
        if args.admission_jobs > 0:
            extra["admission"] = admission(args.admission_jobs, 64)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(pb)
        log(f"[bench] cpu baseline {cpu['value']:.4g} pair-interactions/s on {cpu['cores']} threads")

    rec = {
        "metric": "pair-interactions/s fwd+adjoint (one loss+gradient evaluation)",
        "value": head["pairs_per_s"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "ms_per_step_events": head["ms_per_step_events"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": head["workload"], "precision": args.precision,
                   "pairs_per_step": head["pairs_per_step"]},
        "roofline": head["roofline"],
        "whole_eval_alu_frac": head["whole_eval_alu_frac"],
        "issue_ceiling": head["issue_ceiling"],
        "kernel_us": head["kernel_us"],
        "cpu_baseline": cpu,
    }
    rec.update(extra)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
