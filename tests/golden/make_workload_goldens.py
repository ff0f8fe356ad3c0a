"""Expected values of the full-size workloads, written by the FP64 CPU oracle.

Each target runs the oracle (and only the oracle: inputs come from the seeded
generators of ``paper_1907_04839_amd.synth``, which hold none of the method's
arithmetic) on one workload at its own size and settings, and stores what the
GPU parity tests compare against:

  blobs65536    two Gaussian blobs, N = 65536, sigma 5, T = 50: one loss and
                gradient (eq. 3 through Alg. 1's forward and backward loops),
                q(1), and the energy H(q(1), p(1)) of the final state (eq. 1)
  ellipsoid4096 the 4096-landmark ellipsoid registration, T = 40: the oracle's
                own L-BFGS run (Alg. 1 steps (e)-(f)) for 200 iterations from
                p0 = 0, with q(1), the velocity v0 = K(q0) p0 (eq. 2's Hp) at
                the solution and the (loss, |g|) trace; and the same run with
                compensated sums (keys ending in _c), whose distance from the
                first is the spread of the result under rounding alone
  serving8      the first 8 jobs of the seeded serving stream (seeds
                40000 + j, N log-uniform in [500, 8000]), T = 40: the oracle's
                L-BFGS run for 100 iterations each, as above
  serving8_spread  the same 8 solves with compensated sums, added to the
                serving8 record (keys ending in _c)

Usage:  python tests/golden/make_workload_goldens.py [target ...] [--threads K]
(several minutes to tens of minutes per target on a few host cores; the
results do not depend on the thread count).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1907_04839_amd import synth  # noqa: E402

# Solver settings of the stored runs: the library's defaults (m 5, max_fev 20,
# c1 1e-4, c2 0.9, p0 = 0 at the start) with the workloads' iteration counts.
SOLVE_ELLIPSOID = dict(max_iter=200, gtol=1e-8)
SOLVE_SERVING = dict(max_iter=100, gtol=1e-6)
SERVING_JOBS = 8


def path(name: str) -> str:
    return os.path.join(HERE, f"{name}.npz")


def log(msg: str) -> None:
    print(f"[goldens {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def make_blobs65536() -> None:
    pb = synth.two_blobs()
    log(f"blobs65536: gradient, N={pb.n} T={pb.T}")
    g = oracle.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, pb.T)
    log("blobs65536: forward for p(1)")
    f = oracle.shoot_forward(pb.q0, pb.p0, pb.sigma, pb.T)
    assert np.array_equal(f["q1"], g["q1"])
    HT = oracle.hamiltonian(f["q1"], f["p1"], pb.sigma)
    np.savez(path("blobs65536_T50"), n=pb.n, T=pb.T, sigma=pb.sigma, lam=pb.lam, seed=pb.seed,
             loss=g["loss"], H0=g["H0"], mismatch=g["mismatch"], HT=HT, q1=g["q1"],
             grad=g["grad"])
    log(f"blobs65536: loss {g['loss']:.17g} H0 {g['H0']:.17g} H(q1,p1) {HT:.17g}")


def solve_record(pb, settings, compensated: bool = False) -> dict:
    opts = oracle.SolveOpts(max_iter=settings["max_iter"], gtol=settings["gtol"])
    r = oracle.solve(pb.q0, pb.target, pb.sigma, pb.lam, pb.T, opts, compensated=compensated)
    q1 = oracle.shoot_forward(pb.q0, r["p0"], pb.sigma, pb.T)["q1"]
    v0 = oracle.pair_forward(pb.q0, r["p0"], pb.sigma)[1]
    return dict(n=pb.n, T=pb.T, sigma=pb.sigma, lam=pb.lam, seed=pb.seed,
                max_iter=settings["max_iter"], gtol=settings["gtol"], p0=r["p0"],
                loss=r["loss"], H0=r["H0"], mismatch=r["mismatch"], grad_norm=r["grad_norm"],
                avg_dist=r["avg_dist"], max_dist=r["max_dist"], iters=r["iters"],
                fevals=r["fevals"], status=r["status"], trace=r["trace"], q1=q1, v0=v0)


def make_ellipsoid4096() -> None:
    pb = synth.ellipsoid_warp()
    log(f"ellipsoid4096: solve, N={pb.n} T={pb.T} {SOLVE_ELLIPSOID}")
    rec = solve_record(pb, SOLVE_ELLIPSOID)
    log(f"ellipsoid4096: loss {rec['loss']:.17g} iters {rec['iters']} fevals {rec['fevals']}")
    # the same solve with Neumaier-compensated pair sums: it differs from the
    # first only in rounding, so its distance from it after 200 iterations is
    # the spread that rounding alone gives this (unconverged) optimiser path
    log("ellipsoid4096: the same solve with compensated sums")
    rc = solve_record(pb, SOLVE_ELLIPSOID, compensated=True)
    for k in ("loss", "q1", "v0", "p0", "trace", "iters", "fevals"):
        rec[k + "_c"] = rc[k]
    np.savez(path("ellipsoid4096_solve200"), **rec)
    log(f"ellipsoid4096 (compensated): loss {rc['loss']:.17g} iters {rc['iters']} "
        f"fevals {rc['fevals']}")


def make_serving8() -> None:
    recs = {}
    for j in range(SERVING_JOBS):
        pb = synth.serving_job(j)
        log(f"serving job {j}: solve, N={pb.n} T={pb.T} {SOLVE_SERVING}")
        r = solve_record(pb, SOLVE_SERVING)
        for k, v in r.items():
            recs[f"job{j}_{k}"] = v
        log(f"serving job {j}: loss {r['loss']:.17g} iters {r['iters']} fevals {r['fevals']}")
    np.savez(path("serving8_solve100"), jobs=SERVING_JOBS, **recs)


def make_serving8_spread() -> None:
    """The same 8 solves with compensated sums, added to the stored record
    (keys job{j}_*_c): the spread of each job's result under rounding alone."""
    old = dict(np.load(path("serving8_solve100")))
    for j in range(SERVING_JOBS):
        pb = synth.serving_job(j)
        assert int(old[f"job{j}_n"]) == pb.n
        log(f"serving job {j}: compensated solve, N={pb.n} T={pb.T} {SOLVE_SERVING}")
        r = solve_record(pb, SOLVE_SERVING, compensated=True)
        for k in ("loss", "q1", "v0", "p0", "iters", "fevals"):
            old[f"job{j}_{k}_c"] = r[k]
        log(f"serving job {j} (compensated): loss {r['loss']:.17g}")
    np.savez(path("serving8_solve100"), **old)


TARGETS = {"blobs65536": make_blobs65536, "ellipsoid4096": make_ellipsoid4096,
           "serving8": make_serving8, "serving8_spread": make_serving8_spread}


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("targets", nargs="*", default=["blobs65536", "ellipsoid4096", "serving8",
                                                   "serving8_spread"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    oracle.set_threads(a.threads)
    for t in a.targets:
        TARGETS[t]()


if __name__ == "__main__":
    main()
