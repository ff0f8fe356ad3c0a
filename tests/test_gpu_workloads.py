"""The workloads at their own sizes and settings against the FP64 oracle.

The oracle's runs at these sizes take minutes to tens of minutes of host time
(4.3e11 pair terms for one 65536-landmark gradient at T = 50; hundreds of
loss+gradient evaluations for the solves), so their results are stored under
tests/golden/ by tests/golden/make_workload_goldens.py, which calls only the
oracle and the seeded input generators:

  * precision study: two Gaussian blobs, N = 65536, sigma 5, T = 50, one
    gradient in FP32 (one running sum per wave), FP32-compensated and FP64;
    loss, H(q0,p0), q(1), dL/dp0 and the final energy H(q(1),p(1));
  * the 4096-landmark ellipsoid registration, T = 40, 200 L-BFGS iterations
    in FP32-compensated and FP64: loss, q(1) and v0 = K(q0) p0 at the solution
    and the first 10 iterations' (loss, |g|);
  * the first 8 jobs of the serving stream (their own N, T = 40, 100
    iterations, FP32-compensated pair sums) served in one batch.

A solution's q(1) and v0 are computed by the library (FP64 forward flow and
velocity) from the GPU's p0; the references are the oracle's own.  p0 itself
is reported only: K(q0) is near singular on these clouds, so solutions that
differ in its near-null directions are equally good (q(1), v0 and the loss
agree).

The solves stop at their iteration cap, far from a stationary point.  Two
L-BFGS runs from the same start take the same steps only while they take the
same decisions; once rounding flips one (a Wolfe test, a cubic step), the
iterates are different points along nearby descent paths and their end
points differ by what the landscape does to that perturbation, not by the
precision of the pair sums.  The oracle shows this against itself: its plain
and its Neumaier-compensated solve of the 4096-landmark registration agree to
1e-8 for 114 iterations and end 4.8e-6 apart in loss, 9e-5 in q(1) and 4e-4
in v0.  So the registration's end points are gated at max(bar, 10 x that
spread), and the iterations before the paths part iteration by iteration.
The served FP32 jobs leave the FP64 path within a few iterations and are
compared as registrations of equal quality (see their test)."""
import os

import numpy as np
import pytest

from paper_1907_04839_amd import synth

from conftest import ROW_TOL, rel_err, row_err, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    assert os.path.exists(path), f"{path} missing: run tests/golden/make_workload_goldens.py"
    return np.load(path)


def host(t):
    return t.detach().cpu().numpy()


# ----------------------------------------------------------------- precision study

@pytest.mark.parametrize("mode", ["fp64", "fp32c", "fp32"])
def test_blobs65536_T50_precision_study(gpu_ctx, mode):
    import torch
    pb = synth.two_blobs()
    o = golden("blobs65536_T50")
    assert int(o["n"]) == pb.n and int(o["T"]) == pb.T
    args = (to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), pb.T, pb.sigma, pb.lam)
    r = gpu_ctx.shoot_grad(*args, precision=mode)
    rf = gpu_ctx.shoot_grad(*args, precision=mode, energy="final", want_q1=False)
    torch.cuda.synchronize()
    e = dict(loss=abs(r.loss.item() - float(o["loss"])) / abs(float(o["loss"])),
             H0=abs(r.H0.item() - float(o["H0"])) / abs(float(o["H0"])),
             HT=abs(rf.H0.item() - float(o["HT"])) / abs(float(o["HT"])),
             q1=rel_err(host(r.q1), o["q1"]), q1_row=row_err(host(r.q1), o["q1"]),
             grad=rel_err(host(r.grad), o["grad"]), grad_row=row_err(host(r.grad), o["grad"]))
    print(f"[precision blobs65536 T=50 {mode}] " + " ".join(f"{k}={v:.2e}" for k, v in e.items()),
          flush=True)
    # FP32 with one running sum per wave over the wave's 2048 j of 65536
    # (the launch plan's j split): expected to lose accuracy with N
    tol = {"fp64": 1e-12, "fp32c": 1e-5, "fp32": 1e-4}[mode]
    row_tol = {"fp64": ROW_TOL["fp64"], "fp32c": ROW_TOL["fp32c"], "fp32": 1e-3}[mode]
    for k, v in e.items():
        assert v <= (row_tol if k.endswith("_row") else tol), (k, v, e)


# ----------------------------------------------------------------- full registrations

def _solution_checks(ctx, pb, p0_gpu, o):
    """loss-independent checks of a GPU solution against a stored oracle solve:
    q(1) (FP64 forward flow of the GPU's p0) and v0 = K(q0) p0 (FP64 velocity
    at the landmarks), both computed by the library."""
    import torch
    q0 = to_dev(pb.q0)
    p0 = to_dev(p0_gpu)
    q1, _, _ = ctx.shoot_forward(q0, p0, pb.T, pb.sigma, precision="fp64")
    v0 = ctx.velocity(q0, p0, q0, pb.sigma, precision="fp64")
    torch.cuda.synchronize()
    return dict(q1=row_err(host(q1), o["q1"]), v0=rel_err(host(v0), o["v0"]),
                v0_row=row_err(host(v0), o["v0"]), p0=rel_err(p0_gpu, o["p0"]))


def _spread_gate(e, spread, tol, keys):
    """Each end-point error within max(tol, 10 x the oracle's own spread under a
    change of rounding alone)."""
    for k in keys:
        bar = max(tol, 10.0 * spread[k])
        assert e[k] <= bar, (k, e[k], bar, e, spread)


def _spread(o, prefix=""):
    """The oracle's result against the same solve with compensated sums."""
    g = lambda k: o[prefix + k]  # noqa: E731
    return dict(loss=abs(float(g("loss_c")) - float(g("loss"))) / float(g("loss")),
                q1=row_err(g("q1_c"), g("q1")), v0=rel_err(g("v0_c"), g("v0")),
                v0_row=row_err(g("v0_c"), g("v0")))


@pytest.mark.parametrize("mode", ["fp64", "fp32c"])
def test_ellipsoid4096_full_registration(gpu_ctx, mode):
    """The paper-shaped registration: 200 iterations from p0 = 0 (stopped by the
    cap, not by convergence).  Gates: the (loss, |g|) trace iteration by
    iteration while the optimiser paths coincide (the first 10 iterations at
    the bar; in FP64 also the first 100, the loss to 1e-8 and |g| within 10 x
    the oracle's own spread over them), and the end point
    (loss, q(1), v0 = K(q0) p0) within max(bar, 10 x the spread the oracle
    itself shows between its plain and its compensated solve)."""
    import torch
    pb = synth.ellipsoid_warp()
    o = golden("ellipsoid4096_solve200")
    assert int(o["n"]) == pb.n and int(o["max_iter"]) == pb.iters == 200
    gtol = 1e-8 if mode == "fp64" else 1e-6
    r = gpu_ctx.solve(to_dev(pb.q0), to_dev(pb.target), pb.T, pb.sigma, pb.lam, precision=mode,
                      max_iter=pb.iters, gtol=gtol, want_trace=True)
    torch.cuda.synchronize()
    p0 = host(r["p0"])
    tr, otr, ctr = np.asarray(r["trace"]), o["trace"], o["trace_c"]
    assert min(len(tr), len(otr), len(ctr)) > 100, (len(tr), len(otr), len(ctr))

    def trace_err(a, b, k, col):
        return float((np.abs(a[:k, col] - b[:k, col]) / b[:k, col]).max())
    # the first 10 iterations at the bar; in FP64 the first 100 too: the loss at
    # 1e-8, |g| (first-order sensitive to the drift of the path, unlike the
    # loss) at 10 x the oracle's own plain-vs-compensated spread over them
    tol = 1e-12 if mode == "fp64" else 1e-5
    e = dict(loss=abs(r["loss"] - float(o["loss"])) / float(o["loss"]),
             trace10_loss=trace_err(tr, otr, 11, 0), trace10_g=trace_err(tr, otr, 11, 1))
    gates = dict(trace10_loss=tol, trace10_g=tol)
    if mode == "fp64":
        e.update(trace100_loss=trace_err(tr, otr, 101, 0), trace100_g=trace_err(tr, otr, 101, 1))
        gates.update(trace100_loss=1e-8,
                     trace100_g=max(1e-8, 10.0 * trace_err(ctr, otr, 101, 1)))
    e.update(_solution_checks(gpu_ctx, pb, p0, o))
    spread = _spread(o)
    kk = min(len(tr), len(otr))
    rel = np.abs(tr[:kk, 0] - otr[:kk, 0]) / otr[:kk, 0]
    apart = int(np.argmax(rel > 1e-8)) if (rel > 1e-8).any() else kk
    print(f"[registration ellipsoid4096 {mode}] iters {r['iters']}/{int(o['iters'])} fevals "
          f"{r['fevals']}/{int(o['fevals'])} loss {r['loss']:.12g}/{float(o['loss']):.12g}; "
          f"traces agree to 1e-8 for {apart} iterations; " +
          " ".join(f"{a}={b:.2e}" for a, b in e.items()) + "; oracle spread " +
          " ".join(f"{a}={b:.2e}" for a, b in spread.items()), flush=True)
    for k, bar in gates.items():
        assert e[k] <= bar, (k, e[k], bar, e)
    _spread_gate(e, spread, tol, ("loss", "q1", "v0", "v0_row"))
    # registration quality: the average landmark distance to the target
    assert abs(r["avg_dist"] - float(o["avg_dist"])) <= 0.01 * float(o["avg_dist"]), \
        (r["avg_dist"], float(o["avg_dist"]))


def test_serving_stream_jobs_match_oracle_solves():
    """The first 8 jobs of the seeded stream at their own N (656-7657), T = 40,
    100 iterations, FP32-compensated pair sums, served together; each against
    the oracle's FP64 L-BFGS run of the same job.  An FP32 solve leaves the
    FP64 path within a few iterations (the FP32 pair sums differ from the FP64
    ones by ~1e-6), so after 100 unconverged iterations the served job and the
    oracle sit at different points of nearby descent paths: the end points are
    compared as registrations of equal quality -- loss within 1e-3, q(1)
    within 5e-3 of the landmark scale, v0 within 1e-2, AverageDist within 5 %
    (measured: at most 3.1e-4, 1.3e-3, 2.3e-3 and 2.0 %).  That the served job
    runs the oracle's algorithm is checked elsewhere: a served job equals the
    same job solved alone (test_gpu_serve.py) and lddmm_solve follows the
    oracle's trace (the registration test above).  Where the golden record
    holds the oracle's compensated solves, their spread is printed beside."""
    import torch
    from paper_1907_04839_amd import lddmm
    o = golden("serving8_solve100")
    jobs = [synth.serving_job(j) for j in range(int(o["jobs"]))]
    with lddmm.Server(40, "fp32c", max_slots=8, max_n=8192, hbm_budget_bytes=1 << 30) as s:
        ids = [s.submit(pb.q0, pb.target, pb.sigma, pb.lam, max_iter=pb.iters) for pb in jobs]
        res = [s.result(i, timeout=300) for i in ids]
    gates = dict(loss=1e-3, q1=5e-3, v0=1e-2, avg_dist=0.05)
    with lddmm.Context(0) as ctx:
        for j, (pb, r) in enumerate(zip(jobs, res)):
            oj = {k[len(f"job{j}_"):]: o[k] for k in o.files if k.startswith(f"job{j}_")}
            assert int(oj["n"]) == pb.n and int(oj["max_iter"]) == pb.iters
            e = dict(loss=abs(r["loss"] - float(oj["loss"])) / float(oj["loss"]),
                     avg_dist=abs(r["avg_dist"] - float(oj["avg_dist"])) / float(oj["avg_dist"]))
            e.update(_solution_checks(ctx, pb, r["p0"], oj))
            spread = _spread(oj) if "loss_c" in oj else {}
            print(f"[serving job {j} n={pb.n}] iters {r['iters']}/{int(oj['iters'])} fevals "
                  f"{r['fevals']}/{int(oj['fevals'])} " +
                  " ".join(f"{a}={b:.2e}" for a, b in e.items()) +
                  ("; oracle spread " + " ".join(f"{a}={b:.2e}" for a, b in spread.items())
                   if spread else ""), flush=True)
            for k, bar in gates.items():
                assert e[k] <= bar, (j, k, e[k], bar, e)
        torch.cuda.synchronize()
