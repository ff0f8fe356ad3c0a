"""Continuous-batching server: a job's result is the same alone and in any
mix (bitwise: its decomposition and summation order do not depend on the
batch), admission by HBM footprint, jobs joining mid-flight, rejections, and
parity with the oracle's solver."""
import time

import numpy as np
import pytest

from paper_1907_04839_amd import synth

from conftest import rel_err, row_err

pytestmark = pytest.mark.gpu

T = 12


def small_job(j, n, iters=12):
    pb = synth.serving_job(j, n=n)
    pb.T = T
    pb.iters = iters
    return pb


def alone(pb, precision="fp32c", **kw):
    from paper_1907_04839_amd import lddmm
    with lddmm.Server(T, precision, max_slots=4, max_n=4096, hbm_budget_bytes=256 << 20) as s:
        jid = s.submit(pb.q0, pb.target, pb.sigma, pb.lam, max_iter=pb.iters, **kw)
        return s.result(jid, timeout=120)


def same(a, b):
    np.testing.assert_array_equal(a["p0"], b["p0"])
    for k in ("loss", "H0", "mismatch", "grad_norm", "avg_dist", "max_dist", "iters", "fevals",
              "status"):
        assert a[k] == b[k], k


def test_result_is_bitwise_the_same_alone_and_in_the_mix():
    from paper_1907_04839_amd import lddmm
    jobs = [small_job(j, n) for j, n in enumerate([700, 1500, 333, 2100, 64, 1000])]
    solo = [alone(pb) for pb in jobs]
    with lddmm.Server(T, "fp32c", max_slots=8, max_n=4096, hbm_budget_bytes=512 << 20) as s:
        ids = [s.submit(pb.q0, pb.target, pb.sigma, pb.lam, max_iter=pb.iters) for pb in jobs]
        mixed = [s.result(i, timeout=300) for i in ids]
        st = s.stats()
    assert st["completed"] == len(jobs)
    for a, b in zip(solo, mixed):
        same(a, b)


def test_admission_waits_for_hbm_and_slots():
    """A budget that holds two jobs: five jobs still finish, never more than
    two on the device, with the same results as alone."""
    from paper_1907_04839_amd import lddmm
    jobs = [small_job(10 + j, 1200) for j in range(5)]
    cfg = lddmm.server_config(T, "fp32c", max_slots=8, max_n=4096)
    fp = lddmm.job_footprint(cfg, 1200)
    budget = 2 * fp + fp // 2
    solo = alone(jobs[0])
    with lddmm.Server(T, "fp32c", max_slots=8, max_n=4096, hbm_budget_bytes=budget) as s:
        ids = [s.submit(pb.q0, pb.target, pb.sigma, pb.lam, max_iter=pb.iters) for pb in jobs]
        peak = 0
        deadline = time.time() + 300
        while s.stats()["completed"] < len(jobs) and time.time() < deadline:
            st = s.stats()
            peak = max(peak, st["running"])
            assert st["hbm_used_bytes"] <= budget
            time.sleep(0.002)
        res = [s.result(i, timeout=60) for i in ids]
    assert 1 <= peak <= 2
    same(res[0], solo)


def test_job_arriving_mid_flight_joins_without_perturbing():
    from paper_1907_04839_amd import lddmm
    a, b = small_job(20, 2500, iters=20), small_job(21, 900)
    ra, rb = alone(a), alone(b)
    with lddmm.Server(T, "fp32c", max_slots=4, max_n=4096, hbm_budget_bytes=256 << 20) as s:
        ia = s.submit(a.q0, a.target, a.sigma, a.lam, max_iter=a.iters)
        deadline = time.time() + 60
        while s.stats()["rounds"] < 3 and time.time() < deadline:
            time.sleep(0.001)
        ib = s.submit(b.q0, b.target, b.sigma, b.lam, max_iter=b.iters)
        res_a, res_b = s.result(ia, timeout=120), s.result(ib, timeout=120)
    assert res_b["admit_s"] > res_a["admit_s"]
    same(res_a, ra)
    same(res_b, rb)


def test_submissions_are_validated():
    from paper_1907_04839_amd import lddmm
    pb = small_job(30, 200)
    with lddmm.Server(T, "fp32c", max_slots=2, max_n=1024, hbm_budget_bytes=64 << 20) as s:
        big = small_job(31, 2000)
        with pytest.raises(lddmm.LddmmError) as e:
            s.submit(big.q0, big.target, big.sigma, big.lam)        # n > max_n
        assert e.value.status == lddmm.EINVAL
        with pytest.raises(lddmm.LddmmError) as e:
            s.submit(pb.q0, pb.target, -1.0, pb.lam)                 # sigma <= 0
        assert e.value.status == lddmm.EINVAL
        with pytest.raises(lddmm.LddmmError) as e:
            s.submit(pb.q0, pb.target, pb.sigma, pb.lam, m=0)        # bad option
        assert e.value.status == lddmm.EINVAL
    fp = lddmm.job_footprint(lddmm.server_config(T, "fp32c", max_n=4096), pb.n)
    with lddmm.Server(T, "fp32c", max_slots=2, max_n=4096, hbm_budget_bytes=fp // 2) as s:
        with pytest.raises(lddmm.LddmmError) as e:
            s.submit(pb.q0, pb.target, pb.sigma, pb.lam)            # footprint > budget
        assert e.value.status == lddmm.ENOMEM


def test_fp64_server_matches_oracle_solver(orc_mt, gpu_ctx):
    """Served FP64 registrations take the oracle's L-BFGS iterates."""
    import torch
    from paper_1907_04839_amd import lddmm
    jobs = [small_job(40 + j, n, iters=10) for j, n in enumerate([300, 800])]
    with lddmm.Server(T, "fp64", max_slots=4, max_n=4096, hbm_budget_bytes=256 << 20) as s:
        ids = [s.submit(pb.q0, pb.target, pb.sigma, pb.lam, max_iter=pb.iters) for pb in jobs]
        res = [s.result(i, timeout=120) for i in ids]
    for pb, r in zip(jobs, res):
        o = orc_mt.solve(pb.q0, pb.target, pb.sigma, pb.lam, T, orc_mt.SolveOpts(max_iter=pb.iters))
        q1g = gpu_ctx.shoot_forward(torch.from_numpy(pb.q0).cuda(), torch.from_numpy(r["p0"]).cuda(),
                                    T, pb.sigma, precision="fp64")[0].cpu().numpy()
        q1o = orc_mt.shoot_forward(pb.q0, o["p0"], pb.sigma, T)["q1"]
        el = abs(r["loss"] - o["loss"]) / o["loss"]
        print(f"[serve fp64 n={pb.n}] iters {r['iters']}/{o['iters']} fevals "
              f"{r['fevals']}/{o['fevals']} loss={el:.2e} q1={rel_err(q1g, q1o):.2e} "
              f"q1_row={row_err(q1g, q1o):.2e}", flush=True)
        assert r["iters"] == o["iters"] and r["fevals"] == o["fevals"]
        assert el < 1e-10 and rel_err(q1g, q1o) < 1e-10 and row_err(q1g, q1o) < 1e-10
        assert abs(r["avg_dist"] - o["avg_dist"]) < 1e-9 * o["avg_dist"]


def test_served_result_matches_plain_solve_within_tolerance(gpu_ctx):
    """The server and lddmm_solve split the pair sums differently (the server
    never splits j across workgroups), so results agree to FP32 tolerance."""
    import torch
    pb = small_job(50, 3000, iters=10)
    r = alone(pb)
    s = gpu_ctx.solve(torch.from_numpy(pb.q0).cuda(), torch.from_numpy(pb.target).cuda(), T,
                      pb.sigma, pb.lam, "fp32c", max_iter=pb.iters)
    torch.cuda.synchronize()
    assert abs(r["loss"] - s["loss"]) / s["loss"] < 1e-5
    assert r["iters"] == s["iters"]


def test_rk4_server_matches_plain_rk4_solve():
    """A server configured for Runge-Kutta steps: in FP64 its registrations take
    lddmm_solve's RK4 iterates (the two split the pair sums differently, so
    they agree to rounding), and in FP32 a job's result is bitwise the same
    alone and in a mix."""
    import torch
    from paper_1907_04839_amd import lddmm
    Tr = 4
    jobs = [small_job(60 + j, n, iters=8) for j, n in enumerate([500, 1300])]
    with lddmm.Server(Tr, "fp64", max_slots=4, max_n=4096, hbm_budget_bytes=256 << 20,
                      integrator="rk4") as s:
        ids = [s.submit(pb.q0, pb.target, pb.sigma, pb.lam, max_iter=pb.iters) for pb in jobs]
        res = [s.result(i, timeout=120) for i in ids]
    with lddmm.Context(0) as ctx:
        for pb, r in zip(jobs, res):
            ref = ctx.solve(torch.from_numpy(pb.q0).cuda(), torch.from_numpy(pb.target).cuda(),
                            Tr, pb.sigma, pb.lam, "fp64", max_iter=pb.iters, integrator="rk4")
            torch.cuda.synchronize()
            el = abs(r["loss"] - ref["loss"]) / ref["loss"]
            print(f"[serve rk4 fp64 n={pb.n}] iters {r['iters']}/{ref['iters']} loss {el:.2e}",
                  flush=True)
            assert r["iters"] == ref["iters"] and el < 1e-10
    mix = [small_job(70 + j, n, iters=6) for j, n in enumerate([900, 200, 1700])]

    def serve(batch):
        with lddmm.Server(Tr, "fp32c", max_slots=8, max_n=4096, hbm_budget_bytes=256 << 20,
                          integrator="rk4") as s:
            ids = [s.submit(pb.q0, pb.target, pb.sigma, pb.lam, max_iter=pb.iters)
                   for pb in batch]
            return [s.result(i, timeout=120) for i in ids]
    mixed = serve(mix)
    for pb, m in zip(mix, mixed):
        same(serve([pb])[0], m)


def test_rk4_footprint_and_integrator_mismatch():
    import ctypes
    from paper_1907_04839_amd import lddmm
    n = 1000
    eu = lddmm.job_footprint(lddmm.server_config(T, "fp32c"), n)
    rk = lddmm.job_footprint(lddmm.server_config(T, "fp32c", integrator="rk4"), n)
    # 3 T more point records and two FP64 [6][N] accumulators
    assert abs(rk - eu - (3 * T * n * 32 + 2 * 48 * n)) < 4 * 256
    pb = small_job(80, 300)
    with lddmm.Server(T, "fp32c", max_slots=2, max_n=1024, hbm_budget_bytes=64 << 20,
                      integrator="rk4") as s:
        prm = lddmm.make_params(pb.n, T, pb.sigma, pb.lam, "fp32c")   # Euler steps
        o = lddmm.solve_opts("fp32c")
        jid = ctypes.c_int64(0)
        st = lddmm.lib().lddmm_server_submit(s._h, ctypes.byref(prm), ctypes.byref(o),
                                              pb.q0.ctypes.data, pb.target.ctypes.data, None,
                                              ctypes.byref(jid))
        assert st == lddmm.EINVAL
