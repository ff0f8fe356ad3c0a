"""Classical Runge-Kutta steps (lddmm_params.integrator = RK4) against the FP64
oracle's Runge-Kutta steps and their exact stage adjoint, through the C ABI:
forward, loss and all three gradients, both energy terms, checkpoint segments,
the flow of points, the solver, autograd and the server's rejection.

Bar as for Euler steps: 1e-12 for FP64, 1e-5 for both FP32 modes, on [N,3]
outputs normwise and row by row (row_err; the gradients' FP32 rows at the
row gate ROW_TOL)."""
import numpy as np
import pytest

from paper_1907_04839_amd import synth

from conftest import assert_gates, point_errs, rel_err, row_err, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32c": 1e-5, "fp32": 1e-5}
MODES = ["fp64", "fp32c", "fp32"]


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,T", [(1, 3), (65, 2), (300, 3), (2500, 2)])
def test_rk4_forward_matches_oracle(gpu_ctx, orc_mt, mode, n, T):
    import torch
    pb = synth.random_problem(400 + n, n, T=T)
    q1, p1, H0 = gpu_ctx.shoot_forward(to_dev(pb.q0), to_dev(pb.p0), T, pb.sigma,
                                       precision=mode, integrator="rk4")
    torch.cuda.synchronize()
    o = orc_mt.shoot_forward(pb.q0, pb.p0, pb.sigma, T, integrator="rk4")
    e = (row_err(host(q1), o["q1"]), row_err(host(p1), o["p1"]),
         abs(float(H0) - o["H0"]) / o["H0"])
    print(f"[rk4 fwd n={n} T={T} {mode}] q1={e[0]:.2e} p1={e[1]:.2e} H0={e[2]:.2e}", flush=True)
    assert max(e) <= TOL[mode]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,T,ckpt,energy", [(1, 4, 0, "initial"), (64, 3, 0, "initial"),
                                             (300, 4, 2, "initial"), (777, 3, 0, "final"),
                                             (3001, 2, 1, "final")])
def test_rk4_gradients_match_oracle(gpu_ctx, orc_mt, mode, n, T, ckpt, energy):
    import torch
    pb = synth.random_problem(500 + n, n, T=T)
    r = gpu_ctx.shoot_grad(to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), T, pb.sigma, pb.lam,
                           precision=mode, ckpt_every=ckpt, want_grad_q0=True, want_grad_x=True,
                           energy=energy, integrator="rk4")
    torch.cuda.synchronize()
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, T, all_grads=True,
                          energy=energy, integrator="rk4")
    errs = dict(loss=abs(r.loss.item() - o["loss"]) / abs(o["loss"]),
                H=abs(r.H0.item() - o["H0"]) / abs(o["H0"]),
                **point_errs("q1", host(r.q1), o["q1"]),
                **point_errs("grad", host(r.grad), o["grad"]),
                **point_errs("grad_q0", host(r.grad_q0), o["grad_q0"]),
                **point_errs("grad_x", host(r.grad_x), o["grad_x"]))
    print(f"[rk4 grad n={n} T={T} ckpt={ckpt} {energy} {mode}] "
          + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    assert_gates(errs, mode, TOL[mode])


# Runge-Kutta stage kernels take their own workgroup widths: sizes at the ends
# of the (8,2) plans (144, 271: not widened, fewer than 16 j per wave), the
# (8,3) plan at 350 and the (8,4) plan at 800 (FP32-compensated 12/12, FP32 and
# FP64 16/16), and the (8,8) plan at 1847 (232 workgroups: the same widths) and
# 4096 (512 workgroups: FP32-compensated and FP32 12/12, FP64 8/8).
RK4_PLAN_SWEEP = [144, 271, 350, 800, 1847, 4096]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", RK4_PLAN_SWEEP)
def test_rk4_every_stage_plan_matches_oracle(gpu_ctx, orc_mt, mode, n):
    import torch
    pb = synth.random_problem(900 + n, n, T=2)
    r = gpu_ctx.shoot_grad(to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), 2, pb.sigma, pb.lam,
                           precision=mode, want_grad_q0=True, integrator="rk4")
    torch.cuda.synchronize()
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, 2, all_grads=True,
                          integrator="rk4")
    errs = dict(loss=abs(r.loss.item() - o["loss"]) / abs(o["loss"]),
                **point_errs("q1", host(r.q1), o["q1"]),
                **point_errs("grad", host(r.grad), o["grad"]),
                **point_errs("grad_q0", host(r.grad_q0), o["grad_q0"]))
    print(f"[rk4 plan n={n} {mode}] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()),
          flush=True)
    assert_gates(errs, mode, TOL[mode])


@pytest.mark.parametrize("mode", MODES)
def test_rk4_checkpoint_segments_are_bitwise_identical(gpu_ctx, mode):
    import torch
    pb = synth.random_problem(61, 700, T=7)
    q0, p0, x = to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target)
    out = []
    for every in (0, 1, 3, 6, 7):
        r = gpu_ctx.shoot_grad(q0, p0, x, pb.T, pb.sigma, pb.lam, precision=mode, ckpt_every=every,
                               integrator="rk4")
        torch.cuda.synchronize()
        out.append((r.loss.item(), host(r.grad), host(r.q1)))
    for loss, g, q1 in out[1:]:
        assert loss == out[0][0]
        np.testing.assert_array_equal(g, out[0][1])
        np.testing.assert_array_equal(q1, out[0][2])


def test_rk4_single_landmark_moves_in_a_straight_line(gpu_ctx):
    import torch
    q0 = np.array([[0.3, -1.2, 2.0]])
    p0 = np.array([[0.7, 0.1, -0.4]])
    for mode in MODES:
        q1, p1, _ = gpu_ctx.shoot_forward(to_dev(q0), to_dev(p0), 5, 1.3, precision=mode,
                                          integrator="rk4")
        torch.cuda.synchronize()
        # exact up to rounding in FP64; the FP32 paths see p rounded to FP32 in the pair terms
        atol = 1e-14 if mode == "fp64" else 1e-7 * np.abs(p0).max()
        np.testing.assert_allclose(host(q1), q0 + p0, rtol=0, atol=atol)
        np.testing.assert_array_equal(host(p1), p0)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("ckpt", [0, 2])
def test_rk4_flow_matches_oracle(gpu_ctx, orc_mt, mode, ckpt):
    import torch
    pb = synth.random_problem(71, 600, T=5)
    x0 = np.random.default_rng(72).normal(size=(1500, 3)) * 2.0
    x1, q1, _ = gpu_ctx.flow(to_dev(pb.q0), to_dev(pb.p0), to_dev(x0), pb.T, pb.sigma,
                             precision=mode, ckpt_every=ckpt, want_landmarks=True,
                             integrator="rk4")
    torch.cuda.synchronize()
    o = orc_mt.flow(pb.q0, pb.p0, x0, pb.sigma, pb.T, integrator="rk4")
    e = (row_err(host(x1), o["x1"]), row_err(host(q1), o["q1"]))
    print(f"[rk4 flow ckpt={ckpt} {mode}] x1={e[0]:.2e} q1={e[1]:.2e}", flush=True)
    assert max(e) <= TOL[mode]


def test_rk4_solve_reaches_scipy_minimum(gpu_ctx, orc):
    """The GPU solver with Runge-Kutta steps reaches the minimum that scipy's
    L-BFGS-B finds on the oracle's Runge-Kutta loss and gradient (64-landmark box)."""
    import scipy.optimize as so
    import torch
    pb = synth.box_displacement()
    n = pb.n

    def f(v):
        r = orc.shoot_grad(pb.q0, v.reshape(n, 3), pb.target, pb.sigma, pb.lam, pb.T,
                           integrator="rk4")
        return r["loss"], r["grad"].ravel()
    ref = so.minimize(f, np.zeros(3 * n), jac=True, method="L-BFGS-B",
                      options=dict(maxiter=500, gtol=1e-10, ftol=1e-15))
    q0, x = to_dev(pb.q0), to_dev(pb.target)
    r = gpu_ctx.solve(q0, x, pb.T, pb.sigma, pb.lam, "fp64", integrator="rk4", max_iter=300,
                      gtol=1e-9)
    g = gpu_ctx.shoot_grad(q0, r["p0"], x, pb.T, pb.sigma, pb.lam, precision="fp64",
                           integrator="rk4")
    torch.cuda.synchronize()
    q1_ref = orc.shoot_forward(pb.q0, ref.x.reshape(n, 3), pb.sigma, pb.T, integrator="rk4")["q1"]
    el = abs(r["loss"] - ref.fun) / ref.fun
    eq = rel_err(host(g.q1), q1_ref)
    print(f"[rk4 solve box64] loss {r['loss']:.10g} vs scipy {ref.fun:.10g} ({el:.1e}), "
          f"q1 {eq:.1e}, iters {r['iters']}", flush=True)
    assert abs(r["loss"] - g.loss.item()) <= 1e-12 * g.loss.item()
    assert el < 1e-9 and eq < 1e-6


def test_rk4_autograd_matches_oracle(orc_mt):
    import torch
    from paper_1907_04839_amd import autograd
    pb = synth.random_problem(81, 400, T=3)
    p0 = to_dev(pb.p0).requires_grad_(True)
    q0 = to_dev(pb.q0).requires_grad_(True)
    x = to_dev(pb.target).requires_grad_(True)
    L = autograd.shoot_loss(p0, q0, x, pb.T, pb.sigma, pb.lam, "fp64", integrator="rk4")
    L.backward()
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, pb.T, all_grads=True,
                          integrator="rk4")
    assert abs(L.item() - o["loss"]) <= 1e-12 * abs(o["loss"])
    assert row_err(host(p0.grad), o["grad"]) <= 1e-12
    assert row_err(host(q0.grad), o["grad_q0"]) <= 1e-12
    assert row_err(host(x.grad), o["grad_x"]) <= 1e-12


def test_euler_server_rejects_rk4_jobs():
    import ctypes
    from paper_1907_04839_amd import lddmm
    pb = synth.random_problem(1170, 50, T=12)
    with lddmm.Server(12, "fp32c", max_slots=2, max_n=1024, hbm_budget_bytes=64 << 20) as s:
        prm = lddmm.make_params(pb.n, 12, pb.sigma, pb.lam, "fp32c", integrator="rk4")
        o = lddmm.solve_opts("fp32c")
        jid = ctypes.c_int64(0)
        st = lddmm.lib().lddmm_server_submit(s._h, ctypes.byref(prm), ctypes.byref(o),
                                              pb.q0.ctypes.data, pb.target.ctypes.data, None,
                                              ctypes.byref(jid))
        assert st == lddmm.EINVAL


@pytest.mark.parametrize("mode", MODES)
def test_rk4_planar_equals_3d_and_oracle(gpu_ctx, orc_mt, mode):
    """Runge-Kutta stages through the planar instances: on z = 0 data bitwise the
    3D instances' results (gradients, flow), and the oracle's within the bar."""
    import torch
    pb = synth.planar(synth.random_problem(91, 700, T=3))
    args = (to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), pb.T, pb.sigma, pb.lam)
    kw = dict(precision=mode, ckpt_every=2, want_grad_q0=True, want_grad_x=True,
              integrator="rk4")
    r2 = gpu_ctx.shoot_grad(*args, dim=2, **kw)
    r3 = gpu_ctx.shoot_grad(*args, dim=3, **kw)
    x = np.concatenate([3.0 * np.random.default_rng(92).standard_normal((900, 2)),
                        np.zeros((900, 1))], axis=1)
    f2 = gpu_ctx.flow(args[0], args[1], to_dev(x), pb.T, pb.sigma, precision=mode, dim=2,
                      integrator="rk4")
    f3 = gpu_ctx.flow(args[0], args[1], to_dev(x), pb.T, pb.sigma, precision=mode, dim=3,
                      integrator="rk4")
    torch.cuda.synchronize()
    for k in ("grad", "grad_q0", "grad_x", "q1"):
        np.testing.assert_array_equal(host(getattr(r2, k)), host(getattr(r3, k)), err_msg=k)
    np.testing.assert_array_equal(host(f2), host(f3))
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, pb.T, all_grads=True,
                          integrator="rk4")
    e = max(row_err(host(r2.grad), o["grad"]), row_err(host(r2.grad_q0), o["grad_q0"]),
            abs(r2.loss.item() - o["loss"]) / abs(o["loss"]))
    print(f"[rk4 planar {mode}] vs oracle {e:.2e}", flush=True)
    assert e <= TOL[mode]
