"""GPU path vs the FP64 CPU oracle, through the C ABI.

Bar: 1e-12 for the FP64 path and 1e-5 for both FP32 paths, on scalars as
|diff|/|ref| and on [N,3] outputs normwise (rel_err) and row by row (row_err:
each row's error over its own norm, floored at the RMS row norm).  The
multi-step gradients of the full-size workloads (check_grad) hold their FP32
rows to ROW_TOL (10x, the rounding of FP32 positions carried through T
steps); every other row gate here is at the normwise bar.  Sizes span several
64-wide i-blocks, j-splits over several workgroups and ragged tails; the
full-size workloads are checked on sampled rows and through properties that
hold at any size.
"""
import numpy as np
import pytest

from paper_1907_04839_amd import synth

from conftest import ROW_TOL, rel_err, row_err, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32c": 1e-5, "fp32": 1e-5}
MODES = ["fp64", "fp32c", "fp32"]


def host(t):
    return t.detach().cpu().numpy()


def run_grad(ctx, pb, mode, p0=None, ckpt=0, T=None):
    import torch
    r = ctx.shoot_grad(to_dev(pb.q0), to_dev(pb.p0 if p0 is None else p0), to_dev(pb.target),
                       pb.T if T is None else T, pb.sigma, pb.lam, precision=mode,
                       ckpt_every=ckpt)
    torch.cuda.synchronize()
    return dict(loss=float(r.loss), H0=float(r.H0), mismatch=float(r.mismatch),
                grad=host(r.grad), q1=host(r.q1))


def check_grad(g, o, mode, tag=""):
    errs = dict(loss=abs(g["loss"] - o["loss"]) / abs(o["loss"]),
                H0=abs(g["H0"] - o["H0"]) / max(abs(o["H0"]), 1e-300),
                grad=rel_err(g["grad"], o["grad"]), q1=rel_err(g["q1"], o["q1"]),
                grad_row=row_err(g["grad"], o["grad"]), q1_row=row_err(g["q1"], o["q1"]))
    print(f"[{tag} {mode}] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        if k == "H0" and o["H0"] == 0.0:
            assert g["H0"] == 0.0
            continue
        assert v <= (ROW_TOL if k.endswith("_row") else TOL)[mode], (k, v)


# ----------------------------------------------------------------- forward

@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,T", [(1, 3), (2, 1), (63, 4), (64, 1), (65, 5), (777, 3), (2500, 2)])
def test_forward_matches_oracle(gpu_ctx, orc_mt, mode, n, T):
    import torch
    pb = synth.random_problem(100 + n, n, T=T)
    q1, p1, H0 = gpu_ctx.shoot_forward(to_dev(pb.q0), to_dev(pb.p0), T, pb.sigma, precision=mode)
    torch.cuda.synchronize()
    o = orc_mt.shoot_forward(pb.q0, pb.p0, pb.sigma, T)
    e = (row_err(host(q1), o["q1"]), row_err(host(p1), o["p1"]), abs(float(H0) - o["H0"]) / o["H0"])
    print(f"[fwd n={n} T={T} {mode}] q1={e[0]:.2e} p1={e[1]:.2e} H0={e[2]:.2e}", flush=True)
    assert max(e) <= TOL[mode]


def test_single_landmark_moves_in_a_straight_line(gpu_ctx):
    import torch
    q0 = np.array([[10.0, -20.0, 5.0]])
    p0 = np.array([[0.3, 0.4, -1.2]])
    for mode in MODES:
        q1, p1, H0 = gpu_ctx.shoot_forward(to_dev(q0), to_dev(p0), 17, 2.0, precision=mode)
        torch.cuda.synchronize()
        # exact in FP64; the FP32 paths see p rounded to FP32 in the pair terms
        atol = 1e-13 if mode == "fp64" else 1e-7 * np.abs(p0).max()
        np.testing.assert_allclose(host(q1), q0 + p0, rtol=0, atol=atol)
        np.testing.assert_array_equal(host(p1), p0)
        assert abs(float(H0) - 0.5 * (p0 ** 2).sum()) < (1e-15 if mode == "fp64" else 1e-7)


def test_zero_momentum_gives_no_motion(gpu_ctx):
    import torch
    pb = synth.random_problem(7, 300, T=6)
    for mode in MODES:
        q1, p1, H0 = gpu_ctx.shoot_forward(to_dev(pb.q0), to_dev(np.zeros_like(pb.q0)), 6,
                                           pb.sigma, precision=mode)
        torch.cuda.synchronize()
        np.testing.assert_allclose(host(q1), pb.q0, rtol=0, atol=1e-13)
        assert np.all(host(p1) == 0.0) and float(H0) == 0.0


# ----------------------------------------------------------------- gradient

@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,T", [(1, 4), (64, 6), (257, 3), (300, 5), (777, 6), (3001, 4)])
def test_gradient_matches_oracle(gpu_ctx, orc_mt, mode, n, T):
    pb = synth.random_problem(200 + n, n, T=T)
    g = run_grad(gpu_ctx, pb, mode)
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, T)
    check_grad(g, o, mode, f"grad n={n} T={T}")


# Every (waves per workgroup W, j-chunks S) plan that sizes up to 20000 take, at its
# smallest N and at a ragged N inside its range (N and the per-wave j range not
# multiples of 64): (1,1) 1 16 31, (2,1) 32 40 47, (2,2) 48 56 63, (4,1) 64 72 79,
# (4,2) 80 104 127, (8,1) 128 136 143, (8,2) 144 208 271, (8,3) 272 336 399,
# (8,4) 400 911 19089, (8,8) 912 9800.  The (8,8), (8,4) and (8,3) plans run
# wider workgroups (forward/adjoint waves): FP32-compensated 12/12, FP32 16/16,
# FP64 12/12, or 16/16 wherever a launch has at most 256 workgroups (e.g.
# 272-399, 911).
PLAN_SWEEP = [1, 16, 31, 32, 40, 47, 48, 56, 63, 64, 72, 79, 80, 104, 127, 128, 136, 143, 144,
              208, 271, 272, 336, 399, 400, 911, 912, 9800, 19089]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", PLAN_SWEEP)
def test_every_launch_plan_matches_oracle(gpu_ctx, orc_mt, mode, n):
    pb = synth.random_problem(700 + n, n, T=2)
    g = run_grad(gpu_ctx, pb, mode)
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, 2)
    check_grad(g, o, mode, f"plan n={n}")


@pytest.mark.parametrize("mode", MODES)
def test_box64_workload(gpu_ctx, orc_mt, mode):
    """The 64-landmark box problem (sigma 10, T 10) at p0 = 0 and at a random p0."""
    pb = synth.box_displacement()
    rng = np.random.default_rng(5)
    for p0 in (pb.p0, 2.0 * rng.standard_normal(pb.q0.shape)):
        g = run_grad(gpu_ctx, pb, mode, p0=p0)
        o = orc_mt.shoot_grad(pb.q0, p0, pb.target, pb.sigma, pb.lam, pb.T)
        check_grad(g, o, mode, "box64")


@pytest.mark.slow
@pytest.mark.parametrize("mode", MODES)
def test_ellipsoid4096_T40_workload(gpu_ctx, orc_mt, mode):
    """The 4096-landmark ellipsoid workload at its full size (T = 40), at a
    momentum that moves the cloud most of the way to the target."""
    pb = synth.ellipsoid_warp()
    p0 = 0.8 * (pb.target - pb.q0)
    g = run_grad(gpu_ctx, pb, mode, p0=p0)
    o = orc_mt.shoot_grad(pb.q0, p0, pb.target, pb.sigma, pb.lam, pb.T)
    check_grad(g, o, mode, "ellipsoid4096")


@pytest.mark.slow
@pytest.mark.parametrize("mode", MODES)
def test_sphere16384_two_steps_full_oracle(gpu_ctx, orc_mt, mode):
    """The 16384-landmark sphere at its real shape (one workgroup per i-block,
    fused update), two Euler steps so both adjoint terms are exercised."""
    pb = synth.sphere_autograd()
    g = run_grad(gpu_ctx, pb, mode, T=2)
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, 2)
    check_grad(g, o, mode, "sphere16384 T=2")


@pytest.mark.parametrize("mode", MODES)
def test_blobs65536_one_step_sampled_rows(gpu_ctx, orc_mt, mode):
    """Full-size two-blob cloud: one Euler step (T = 1, so Hp = q1 - q0 and
    Hq = p0 - p1) checked on 192 sampled rows against the oracle's row sums."""
    import torch
    pb = synth.two_blobs()
    rows = np.random.default_rng(3).choice(pb.n, size=192, replace=False)
    rows = np.concatenate([[0, pb.n - 1], rows])
    q1, p1, _ = gpu_ctx.shoot_forward(to_dev(pb.q0), to_dev(pb.p0), 1, pb.sigma, precision=mode)
    torch.cuda.synchronize()
    Hq, Hp = orc_mt.pair_forward_rows(pb.q0, pb.p0, pb.sigma, rows)
    e_hp = row_err(host(q1)[rows] - pb.q0[rows], Hp)
    e_hq = row_err(pb.p0[rows] - host(p1)[rows], Hq)
    print(f"[blobs65536 step {mode}] Hp={e_hp:.2e} Hq={e_hq:.2e}", flush=True)
    assert max(e_hp, e_hq) <= TOL[mode]


@pytest.mark.parametrize("mode", MODES)
def test_blobs65536_one_step_gradients_sampled_rows(gpu_ctx, orc_mt, mode):
    """Full-size two-blob cloud, one Euler step (T = 1, dt = 1): after the step
    a = 2 lambda (q(1) - x) and b = 0, so dL/dp0 = B + Hp(q0,p0) and
    dL/dq0 = a + A + Hq(q0,p0), with (A, B) the adjoint pair sums at (q0, p0, a, 0).
    The oracle's full forward sums give q(1) and a; its adjoint row sums give
    sampled rows of both gradients (the adjoint kernel's plan at this size)."""
    import torch
    pb = synth.two_blobs()
    Hq, Hp = orc_mt.pair_forward(pb.q0, pb.p0, pb.sigma)
    a = 2.0 * pb.lam * (pb.q0 + Hp - pb.target)
    rows = np.random.default_rng(4).choice(pb.n, size=160, replace=False)
    rows = np.concatenate([[0, 63, 64, pb.n - 1], rows])
    A, B = orc_mt.pair_adjoint_rows(pb.q0, pb.p0, a, np.zeros_like(a), pb.sigma, rows)
    r = gpu_ctx.shoot_grad(to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), 1, pb.sigma, pb.lam,
                           precision=mode, want_grad_q0=True)
    torch.cuda.synchronize()
    e_p = row_err(host(r.grad)[rows], B + Hp[rows])
    e_q = row_err(host(r.grad_q0)[rows], a[rows] + A + Hq[rows])
    print(f"[blobs65536 one-step gradients {mode}] p0={e_p:.2e} q0={e_q:.2e}", flush=True)
    assert max(e_p, e_q) <= TOL[mode]


@pytest.mark.parametrize("mode", MODES)
def test_262144_landmarks_one_step_sampled_rows(gpu_ctx, orc_mt, mode):
    """A cloud four times the largest workload (N = 262144: 4 waves per i-block
    and the Euler update fused into the pair kernel, the plan every larger N
    takes): one step checked on sampled rows.  Naive FP32 keeps one running
    sum over 65536 pairs per wave here (measured 3e-6)."""
    import torch
    pb = synth.two_blobs(seed=1007, n=262144, T=1)
    rows = np.random.default_rng(5).choice(pb.n, size=128, replace=False)
    rows = np.concatenate([[0, 63, 64, pb.n - 1], rows])
    q1, p1, _ = gpu_ctx.shoot_forward(to_dev(pb.q0), to_dev(pb.p0), 1, pb.sigma, precision=mode)
    torch.cuda.synchronize()
    Hq, Hp = orc_mt.pair_forward_rows(pb.q0, pb.p0, pb.sigma, rows)
    e_hp = row_err(host(q1)[rows] - pb.q0[rows], Hp)
    e_hq = row_err(pb.p0[rows] - host(p1)[rows], Hq)
    print(f"[262144 step {mode}] Hp={e_hp:.2e} Hq={e_hq:.2e}", flush=True)
    assert max(e_hp, e_hq) <= TOL[mode]


# ----------------------------------------------------------------- properties

@pytest.mark.parametrize("mode", MODES)
def test_checkpoint_recompute_is_bitwise_identical(gpu_ctx, mode):
    pb = synth.random_problem(31, 700, T=23)
    full = run_grad(gpu_ctx, pb, mode)
    for every in (1, 4, 10, 22, 23, 100):     # 23 = T and beyond: the whole trajectory
        ck = run_grad(gpu_ctx, pb, mode, ckpt=every)
        assert ck["loss"] == full["loss"]
        np.testing.assert_array_equal(ck["grad"], full["grad"])
        np.testing.assert_array_equal(ck["q1"], full["q1"])


@pytest.mark.parametrize("mode", MODES)
def test_results_are_bitwise_reproducible(gpu_ctx, mode):
    pb = synth.random_problem(32, 3000, T=5)
    a = run_grad(gpu_ctx, pb, mode)
    b = run_grad(gpu_ctx, pb, mode)
    assert a["loss"] == b["loss"]
    np.testing.assert_array_equal(a["grad"], b["grad"])


def test_translation_invariance(gpu_ctx):
    pb = synth.random_problem(33, 500, T=5)
    a = run_grad(gpu_ctx, pb, "fp64")
    tau = np.array([[1000.0, -250.0, 37.5]])
    pb2 = synth.Problem("shifted", pb.q0 + tau, pb.target + tau, pb.p0, pb.sigma, pb.lam, pb.T)
    b = run_grad(gpu_ctx, pb2, "fp64")
    assert abs(a["loss"] - b["loss"]) < 1e-12 * a["loss"]
    assert row_err(b["grad"], a["grad"]) < 1e-12
    assert row_err(b["q1"] - tau, a["q1"]) < 1e-12


def test_total_momentum_conserved_at_full_size(gpu_ctx):
    """sum_i p_i is a flow invariant: checked on the 65536-landmark cloud."""
    import torch
    pb = synth.two_blobs()
    for mode in MODES:
        _, p1, _ = gpu_ctx.shoot_forward(to_dev(pb.q0), to_dev(pb.p0), 5, pb.sigma, precision=mode)
        torch.cuda.synchronize()
        d = np.abs(host(p1).sum(0) - pb.p0.sum(0)).max()
        scale = np.abs(pb.p0).sum()
        print(f"[momentum {mode}] {d / scale:.2e}", flush=True)
        assert d <= (1e-12 if mode == "fp64" else 1e-6) * scale


# ----------------------------------------------------------------- boundary

def test_invalid_arguments_are_rejected(gpu_ctx):
    import ctypes
    from paper_1907_04839_amd import lddmm
    L = lddmm.lib()
    q = to_dev(np.zeros((4, 3)))
    out3 = to_dev(np.zeros((3, 1))).view(-1)
    for prm in (lddmm.make_params(0, 3, 1.0, 1.0), lddmm.make_params(4, 0, 1.0, 1.0),
                lddmm.make_params(4, 3, 0.0, 1.0), lddmm.make_params(4, 3, 1.0, -1.0),
                lddmm.make_params(4, 3, 1.0, 1.0, precision=9)):
        rc = L.lddmm_shoot_grad(gpu_ctx.handle, ctypes.byref(prm), q.data_ptr(), q.data_ptr(),
                                q.data_ptr(), out3.data_ptr(), q.data_ptr(), None, None)
        assert rc == lddmm.EINVAL
        assert L.lddmm_last_error(gpu_ctx.handle)
    prm = lddmm.make_params(4, 3, 1.0, 1.0)
    assert L.lddmm_shoot_grad(gpu_ctx.handle, ctypes.byref(prm), None, q.data_ptr(), q.data_ptr(),
                              out3.data_ptr(), q.data_ptr(), None, None) == lddmm.EINVAL
    assert L.lddmm_shoot_grad(None, ctypes.byref(prm), q.data_ptr(), q.data_ptr(), q.data_ptr(),
                              out3.data_ptr(), q.data_ptr(), None, None) == lddmm.EINVAL
    assert L.lddmm_shoot_forward(gpu_ctx.handle, None, q.data_ptr(), q.data_ptr(), None, None,
                                 None, None) == lddmm.EINVAL


def test_workspace_beyond_hbm_is_enomem_and_the_context_recovers(orc):
    """A problem whose workspace cannot exist (2^26 landmarks, 2^20 steps: ~2 PB of
    trajectory) fails with ENOMEM before anything is enqueued; the same context
    then evaluates a small problem correctly."""
    import ctypes
    import torch
    from paper_1907_04839_amd import lddmm
    L = lddmm.lib()
    q = to_dev(np.zeros((4, 3)))                 # never read: the call fails first
    out3 = to_dev(np.zeros(3))
    with lddmm.Context(0) as ctx:
        prm = lddmm.make_params(1 << 26, 1 << 20, 1.0, 1.0)
        rc = L.lddmm_shoot_grad(ctx.handle, ctypes.byref(prm), q.data_ptr(), q.data_ptr(),
                                q.data_ptr(), out3.data_ptr(), q.data_ptr(), None, None)
        assert rc == lddmm.ENOMEM
        assert b"hipMalloc" in L.lddmm_last_error(ctx.handle)
        pb = synth.random_problem(1320, 200, T=4)
        g = run_grad(ctx, pb, "fp64")
        torch.cuda.synchronize()
    o = orc.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, 4)
    check_grad(g, o, "fp64", "after ENOMEM")


def test_context_budget_is_enforced_and_the_context_recovers(orc):
    """A context created with an HBM budget of 4 MiB refuses (ENOMEM, nothing
    enqueued) an evaluation whose workspace exceeds it and a solve whose two
    workspaces together would, then evaluates and solves problems that fit."""
    import torch
    from paper_1907_04839_amd import lddmm
    big = synth.random_problem(1322, 20000, T=40)
    assert lddmm.workspace_size(lddmm.make_params(big.n, big.T, 1.5, 1.0)) > 4 << 20
    pb = synth.random_problem(1321, 300, T=4)
    with lddmm.Context(0, hbm_budget_bytes=4 << 20) as ctx:
        with pytest.raises(lddmm.LddmmError) as e:
            ctx.shoot_grad(to_dev(big.q0), to_dev(big.p0), to_dev(big.target), big.T, big.sigma,
                           big.lam, "fp32c")
        assert e.value.status == lddmm.ENOMEM and "budget" in str(e.value)
        # 4000 landmarks, T = 2: the workspace (3.4 MiB) fits, with the solver's
        # (16 vectors of 3N doubles, 1.5 MiB) it does not
        mid = synth.random_problem(1323, 4000, T=2)
        ws = lddmm.workspace_size(lddmm.make_params(mid.n, mid.T, 1.5, 1.0, "fp32c"))
        assert ws < 4 << 20 < ws + 16 * 3 * mid.n * 8
        with pytest.raises(lddmm.LddmmError) as e:
            ctx.solve(to_dev(mid.q0), to_dev(mid.target), mid.T, mid.sigma, mid.lam, "fp32c",
                      max_iter=2)
        assert e.value.status == lddmm.ENOMEM
        g = run_grad(ctx, pb, "fp64")
        r = ctx.solve(to_dev(pb.q0), to_dev(pb.target), pb.T, pb.sigma, pb.lam, "fp64",
                      max_iter=3)
        torch.cuda.synchronize()
    o = orc.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, 4)
    check_grad(g, o, "fp64", "within budget")
    assert r["iters"] == 3


def test_nonfinite_input_is_flagged(gpu_ctx):
    import torch
    from paper_1907_04839_amd import lddmm
    pb = synth.random_problem(41, 100, T=3)
    x = pb.target.copy()
    x[5, 1] = np.nan
    gpu_ctx.shoot_grad(to_dev(pb.q0), to_dev(pb.p0), to_dev(x), 3, pb.sigma, pb.lam, "fp32c")
    with pytest.raises(lddmm.LddmmError) as e:
        gpu_ctx.check()
    assert e.value.status == lddmm.ENONFINITE
    assert gpu_ctx.check() == lddmm.OK      # flag cleared
    torch.cuda.synchronize()


# ----------------------------------------------------------------- gradients w.r.t. q0, target

@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,T,ckpt", [(1, 3, 0), (200, 5, 0), (2500, 6, 0), (900, 9, 4)])
def test_gradients_wrt_q0_and_target_match_oracle(gpu_ctx, orc_mt, mode, n, T, ckpt):
    import torch
    pb = synth.random_problem(500 + n, n, T=T)
    r = gpu_ctx.shoot_grad(to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), T, pb.sigma, pb.lam,
                           precision=mode, ckpt_every=ckpt, want_grad_q0=True, want_grad_x=True)
    torch.cuda.synchronize()
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, T, all_grads=True)
    eq, ex = row_err(host(r.grad_q0), o["grad_q0"]), row_err(host(r.grad_x), o["grad_x"])
    ep = row_err(host(r.grad), o["grad"])
    print(f"[grad_all n={n} T={T} ckpt={ckpt} {mode}] p0={ep:.2e} q0={eq:.2e} x={ex:.2e}",
          flush=True)
    assert max(eq, ex, ep) <= TOL[mode]
    # the p0-gradient is the same with or without the extra outputs
    r0 = gpu_ctx.shoot_grad(to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), T, pb.sigma, pb.lam,
                            precision=mode, ckpt_every=ckpt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(r0.grad), host(r.grad))


# ----------------------------------------------------------------- energy term at t = 1

@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,T,ckpt", [(1, 3, 0), (300, 5, 0), (2500, 6, 0), (900, 9, 4)])
def test_final_energy_variant_matches_oracle(gpu_ctx, orc_mt, mode, n, T, ckpt):
    import torch
    pb = synth.random_problem(1100 + n, n, T=T)
    r = gpu_ctx.shoot_grad(to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), T, pb.sigma, pb.lam,
                           precision=mode, ckpt_every=ckpt, want_grad_q0=True, want_grad_x=True,
                           energy="final")
    torch.cuda.synchronize()
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, T, all_grads=True,
                          energy="final")
    el = abs(r.loss.item() - o["loss"]) / abs(o["loss"])
    eh = abs(r.H0.item() - o["H0"]) / abs(o["H0"])
    eg = max(row_err(host(r.grad), o["grad"]), row_err(host(r.grad_q0), o["grad_q0"]),
             row_err(host(r.grad_x), o["grad_x"]))
    print(f"[energy final n={n} T={T} ckpt={ckpt} {mode}] loss={el:.2e} H={eh:.2e} "
          f"grads={eg:.2e}", flush=True)
    assert max(el, eh, eg) <= TOL[mode]


def test_final_energy_solve_reaches_scipy_minimum(gpu_ctx, orc):
    """On the 64-landmark box problem the GPU solver, minimising the loss with the
    energy at t = 1, reaches the minimum that scipy's L-BFGS-B finds on the
    oracle's variant loss and gradient (gradient norm 1e-6 there)."""
    import scipy.optimize as so
    import torch
    pb = synth.box_displacement()
    n = pb.n

    def f(v):
        r = orc.shoot_grad(pb.q0, v.reshape(n, 3), pb.target, pb.sigma, pb.lam, pb.T,
                           energy="final")
        return r["loss"], r["grad"].ravel()
    ref = so.minimize(f, np.zeros(3 * n), jac=True, method="L-BFGS-B",
                      options=dict(maxiter=500, gtol=1e-10, ftol=1e-15))
    q0, x = to_dev(pb.q0), to_dev(pb.target)
    r = gpu_ctx.solve(q0, x, pb.T, pb.sigma, pb.lam, "fp64", energy="final", max_iter=300,
                      gtol=1e-9)
    g = gpu_ctx.shoot_grad(q0, r["p0"], x, pb.T, pb.sigma, pb.lam, precision="fp64",
                           energy="final")
    torch.cuda.synchronize()
    q1_ref = orc.shoot_forward(pb.q0, ref.x.reshape(n, 3), pb.sigma, pb.T)["q1"]
    el = abs(r["loss"] - ref.fun) / ref.fun
    eq = rel_err(host(g.q1), q1_ref)
    print(f"[final-energy solve box64] loss {r['loss']:.10g} vs scipy {ref.fun:.10g} ({el:.1e}), "
          f"q1 {eq:.1e}, iters {r['iters']}", flush=True)
    assert abs(r["loss"] - g.loss.item()) <= 1e-12 * g.loss.item()
    assert el < 1e-9 and eq < 1e-6


def test_server_rejects_final_energy():
    import ctypes
    from paper_1907_04839_amd import lddmm
    pb = synth.random_problem(1160, 50, T=12)
    with lddmm.Server(12, "fp32c", max_slots=2, max_n=1024, hbm_budget_bytes=64 << 20) as s:
        prm = lddmm.make_params(pb.n, 12, pb.sigma, pb.lam, "fp32c", energy="final")
        o = lddmm.solve_opts("fp32c")
        jid = ctypes.c_int64(0)
        st = lddmm.lib().lddmm_server_submit(s._h, ctypes.byref(prm), ctypes.byref(o),
                                              pb.q0.ctypes.data, pb.target.ctypes.data, None,
                                              ctypes.byref(jid))
        assert st == lddmm.EINVAL


# ----------------------------------------------------------------- degenerate kernel widths, lambda = 0

@pytest.mark.parametrize("mode", MODES)
def test_tiny_sigma_decouples_every_landmark(gpu_ctx, mode):
    """sigma far below the spacing: every off-diagonal kernel value underflows to 0,
    each landmark moves alone in a straight line, q(1) = q0 + p0, and the gradient
    is the single-landmark closed form p0 + 2 lambda (q0 + p0 - x)."""
    import torch
    rng = np.random.default_rng(1300)
    n, T, lam = 3001, 7, 1.7
    q0 = 10.0 * rng.standard_normal((n, 3))
    p0 = 0.3 * rng.standard_normal((n, 3))
    x = q0 + 0.5 * rng.standard_normal((n, 3))
    r = gpu_ctx.shoot_grad(to_dev(q0), to_dev(p0), to_dev(x), T, 1e-3, lam, precision=mode)
    torch.cuda.synchronize()
    q1 = q0 + p0
    g = p0 + 2.0 * lam * (q1 - x)
    eq, eg = row_err(host(r.q1) - q0, p0), row_err(host(r.grad), g)
    print(f"[tiny sigma {mode}] q1 {eq:.2e} grad {eg:.2e}", flush=True)
    tol = 1e-13 if mode == "fp64" else 2e-7    # FP32 records hold p and a rounded to FP32
    assert eq < tol and eg < tol


@pytest.mark.parametrize("mode", MODES)
def test_huge_sigma_translates_the_cloud_rigidly(gpu_ctx, mode):
    """sigma far above the cloud: every kernel value is 1 (to 1e-12), Hp_i is the
    total momentum P and Hq vanishes, so every landmark moves by P."""
    import torch
    rng = np.random.default_rng(1301)
    n, T = 2000, 5
    q0 = rng.standard_normal((n, 3))
    p0 = 1e-3 * rng.standard_normal((n, 3))
    q1, p1, _ = gpu_ctx.shoot_forward(to_dev(q0), to_dev(p0), T, 1e6, precision=mode)
    torch.cuda.synchronize()
    P = p0.sum(0)
    e = np.abs(host(q1) - q0 - P[None, :]).max() / np.abs(P).max()
    print(f"[huge sigma {mode}] displacement error {e:.2e}", flush=True)
    assert e < (1e-9 if mode == "fp64" else 1e-5)
    np.testing.assert_allclose(host(p1), p0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("mode", MODES)
def test_zero_lambda_gradient_is_Hp0(gpu_ctx, orc_mt, mode):
    """lambda = 0: the terminal adjoint is 0 and stays 0, so dL/dp0 = Hp(q0, p0) and
    the loss is H(q0, p0)."""
    import torch
    pb = synth.random_problem(1302, 1500, T=4)
    r = gpu_ctx.shoot_grad(to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), 4, pb.sigma, 0.0,
                           precision=mode)
    torch.cuda.synchronize()
    _, Hp = orc_mt.pair_forward(pb.q0, pb.p0, pb.sigma)
    H = orc_mt.hamiltonian(pb.q0, pb.p0, pb.sigma)
    eg = row_err(host(r.grad), Hp)
    assert eg < TOL[mode] and abs(r.loss.item() - H) < TOL[mode] * H
    assert r.loss.item() == r.H0.item()


@pytest.mark.parametrize("mode", MODES)
def test_coincident_landmarks(gpu_ctx, orc_mt, mode):
    """Duplicated landmarks (same q0, p0 and target; the pair has Delta = 0 and
    g = 1 off the diagonal) match the oracle, and each copy's q(1) and gradient
    equal the original's bitwise: both see the same data in the same order."""
    rng = np.random.default_rng(1303)
    base = synth.random_problem(1303, 700, T=4)
    dup = rng.choice(700, size=130, replace=False)
    src = np.concatenate([np.arange(700), dup])
    perm = rng.permutation(src.size)       # copies land in other i-blocks and j-chunks
    idx = src[perm]
    q0, p0, x = (np.ascontiguousarray(a[idx]) for a in (base.q0, base.p0, base.target))
    pb = synth.Problem("coincident830", q0, x, p0, base.sigma, base.lam, base.T)
    g = run_grad(gpu_ctx, pb, mode)
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, pb.T)
    check_grad(g, o, mode, "coincident")
    pos = {}
    for k, s in enumerate(idx):
        pos.setdefault(int(s), []).append(k)
    pairs = [(v[0], v[1]) for v in pos.values() if len(v) == 2]
    assert len(pairs) == 130
    a, b = np.array(pairs).T
    assert np.array_equal(g["q1"][a], g["q1"][b])
    assert np.array_equal(g["grad"][a], g["grad"][b])
