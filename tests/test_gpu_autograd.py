"""torch.autograd.Function over the hand-written adjoint: equal to the C-ABI
call, checked against finite differences and the oracle, and bitwise
unchanged when the trajectory is recomputed from checkpoints."""
import numpy as np
import pytest

from paper_1907_04839_amd import synth

from conftest import rel_err, row_err, to_dev

pytestmark = pytest.mark.gpu


def test_loss_and_grad_equal_the_c_abi_call(gpu_ctx):
    import torch
    from paper_1907_04839_amd.autograd import shoot_loss
    pb = synth.random_problem(301, 900, T=7)
    p0 = to_dev(pb.p0).requires_grad_(True)
    L = shoot_loss(p0, to_dev(pb.q0), to_dev(pb.target), pb.T, pb.sigma, pb.lam, "fp32c", 0)
    L.backward()
    r = gpu_ctx.shoot_grad(to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), pb.T, pb.sigma,
                           pb.lam, "fp32c")
    torch.cuda.synchronize()
    assert L.item() == r.loss.item()
    assert torch.equal(p0.grad, r.grad)


def test_backward_scales_by_the_incoming_gradient():
    import torch
    from paper_1907_04839_amd.autograd import shoot_loss
    pb = synth.random_problem(302, 100, T=3)
    p0 = to_dev(pb.p0).requires_grad_(True)
    L = shoot_loss(p0, to_dev(pb.q0), to_dev(pb.target), pb.T, pb.sigma, pb.lam, "fp64", 0)
    (3.5 * L).backward()
    g1 = p0.grad.clone()
    p0.grad = None
    shoot_loss(p0, to_dev(pb.q0), to_dev(pb.target), pb.T, pb.sigma, pb.lam, "fp64", 0).backward()
    torch.testing.assert_close(g1, 3.5 * p0.grad, rtol=1e-15, atol=0)


def test_fp64_gradient_matches_central_differences():
    import torch
    from paper_1907_04839_amd.autograd import shoot_loss
    pb = synth.random_problem(303, 40, T=5)
    q0, x = to_dev(pb.q0), to_dev(pb.target)
    p0 = to_dev(pb.p0).requires_grad_(True)
    shoot_loss(p0, q0, x, pb.T, pb.sigma, pb.lam, "fp64", 0).backward()
    g = p0.grad.detach().cpu().numpy()
    eps = 1e-6
    fd = np.zeros_like(g)
    base = to_dev(pb.p0)
    with torch.no_grad():
        for i in range(pb.n):
            for d in range(3):
                e = torch.zeros_like(base)
                e[i, d] = eps
                lp = shoot_loss(base + e, q0, x, pb.T, pb.sigma, pb.lam, "fp64", 0).item()
                lm = shoot_loss(base - e, q0, x, pb.T, pb.sigma, pb.lam, "fp64", 0).item()
                fd[i, d] = (lp - lm) / (2 * eps)
    err = rel_err(g, fd)
    print(f"[autograd FD n=40] {err:.2e}", flush=True)
    assert err < 1e-7


@pytest.mark.parametrize("mode,tol", [("fp64", 1e-12), ("fp32c", 1e-5)])
def test_sphere_subsample_T100_matches_oracle(orc_mt, mode, tol):
    """The 16384-landmark sphere workload's settings (sigma 6, T 100,
    checkpoints every 10 steps) on a seeded 512-landmark subsample."""
    import torch
    from paper_1907_04839_amd.autograd import shoot_loss
    pb = synth.subsample(synth.sphere_autograd(), 512)
    p0 = to_dev(pb.p0).requires_grad_(True)
    L = shoot_loss(p0, to_dev(pb.q0), to_dev(pb.target), pb.T, pb.sigma, pb.lam, mode, 10)
    L.backward()
    torch.cuda.synchronize()
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, pb.T)
    el = abs(L.item() - o["loss"]) / abs(o["loss"])
    eg = row_err(p0.grad.cpu().numpy(), o["grad"])
    print(f"[autograd sphere512 T=100 {mode}] loss={el:.2e} grad={eg:.2e}", flush=True)
    assert el <= tol and eg <= tol


def test_automatic_checkpointing_is_bitwise_identical():
    import torch
    from paper_1907_04839_amd.autograd import ShootConfig, ShootLoss
    pb = synth.random_problem(304, 2000, T=30)
    q0, x = to_dev(pb.q0), to_dev(pb.target)
    grads = []
    for budget in (1 << 34, 200_000):        # everything fits / only a ring of ~6 records fits
        cfg = ShootConfig(pb.T, pb.sigma, pb.lam, "fp32c", "auto", budget)
        p0 = to_dev(pb.p0).requires_grad_(True)
        ShootLoss.apply(p0, q0, x, cfg).backward()
        grads.append(p0.grad.clone())
    assert ShootConfig(pb.T, pb.sigma, pb.lam, "fp32c", "auto", 200_000).resolve_ckpt(pb.n) > 0
    torch.cuda.synchronize()
    assert torch.equal(grads[0], grads[1])


def test_torch_optimizer_drives_the_loss_down():
    import torch
    from paper_1907_04839_amd.autograd import shoot_loss
    pb = synth.box_displacement()
    q0, x = to_dev(pb.q0), to_dev(pb.target)
    p0 = torch.zeros_like(q0, requires_grad=True)
    opt = torch.optim.LBFGS([p0], max_iter=20, line_search_fn="strong_wolfe")

    def closure():
        opt.zero_grad()
        L = shoot_loss(p0, q0, x, pb.T, pb.sigma, pb.lam, "fp64", 0)
        L.backward()
        return L

    L0 = closure().item()
    opt.step(closure)
    L1 = shoot_loss(p0, q0, x, pb.T, pb.sigma, pb.lam, "fp64", 0).item()
    assert L1 < 0.5 * L0


def test_template_and_target_gradients_through_autograd(orc_mt):
    import torch
    from paper_1907_04839_amd.autograd import shoot_loss
    pb = synth.random_problem(305, 300, T=6)
    p0 = to_dev(pb.p0).requires_grad_(True)
    q0 = to_dev(pb.q0).requires_grad_(True)
    x = to_dev(pb.target).requires_grad_(True)
    shoot_loss(p0, q0, x, pb.T, pb.sigma, pb.lam, "fp64", 0).backward()
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, pb.T, all_grads=True)
    assert row_err(p0.grad.cpu().numpy(), o["grad"]) < 1e-12
    assert row_err(q0.grad.cpu().numpy(), o["grad_q0"]) < 1e-12
    assert row_err(x.grad.cpu().numpy(), o["grad_x"]) < 1e-12
    # translation identity on the device result
    tot = (q0.grad.sum(0) + x.grad.sum(0)).abs().max().item()
    assert tot < 1e-10 * q0.grad.abs().sum().item()


def test_sphere16384_directional_derivatives_match_fp64_differences(gpu_ctx):
    """The full 16384-landmark sphere workload (T = 100, checkpoints every 10): the
    gradient from torch.autograd through the hand-written adjoint, in FP64 and in
    compensated FP32, against central differences of the FP64 loss (eps 1e-4) in 64
    seeded random unit directions d.  Gated normwise over the 64 directions and per
    direction, each error over the RMS of the 64 differences."""
    import torch
    from paper_1907_04839_amd.autograd import shoot_loss
    pb = synth.sphere_autograd()
    q0, x = to_dev(pb.q0), to_dev(pb.target)

    def grad(mode):
        p0 = to_dev(pb.p0).requires_grad_(True)
        shoot_loss(p0, q0, x, pb.T, pb.sigma, pb.lam, mode, 10).backward()
        return p0.grad.detach()
    g = {"fp64": grad("fp64"), "fp32c": grad("fp32c")}
    p0 = to_dev(pb.p0)
    loss = lambda p: gpu_ctx.shoot_grad(q0, p, x, pb.T, pb.sigma, pb.lam,  # noqa: E731
                                        precision="fp64", ckpt_every=10, want_q1=False).loss.item()
    rng = np.random.default_rng(1400)
    eps = 1e-4
    fd, gd = [], {m: [] for m in g}
    for k in range(64):
        d = rng.standard_normal(pb.p0.shape)
        d = to_dev(d / np.linalg.norm(d))
        fd.append((loss(p0 + eps * d) - loss(p0 - eps * d)) / (2 * eps))
        for m in g:
            gd[m].append(float((g[m] * d).sum()))
        if k % 16 == 15:
            print(f"[sphere16384 directional FD] {k + 1} directions", flush=True)
    torch.cuda.synchronize()
    fd = np.array(fd)
    rms = float(np.sqrt(np.mean(fd ** 2)))
    errs = {}
    for m in g:
        v = np.array(gd[m])
        errs[m] = (float(np.linalg.norm(v - fd) / np.linalg.norm(fd)),
                   float(np.abs(v - fd).max() / rms))
    print("[sphere16384 directional FD, 64 directions] " +
          " ".join(f"{m}: normwise {a:.2e} worst/rms {b:.2e}" for m, (a, b) in errs.items()),
          flush=True)
    assert max(errs["fp64"]) < 1e-6
    assert errs["fp32c"][0] < 1e-5 and errs["fp32c"][1] < 1e-4
