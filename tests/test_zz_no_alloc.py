"""lddmm_shoot_grad_noalloc (the entry point that allocates nothing) against
lddmm_shoot_grad: same loss, H(q0,p0), mismatch, q(1) and dL/dp0, bitwise,
on two calls in a row (the second on a smaller problem, in the scratch the
first one left behind), and its size limit checked before anything runs."""
import numpy as np
import pytest

from paper_1907_04839_amd import synth

from conftest import to_dev

pytestmark = pytest.mark.gpu


def _pair(ctx, pb, mode, ckpt=0):
    import torch
    q0, p0, x = to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target)
    ref = ctx.shoot_grad(q0, p0, x, pb.T, pb.sigma, pb.lam, precision=mode, ckpt_every=ckpt)
    grad = torch.full_like(q0, float("nan"))
    out3 = torch.full((3,), float("nan"), dtype=torch.float64, device=q0.device)
    q1 = torch.full_like(q0, float("nan"))
    ctx.shoot_grad_noalloc(q0, p0, x, pb.T, pb.sigma, pb.lam, grad, out3, q1, precision=mode,
                           ckpt_every=ckpt)
    torch.cuda.synchronize()
    return ({"out3": torch.stack([ref.loss, ref.H0, ref.mismatch]).cpu().numpy(),
             "grad": ref.grad.cpu().numpy(), "q1": ref.q1.cpu().numpy()},
            {"out3": out3.cpu().numpy(), "grad": grad.cpu().numpy(), "q1": q1.cpu().numpy()})


@pytest.mark.parametrize("mode", ["fp32c", "fp64", "fp32"])
def test_noalloc_matches_shoot_grad_two_calls(gpu_ctx, mode):
    # 3001 landmarks: 47 i-blocks with a ragged tail of 57, several j-chunks;
    # then 700 landmarks in the same scratch
    for n, T, seed in ((3001, 6, 7101), (700, 4, 7102)):
        pb = synth.random_problem(seed, n, T=T)
        ref, got = _pair(gpu_ctx, pb, mode)
        print(f"[noalloc {mode} n={n} T={T}] loss {got['out3'][0]:.17g}", flush=True)
        for k in ("out3", "grad", "q1"):
            assert np.all(np.isfinite(got[k])), (mode, n, k)
            assert np.array_equal(got[k], ref[k]), (mode, n, k)


def test_noalloc_with_checkpoints(gpu_ctx):
    pb = synth.random_problem(7103, 1500, T=12)
    ref, got = _pair(gpu_ctx, pb, "fp32c", ckpt=4)
    for k in ("out3", "grad", "q1"):
        assert np.array_equal(got[k], ref[k]), k


def test_noalloc_rejects_problems_beyond_the_scratch(gpu_ctx):
    import torch
    from paper_1907_04839_amd import lddmm
    n, T = 65536, 50   # whole trajectory: about 126 MiB of workspace
    assert lddmm.workspace_size(lddmm.make_params(n, T, 5.0, 1.0, "fp32c")) > 64 << 20
    z = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    g = torch.empty_like(z)
    o = torch.empty(3, dtype=torch.float64, device="cuda")
    with pytest.raises(lddmm.LddmmError) as e:
        gpu_ctx.shoot_grad_noalloc(z, z, z, T, 5.0, 1.0, g, o, precision="fp32c")
    assert e.value.status == lddmm.ENOMEM
    assert "fixed scratch" in str(e.value)
    # the context still works afterwards
    pb = synth.random_problem(7104, 200, T=3)
    ref, got = _pair(gpu_ctx, pb, "fp32c")
    assert np.array_equal(got["grad"], ref["grad"])
