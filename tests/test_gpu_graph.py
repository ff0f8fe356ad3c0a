"""One loss+gradient evaluation captured in a hipGraph (torch.cuda.CUDAGraph on
the call's stream) and replayed: every replay, with eager work and
synchronisations between them, gives bitwise the eager result.  The context's
workspace must exist before capture (one eager call of the same shape), since
capture cannot allocate."""
import numpy as np
import pytest

from paper_1907_04839_amd import synth

from conftest import to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,ckpt,integ", [("fp32c", 0, "euler"), ("fp64", 3, "euler"),
                                             ("fp32c", 2, "rk4")])
def test_captured_evaluation_replays_bitwise(gpu_ctx, mode, ckpt, integ):
    import torch
    pb = synth.random_problem(1300, 900, T=7)
    q0, p0, x = to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target)
    out = dict(grad=torch.empty_like(q0),
               out3=torch.empty(3, dtype=torch.float64, device=q0.device))
    s = torch.cuda.Stream()

    def run():
        return gpu_ctx.shoot_grad(q0, p0, x, pb.T, pb.sigma, pb.lam, precision=mode,
                                  ckpt_every=ckpt, want_q1=False, out=out, stream=s,
                                  integrator=integ)
    with torch.cuda.stream(s):
        run()                                  # eager: sizes the workspace
    torch.cuda.synchronize()
    ref_g, ref_l = out["grad"].cpu().numpy(), out["out3"].cpu().numpy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        run()
    torch.cuda.synchronize()
    for k in range(3):
        out["grad"].zero_()
        out["out3"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out["grad"].cpu().numpy(), ref_g, err_msg=f"replay {k}")
        np.testing.assert_array_equal(out["out3"].cpu().numpy(), ref_l, err_msg=f"replay {k}")
        # eager work on the same context between replays
        with torch.cuda.stream(s):
            gpu_ctx.shoot_forward(q0, p0, 3, pb.sigma, precision=mode, stream=s)
        torch.cuda.synchronize()
