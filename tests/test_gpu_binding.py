"""The Python binding rejects tensors the C ABI cannot take (wrong device,
dtype, shape or layout) before anything reaches the GPU, and a context keeps
working after such an error."""
import numpy as np
import pytest

from paper_1907_04839_amd import synth

from conftest import to_dev

pytestmark = pytest.mark.gpu


def test_bad_tensors_are_rejected_before_any_call(gpu_ctx):
    import torch
    pb = synth.random_problem(11, 200, T=4)
    q0, p0, x = to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target)
    cases = {
        "host tensor": (q0.cpu(), TypeError),
        "float32": (q0.float(), ValueError),
        "wrong shape": (q0[:150], ValueError),
        "transposed": (q0.t().contiguous().t(), ValueError),
        "[N, 2]": (q0[:, :2].contiguous(), ValueError),
    }
    for name, (bad, err) in cases.items():
        with pytest.raises(err):
            gpu_ctx.shoot_grad(bad, p0, x, pb.T, pb.sigma, pb.lam)
        with pytest.raises(err):
            gpu_ctx.shoot_grad(q0, p0, bad, pb.T, pb.sigma, pb.lam)
        if name != "wrong shape":          # for the flow any number of points is valid
            with pytest.raises(err):
                gpu_ctx.flow(q0, p0, bad, pb.T, pb.sigma)
    r = gpu_ctx.shoot_grad(q0, p0, x, pb.T, pb.sigma, pb.lam, precision="fp64")
    torch.cuda.synchronize()
    assert np.isfinite(r.loss.item())
    gpu_ctx.check()
