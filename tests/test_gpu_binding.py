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


def test_timed_launches_give_the_same_results(gpu_ctx):
    """Launches with timing events (hipExtLaunchKernel) compute exactly what the
    untimed launches do, and the timer counts one forward and one adjoint
    pair-kernel launch per step and one flow launch per call."""
    import torch
    pb = synth.random_problem(12, 700, T=5)
    q0, p0, x = to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target)
    pts = to_dev(synth.random_problem(13, 300, T=1).q0)
    res = {}
    gpu_ctx.timing(reset=True)
    for timed in (False, True):
        gpu_ctx.set_timing(timed)
        try:
            r = gpu_ctx.shoot_grad(q0, p0, x, pb.T, pb.sigma, pb.lam, precision="fp32c")
            x1 = gpu_ctx.flow(q0, p0, pts, pb.T, pb.sigma, precision="fp32c")
            torch.cuda.synchronize()
            res[timed] = (r.loss.item(), r.grad.cpu().numpy(), x1.cpu().numpy())
        finally:
            gpu_ctx.set_timing(False)
    t = gpu_ctx.timing(reset=True)
    assert res[True][0] == res[False][0]
    assert np.array_equal(res[True][1], res[False][1])
    assert np.array_equal(res[True][2], res[False][2])
    # the flow call runs its own forward pass: 2 T forward launches in all
    assert t["fwd_launches"] == 2 * pb.T and t["adj_launches"] == pb.T
    assert t["flow_launches"] == 1
    for k in ("fwd_ms", "adj_ms", "flow_ms"):
        assert 0.0 < t[k] < 1000.0, (k, t[k])
    assert gpu_ctx.timing(reset=True)["fwd_launches"] == 0
