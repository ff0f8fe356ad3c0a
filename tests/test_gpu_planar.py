"""Planar problems (lddmm_params.dim = 2): the specialised pair loops leave the
z terms out.  On inputs whose z components are all 0 every z term of the 3D
loops is an exact 0, so the planar path must give bitwise the 3D path's
results (up to the sign of zero), and both match the oracle."""
import numpy as np
import pytest

from paper_1907_04839_amd import synth

from conftest import assert_gates, point_errs, rel_err, row_err, to_dev

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32c", "fp32"]
TOL = {"fp64": 1e-12, "fp32c": 1e-5, "fp32": 1e-5}


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,T,ckpt", [(1, 3, 0), (300, 5, 0), (2500, 6, 0), (900, 9, 4),
                                      (9000, 2, 0)])
def test_planar_gradients_equal_3d_and_oracle(gpu_ctx, orc_mt, mode, n, T, ckpt):
    import torch
    pb = synth.planar(synth.random_problem(1200 + n, n, T=T))
    args = (to_dev(pb.q0), to_dev(pb.p0), to_dev(pb.target), T, pb.sigma, pb.lam)
    kw = dict(precision=mode, ckpt_every=ckpt, want_grad_q0=True, want_grad_x=True)
    r2 = gpu_ctx.shoot_grad(*args, dim=2, **kw)
    r3 = gpu_ctx.shoot_grad(*args, dim=3, **kw)
    torch.cuda.synchronize()
    for k in ("grad", "grad_q0", "grad_x", "q1"):
        np.testing.assert_array_equal(host(getattr(r2, k)), host(getattr(r3, k)), err_msg=k)
    assert r2.loss.item() == r3.loss.item() and r2.H0.item() == r3.H0.item()
    o = orc_mt.shoot_grad(pb.q0, pb.p0, pb.target, pb.sigma, pb.lam, T, all_grads=True)
    e = dict(loss=abs(r2.loss.item() - o["loss"]) / abs(o["loss"]),
             **point_errs("grad", host(r2.grad), o["grad"]),
             **point_errs("grad_q0", host(r2.grad_q0), o["grad_q0"]))
    print(f"[planar n={n} T={T} ckpt={ckpt} {mode}] vs oracle " +
          " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    assert_gates(e, mode, TOL[mode])
    for k in ("grad", "grad_q0", "q1"):
        assert not host(getattr(r2, k))[:, 2].any(), k


@pytest.mark.parametrize("mode", ["fp64", "fp32c"])
def test_planar_flow_and_velocity_equal_3d(gpu_ctx, mode):
    import torch
    pb = synth.planar(synth.random_problem(1250, 5000, T=6))
    rng = np.random.default_rng(1251)
    x = np.concatenate([4.0 * rng.standard_normal((3000, 2)), np.zeros((3000, 1))], axis=1)
    q0, p0, xd = to_dev(pb.q0), to_dev(pb.p0), to_dev(x)
    f2 = gpu_ctx.flow(q0, p0, xd, 6, pb.sigma, precision=mode, dim=2)
    f3 = gpu_ctx.flow(q0, p0, xd, 6, pb.sigma, precision=mode, dim=3)
    v2 = gpu_ctx.velocity(q0, p0, xd, pb.sigma, precision=mode, dim=2)
    v3 = gpu_ctx.velocity(q0, p0, xd, pb.sigma, precision=mode, dim=3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(f2), host(f3))
    np.testing.assert_array_equal(host(v2), host(v3))


def test_planar_solve_equals_3d(gpu_ctx):
    import torch
    pb = synth.ellipse_warp(n=700, T=10)
    q0, x = to_dev(pb.q0), to_dev(pb.target)
    a = gpu_ctx.solve(q0, x, pb.T, pb.sigma, pb.lam, "fp32c", dim=2, max_iter=15)
    b = gpu_ctx.solve(q0, x, pb.T, pb.sigma, pb.lam, "fp32c", dim=3, max_iter=15)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(a["p0"]), host(b["p0"]))
    assert a["loss"] == b["loss"] and a["iters"] == b["iters"] and a["fevals"] == b["fevals"]


def test_server_takes_planar_jobs_beside_3d_ones():
    """Planar jobs (dim = 2) in a server that also runs 3D jobs: each gives bitwise
    the result of the same job run as 3D (the z terms it leaves out are exact
    zeros), keeps every z component of p0 at 0, and in FP64 takes the iterates of
    lddmm_solve on the planar problem."""
    import torch
    from paper_1907_04839_amd import lddmm
    Tp, iters = 12, 8
    flat = [synth.planar(synth.random_problem(1260 + j, n, T=Tp))
            for j, n in enumerate([50, 700, 1300])]
    solid = [synth.random_problem(1270 + j, n, T=Tp) for j, n in enumerate([400, 900])]

    def serve(batch, precision="fp32c"):
        with lddmm.Server(Tp, precision, max_slots=8, max_n=2048,
                          hbm_budget_bytes=256 << 20) as s:
            ids = [s.submit(pb.q0, pb.target, pb.sigma, pb.lam, dim=d, max_iter=iters)
                   for pb, d in batch]
            return [s.result(i, timeout=120) for i in ids]

    mixed = serve([(pb, 2) for pb in flat] + [(pb, 3) for pb in solid])
    as_3d = serve([(pb, 3) for pb in flat])
    for pb, m, r in zip(flat, mixed, as_3d):
        print(f"[serve planar n={pb.n}] iters {m['iters']} loss {m['loss']:.6e}", flush=True)
        assert np.all(m["p0"][:, 2] == 0.0)
        np.testing.assert_array_equal(m["p0"], r["p0"])
        for k in ("loss", "H0", "mismatch", "iters", "fevals", "status"):
            assert m[k] == r[k], k
    alone = serve([(solid[1], 3)])[0]
    np.testing.assert_array_equal(mixed[-1]["p0"], alone["p0"])

    pb = flat[1]
    got = serve([(pb, 2)], "fp64")[0]
    with lddmm.Context(0) as ctx:
        ref = ctx.solve(to_dev(pb.q0), to_dev(pb.target), Tp, pb.sigma, pb.lam, "fp64", dim=2,
                        max_iter=iters)
        torch.cuda.synchronize()
    el = abs(got["loss"] - ref["loss"]) / ref["loss"]
    print(f"[serve planar fp64] iters {got['iters']}/{ref['iters']} loss {el:.2e}", flush=True)
    assert got["iters"] == ref["iters"] and el < 1e-10
    assert rel_err(got["p0"], host(ref["p0"])) < 1e-9


def test_server_rejects_an_unknown_dim():
    import ctypes
    from paper_1907_04839_amd import lddmm
    pb = synth.planar(synth.random_problem(1261, 50, T=12))
    with lddmm.Server(12, "fp32c", max_slots=2, max_n=1024, hbm_budget_bytes=64 << 20) as s:
        prm = lddmm.make_params(pb.n, 12, pb.sigma, pb.lam, "fp32c", dim=4)
        o = lddmm.solve_opts("fp32c")
        jid = ctypes.c_int64(0)
        st = lddmm.lib().lddmm_server_submit(s._h, ctypes.byref(prm), ctypes.byref(o),
                                              pb.q0.ctypes.data, pb.target.ctypes.data, None,
                                              ctypes.byref(jid))
        assert st == lddmm.EINVAL
