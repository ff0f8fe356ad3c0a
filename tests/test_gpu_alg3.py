"""The materialised-matrix forward step (Sec. 2.4, Alg. 3: N x N term
matrices summed by rocBLAS sgemv) against the FP64 oracle's pair sums of
eq. 2, at the paper's landmark count (1847) and a small ragged case, with the
workspace passed in and allocated inside the call."""
import numpy as np
import pytest

from paper_1907_04839_amd import synth

from conftest import rel_err, row_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,own_ws", [(1847, True), (1847, False), (300, True), (1, True)])
def test_alg3_pair_forward_matches_oracle(orc, n, own_ws):
    import torch
    from paper_1907_04839_amd import alg3
    pb = synth.ellipsoid_warp(n=n, T=40, iters=1) if n > 1 else synth.random_problem(7, 1)
    p = 0.5 * (pb.target - pb.q0) + 0.1 * np.random.default_rng(n).standard_normal((n, 3))
    ref_hq, ref_hp = orc.pair_forward(pb.q0, p, pb.sigma)
    ws = torch.empty(alg3.workspace_bytes(n), dtype=torch.uint8, device="cuda") if own_ws else None
    with alg3.Alg3(0) as a:
        hq, hp = a.pair_forward(to_dev(pb.q0), to_dev(p), pb.sigma, ws=ws)
        torch.cuda.synchronize()
    hq, hp = hq.cpu().numpy(), hp.cpu().numpy()
    e = dict(hp=rel_err(hp, ref_hp), hp_row=row_err(hp, ref_hp),
             hq=rel_err(hq, ref_hq), hq_row=row_err(hq, ref_hq))
    print(f"[alg3 n={n} ws={'caller' if own_ws else 'own'}] " +
          " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    assert max(e.values()) <= 1e-5, e


def test_alg3_rejects_bad_arguments_on_the_host():
    import torch
    from paper_1907_04839_amd import alg3
    z = torch.zeros((8, 3), dtype=torch.float64, device="cuda")
    with alg3.Alg3(0) as a:
        with pytest.raises(RuntimeError, match="sigma"):
            a.pair_forward(z, z, 0.0)
        small = torch.empty(16, dtype=torch.uint8, device="cuda")
        with pytest.raises(RuntimeError, match="workspace"):
            a.pair_forward(z, z, 1.0, ws=small)
