import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def gpu_ctx():
    """A liblddmm context on cuda:0 (GPU tests only)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_04839_amd import lddmm
    ctx = lddmm.Context(0)
    yield ctx
    ctx.close()


@pytest.fixture(scope="session")
def orc_mt(orc):
    """The oracle with its rows spread over the host's cores (results do not
    depend on the thread count)."""
    orc.set_threads(min(16, os.cpu_count() or 1))
    return orc


def to_dev(a):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel_err(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def row_err(a, b):
    """Largest row error over the RMS row norm of the reference,
    max_i |a_i - b_i| / sqrt(mean_i |b_i|^2), for [N, k] outputs.  It is never
    smaller than rel_err, and an error confined to a few rows (one 64-landmark
    block, a ragged tail, one j-chunk's partial) is not diluted by the others.
    Like rel_err it never divides by a single near-zero component."""
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    a2, b2 = a.reshape(b.shape[0], -1), b.reshape(b.shape[0], -1)
    d = np.sqrt(((a2 - b2) ** 2).sum(axis=1)).max(initial=0.0)
    rms = np.sqrt((b2 ** 2).sum(axis=1).mean()) if b2.size else 0.0
    return float(d / max(rms, 1e-300))
