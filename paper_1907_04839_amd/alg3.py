"""Python binding of liblddmm_alg3 (ctypes, argument marshalling only): the
materialised-matrix forward step of the paper's Sec. 2.4 (Alg. 3), an
ablation set beside the fused pair kernels of liblddmm.  Names mirror
``include/lddmm_alg3.h``."""
from __future__ import annotations

import ctypes
import os

import torch  # first: the library then binds to the HIP runtime torch has loaded

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblddmm_alg3.so")
_vp = ctypes.c_void_p
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (__graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.lddmm_alg3_create.argtypes = [ctypes.c_int, ctypes.POINTER(_vp)]
        L.lddmm_alg3_destroy.argtypes = [_vp]
        L.lddmm_alg3_workspace_bytes.argtypes = [ctypes.c_int32]
        L.lddmm_alg3_workspace_bytes.restype = ctypes.c_size_t
        L.lddmm_alg3_pair_forward.argtypes = [_vp, ctypes.c_int32, ctypes.c_double, _vp, _vp, _vp,
                                              _vp, _vp, ctypes.c_size_t, _vp]
        L.lddmm_alg3_last_error.argtypes = [_vp]
        L.lddmm_alg3_last_error.restype = ctypes.c_char_p
        for f in ("lddmm_alg3_create", "lddmm_alg3_destroy", "lddmm_alg3_pair_forward"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def workspace_bytes(n: int) -> int:
    return int(lib().lddmm_alg3_workspace_bytes(int(n)))


class Alg3:
    """rocBLAS handle on one GPU; ``pair_forward`` runs one materialised step."""

    def __init__(self, device: int = 0):
        h = _vp()
        rc = lib().lddmm_alg3_create(int(device), ctypes.byref(h))
        if rc != 0:
            raise RuntimeError(f"lddmm_alg3_create: {lib().lddmm_alg3_last_error(None).decode()}")
        self._h = h
        self.device = int(device)

    def close(self):
        if getattr(self, "_h", None):
            lib().lddmm_alg3_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def pair_forward(self, q: torch.Tensor, p: torch.Tensor, sigma: float,
                     ws: torch.Tensor | None = None, out=None, stream=None):
        """(Hq, Hp) at (q, p), [N,3] float64 CUDA tensors.  ws: a uint8 CUDA
        tensor of at least workspace_bytes(N) (None: allocated and freed inside
        the call, as the paper's listing does)."""
        n = q.shape[0]
        for name, t in (("q", q), ("p", p)):
            if not (t.is_cuda and t.dtype == torch.float64 and tuple(t.shape) == (n, 3)
                    and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 [{n}, 3] CUDA tensor")
        hq, hp = out if out is not None else (torch.empty_like(q), torch.empty_like(q))
        s = (torch.cuda.current_stream() if stream is None else stream).cuda_stream
        rc = lib().lddmm_alg3_pair_forward(
            self._h, n, float(sigma), q.data_ptr(), p.data_ptr(), hq.data_ptr(), hp.data_ptr(),
            ws.data_ptr() if ws is not None else None, ws.numel() if ws is not None else 0, s)
        if rc != 0:
            raise RuntimeError(f"lddmm_alg3_pair_forward ({rc}): "
                               f"{lib().lddmm_alg3_last_error(self._h).decode()}")
        return hq, hp
