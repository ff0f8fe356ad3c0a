"""Python binding of liblddmm (ctypes): argument marshalling only.

Every step of the computation runs in the HIP kernels of ``liblddmm.so``;
PyTorch provides device memory and the current stream.  There is no CPU
fallback: if the library or a GPU is missing, calls raise.

Names mirror ``include/lddmm.h``.  Point sets are float64 CUDA tensors of
shape [N, 3] (contiguous).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # first: liblddmm then binds to the HIP runtime torch has loaded

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblddmm.so")

OK, ENOTCONV, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EBUSY = 0, 1, -1, -2, -3, -4, -5
FP32, FP32_COMP, FP64 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "fp32c": FP32_COMP, "fp64": FP64}

_vp = ctypes.c_void_p


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("T", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("precision", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("energy", ctypes.c_int32),
                ("dim", ctypes.c_int32), ("integrator", ctypes.c_int32)]


class Timing(ctypes.Structure):
    _fields_ = [("fwd_ms", ctypes.c_double), ("adj_ms", ctypes.c_double),
                ("fwd_launches", ctypes.c_int64), ("adj_launches", ctypes.c_int64),
                ("flow_ms", ctypes.c_double), ("flow_launches", ctypes.c_int64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("m", ctypes.c_int32), ("max_fev", ctypes.c_int32),
                ("gtol", ctypes.c_double), ("ftol_rel", ctypes.c_double),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double), ("init", ctypes.c_int32)]


class SolveResult(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_double), ("H0", ctypes.c_double),
                ("mismatch", ctypes.c_double), ("grad_norm", ctypes.c_double),
                ("avg_dist", ctypes.c_double), ("max_dist", ctypes.c_double),
                ("iters", ctypes.c_int32), ("fevals", ctypes.c_int32), ("status", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("max_n", ctypes.c_int32), ("T", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_size_t), ("integrator", ctypes.c_int32)]


class JobTimes(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("done_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("job_evaluations", ctypes.c_int64), ("hbm_used_bytes", ctypes.c_size_t),
                ("hbm_budget_bytes", ctypes.c_size_t)]


class LddmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load liblddmm.so (built in-tree by ``paper_1907_04839_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m "
                               "paper_1907_04839_amd.build or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.lddmm_ctx_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_vp)]
        L.lddmm_ctx_destroy.argtypes = [_vp]
        L.lddmm_workspace_size.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]
        L.lddmm_shoot_forward.argtypes = [_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _vp]
        L.lddmm_shoot_grad.argtypes = [_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.lddmm_shoot_grad_noalloc.argtypes = [_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp,
                                               _vp, _vp, _vp]
        L.lddmm_shoot_grad_all.argtypes = [_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _vp,
                                           _vp, _vp, _vp]
        L.lddmm_velocity.argtypes = [_vp, ctypes.POINTER(Params), _vp, _vp, ctypes.c_int32, _vp,
                                     _vp, _vp]
        L.lddmm_flow.argtypes = [_vp, ctypes.POINTER(Params), _vp, _vp, ctypes.c_int32, _vp, _vp,
                                 _vp, _vp, _vp]
        L.lddmm_ctx_check.argtypes = [_vp, _vp]
        L.lddmm_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]
        L.lddmm_server_job_footprint.argtypes = [ctypes.POINTER(ServerConfig), ctypes.c_int32,
                                                 ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.lddmm_server_submit.argtypes = [_vp, ctypes.POINTER(Params), ctypes.POINTER(SolveOpts),
                                          _vp, _vp, _vp, ctypes.POINTER(ctypes.c_int64)]
        L.lddmm_server_poll.argtypes = [_vp, ctypes.c_int64, _vp, ctypes.POINTER(SolveResult),
                                        ctypes.POINTER(JobTimes)]
        L.lddmm_server_wait.argtypes = [_vp, ctypes.c_int64, ctypes.c_double]
        L.lddmm_server_stats_get.argtypes = [_vp, ctypes.POINTER(ServerStats)]
        L.lddmm_server_last_error.argtypes = [_vp]
        L.lddmm_server_last_error.restype = ctypes.c_char_p
        L.lddmm_server_destroy.argtypes = [_vp]
        L.lddmm_solve_opts_default.argtypes = [ctypes.c_int32, ctypes.POINTER(SolveOpts)]
        L.lddmm_solve.argtypes = [_vp, ctypes.POINTER(Params), ctypes.POINTER(SolveOpts), _vp, _vp,
                                  _vp, ctypes.POINTER(SolveResult), _vp, _vp]
        L.lddmm_ctx_set_timing.argtypes = [_vp, ctypes.c_int]
        L.lddmm_ctx_timing.argtypes = [_vp, ctypes.POINTER(Timing), ctypes.c_int]
        L.lddmm_status_string.argtypes = [ctypes.c_int]
        L.lddmm_status_string.restype = ctypes.c_char_p
        L.lddmm_last_error.argtypes = [_vp]
        L.lddmm_last_error.restype = ctypes.c_char_p
        L.lddmm_version.restype = ctypes.c_char_p
        for f in ("lddmm_ctx_create", "lddmm_ctx_destroy", "lddmm_workspace_size",
                  "lddmm_shoot_forward", "lddmm_shoot_grad", "lddmm_shoot_grad_noalloc",
                  "lddmm_shoot_grad_all",
                  "lddmm_velocity", "lddmm_flow",
                  "lddmm_ctx_check",
                  "lddmm_ctx_set_timing", "lddmm_ctx_timing", "lddmm_solve_opts_default",
                  "lddmm_solve", "lddmm_server_create", "lddmm_server_job_footprint",
                  "lddmm_server_submit", "lddmm_server_poll", "lddmm_server_wait",
                  "lddmm_server_stats_get", "lddmm_server_destroy"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, ctx=None, allow=(OK,)) -> int:
    if rc in allow:
        return rc
    L = lib()
    detail = L.lddmm_last_error(ctx).decode() or L.lddmm_status_string(rc).decode()
    raise LddmmError(rc, detail)


ENERGIES = {"initial": 0, "final": 1}
INTEGRATORS = {"euler": 0, "rk4": 1}


def make_params(n: int, T: int, sigma: float, lam: float, precision="fp32c",
                ckpt_every: int = 0, energy="initial", dim: int = 3,
                integrator="euler") -> Params:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    en = ENERGIES[energy] if isinstance(energy, str) else int(energy)
    it = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    return Params(int(n), int(T), float(sigma), float(lam), prec, int(ckpt_every), en, int(dim),
                  it)


def solve_opts(precision="fp32c", **overrides) -> SolveOpts:
    """Library defaults for ``precision``, with fields overridden by keyword."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o = SolveOpts()
    _check(lib().lddmm_solve_opts_default(prec, ctypes.byref(o)))
    for k, v in overrides.items():
        if k not in dict(SolveOpts._fields_):
            raise TypeError(f"unknown solver option {k}")
        setattr(o, k, v)
    return o


def workspace_size(params: Params) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().lddmm_workspace_size(ctypes.byref(params), ctypes.byref(b)))
    return int(b.value)


def _pts(t: torch.Tensor, name: str, n: int) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64 or tuple(t.shape) != (n, 3) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 [{n}, 3] tensor")
    return t.data_ptr()


def _stream(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


@dataclass
class GradResult:
    loss: torch.Tensor       # device scalar
    H0: torch.Tensor         # device scalar
    mismatch: torch.Tensor   # device scalar, sum |q(1) - x|^2
    grad: torch.Tensor       # [N,3] dL/dp0
    q1: torch.Tensor | None
    grad_q0: torch.Tensor | None = None   # [N,3] dL/dq0
    grad_x: torch.Tensor | None = None    # [N,3] dL/dtarget


class Context:
    """One GPU and its reusable device workspace (``lddmm_ctx``).

    hbm_budget_bytes caps the context's workspaces (0: no cap); a call that
    would need more raises LddmmError with status ENOMEM."""

    def __init__(self, device: int | None = None, hbm_budget_bytes: int = 0):
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = _vp()
        _check(lib().lddmm_ctx_create(self.device, int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def _pts(self, t: torch.Tensor, name: str, n: int) -> int:
        ptr = _pts(t, name, n)
        if t.device.index != self.device:
            raise ValueError(f"{name} is on cuda:{t.device.index}, the context on cuda:{self.device}")
        return ptr

    def close(self):
        if getattr(self, "_h", None):
            lib().lddmm_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- calls -------------------------------------------------------------
    def shoot_forward(self, q0: torch.Tensor, p0: torch.Tensor, T: int, sigma: float,
                      precision="fp32c", stream=None, dim: int = 3, integrator="euler"):
        """Forward flow in T Euler steps (Alg. 1 forward loop) or, with
        integrator="rk4", T classical Runge-Kutta steps.  Returns (q1, p1, H0)."""
        n = q0.shape[0]
        prm = make_params(n, T, sigma, 0.0, precision, dim=dim, integrator=integrator)
        q1 = torch.empty_like(q0)
        p1 = torch.empty_like(q0)
        H0 = torch.empty((), dtype=torch.float64, device=q0.device)
        _check(lib().lddmm_shoot_forward(self._h, ctypes.byref(prm), self._pts(q0, "q0", n),
                                         self._pts(p0, "p0", n), q1.data_ptr(), p1.data_ptr(),
                                         H0.data_ptr(), _stream(stream)), self._h)
        return q1, p1, H0

    def velocity(self, q: torch.Tensor, p: torch.Tensor, x: torch.Tensor, sigma: float,
                 precision="fp32c", stream=None, out: torch.Tensor | None = None,
                 dim: int = 3) -> torch.Tensor:
        """Velocity field of eq. 4 at the points x [M,3] for the landmark state (q, p)."""
        n, m = q.shape[0], x.shape[0]
        prm = make_params(n, 1, sigma, 0.0, precision, dim=dim)
        v = torch.empty_like(x) if out is None else out
        _check(lib().lddmm_velocity(self._h, ctypes.byref(prm), self._pts(q, "q", n), self._pts(p, "p", n),
                                    m, self._pts(x, "x", m), self._pts(v, "v", m), _stream(stream)),
               self._h)
        return v

    def flow(self, q0: torch.Tensor, p0: torch.Tensor, x0: torch.Tensor, T: int, sigma: float,
             precision="fp32c", ckpt_every: int = 0, want_landmarks: bool = False, stream=None,
             out: torch.Tensor | None = None, dim: int = 3, integrator="euler"):
        """Points x0 [M,3] carried along the landmark motion from (q0, p0) (eq. 4).

        Returns x1, or (x1, q1, p1) with ``want_landmarks``.  ``out`` may be x0
        itself (in place)."""
        n, m = q0.shape[0], x0.shape[0]
        prm = make_params(n, T, sigma, 0.0, precision, ckpt_every, dim=dim, integrator=integrator)
        x1 = torch.empty_like(x0) if out is None else out
        q1 = torch.empty_like(q0) if want_landmarks else None
        p1 = torch.empty_like(q0) if want_landmarks else None
        _check(lib().lddmm_flow(self._h, ctypes.byref(prm), self._pts(q0, "q0", n), self._pts(p0, "p0", n),
                                m, self._pts(x0, "x0", m), self._pts(x1, "x1", m),
                                q1.data_ptr() if q1 is not None else None,
                                p1.data_ptr() if p1 is not None else None, _stream(stream)),
               self._h)
        return (x1, q1, p1) if want_landmarks else x1

    def shoot_grad(self, q0: torch.Tensor, p0: torch.Tensor, target: torch.Tensor, T: int,
                   sigma: float, lam: float, precision="fp32c", ckpt_every: int = 0,
                   want_q1: bool = True, stream=None, out: dict | None = None,
                   want_grad_q0: bool = False, want_grad_x: bool = False,
                   energy="initial", dim: int = 3, integrator="euler") -> GradResult:
        """Loss of eq. 3 and its gradient w.r.t. p0 (Alg. 1 ComputeGradient);
        optionally also w.r.t. q0 and the target (lddmm_shoot_grad_all).

        ``out`` may hold preallocated ``grad`` [N,3], ``out3`` [3] and ``q1``.
        """
        n = q0.shape[0]
        prm = make_params(n, T, sigma, lam, precision, ckpt_every, energy, dim, integrator)
        out = out or {}
        grad = out.get("grad")
        if grad is None:
            grad = torch.empty_like(q0)
        out3 = out.get("out3")
        if out3 is None:
            out3 = torch.empty(3, dtype=torch.float64, device=q0.device)
        q1 = out.get("q1") if want_q1 else None
        if want_q1 and q1 is None:
            q1 = torch.empty_like(q0)
        if want_grad_q0 or want_grad_x:
            gq = torch.empty_like(q0) if want_grad_q0 else None
            gx = torch.empty_like(q0) if want_grad_x else None
            _check(lib().lddmm_shoot_grad_all(
                self._h, ctypes.byref(prm), self._pts(q0, "q0", n), self._pts(p0, "p0", n),
                self._pts(target, "target", n), out3.data_ptr(), self._pts(grad, "grad", n),
                gq.data_ptr() if gq is not None else None,
                gx.data_ptr() if gx is not None else None,
                q1.data_ptr() if q1 is not None else None, _stream(stream)), self._h)
            return GradResult(out3[0], out3[1], out3[2], grad, q1, gq, gx)
        _check(lib().lddmm_shoot_grad(self._h, ctypes.byref(prm), self._pts(q0, "q0", n),
                                      self._pts(p0, "p0", n), self._pts(target, "target", n),
                                      out3.data_ptr(), self._pts(grad, "grad", n),
                                      q1.data_ptr() if q1 is not None else None,
                                      _stream(stream)), self._h)
        return GradResult(out3[0], out3[1], out3[2], grad, q1)

    def shoot_grad_noalloc(self, q0: torch.Tensor, p0: torch.Tensor, target: torch.Tensor,
                           T: int, sigma: float, lam: float, grad: torch.Tensor,
                           out3: torch.Tensor, q1: torch.Tensor | None = None,
                           precision="fp32c", ckpt_every: int = 0, stream=None,
                           energy="initial", dim: int = 3, integrator="euler") -> None:
        """lddmm_shoot_grad_noalloc: the loss and dL/dp0 of shoot_grad into the
        caller's grad [N,3], out3 [3] (and q1), with the library's fixed device
        scratch as the workspace (the library allocates nothing)."""
        n = q0.shape[0]
        prm = make_params(n, T, sigma, lam, precision, ckpt_every, energy, dim, integrator)
        if out3.dtype != torch.float64 or out3.numel() < 3 or not out3.is_cuda:
            raise ValueError("out3 must be a float64 CUDA tensor of at least 3 elements")
        _check(lib().lddmm_shoot_grad_noalloc(
            self._h, ctypes.byref(prm), self._pts(q0, "q0", n), self._pts(p0, "p0", n),
            self._pts(target, "target", n), out3.data_ptr(), self._pts(grad, "grad", n),
            self._pts(q1, "q1", n) if q1 is not None else None, _stream(stream)), self._h)

    def solve(self, q0: torch.Tensor, target: torch.Tensor, T: int, sigma: float, lam: float,
              precision="fp32c", p0: torch.Tensor | None = None, ckpt_every: int = 0,
              want_trace: bool = False, stream=None, energy="initial", dim: int = 3,
              integrator="euler",
              **opts) -> dict:
        """L-BFGS registration on the GPU (Alg. 1).  ``opts`` override the
        library defaults (max_iter, m, max_fev, gtol, ftol_rel, c1, c2, init);
        passing ``p0`` selects init = 2 (start from it)."""
        import numpy as np
        n = q0.shape[0]
        prm = make_params(n, T, sigma, lam, precision, ckpt_every, energy, dim, integrator)
        if p0 is not None:
            opts.setdefault("init", 2)
        o = solve_opts(precision, **opts)
        out = torch.empty_like(q0) if p0 is None else p0.detach().clone().contiguous()
        res = SolveResult()
        tr = np.full(2 * (o.max_iter + 1), np.nan) if want_trace else None
        rc = lib().lddmm_solve(self._h, ctypes.byref(prm), ctypes.byref(o), self._pts(q0, "q0", n),
                               self._pts(target, "target", n), self._pts(out, "p0", n), ctypes.byref(res),
                               tr.ctypes.data if tr is not None else None, _stream(stream))
        _check(rc, self._h, allow=(OK, ENOTCONV))
        r = {k: getattr(res, k) for k, _ in SolveResult._fields_}
        r["p0"] = out
        if tr is not None:
            r["trace"] = tr.reshape(-1, 2)[: res.iters + 1]
        return r

    def set_timing(self, enable: bool) -> None:
        """Time every pair-kernel and point-flow launch with HIP events tied to the kernel."""
        _check(lib().lddmm_ctx_set_timing(self._h, int(bool(enable))), self._h)

    def timing(self, reset: bool = True) -> dict:
        """Summed pair-kernel durations (ms) and launch counts since the last reset."""
        t = Timing()
        _check(lib().lddmm_ctx_timing(self._h, ctypes.byref(t), int(bool(reset))), self._h)
        return dict(fwd_ms=t.fwd_ms, adj_ms=t.adj_ms, fwd_launches=int(t.fwd_launches),
                    adj_launches=int(t.adj_launches), flow_ms=t.flow_ms,
                    flow_launches=int(t.flow_launches))

    def check(self, stream=None) -> int:
        """Synchronise and report a non-finite loss since the last check."""
        return _check(lib().lddmm_ctx_check(self._h, _stream(stream)), self._h)


def server_config(T: int, precision="fp32c", max_slots: int = 32, max_n: int = 8192,
                  hbm_budget_bytes: int = 1 << 30, device: int = 0,
                  integrator="euler") -> ServerConfig:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    it = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    return ServerConfig(int(device), int(max_slots), int(max_n), int(T), prec,
                        int(hbm_budget_bytes), it)


def job_footprint(cfg: ServerConfig, n: int, m: int = 5) -> int:
    """Device bytes one job occupies in a server (host computation)."""
    b = ctypes.c_size_t(0)
    _check(lib().lddmm_server_job_footprint(ctypes.byref(cfg), int(n), int(m), ctypes.byref(b)))
    return int(b.value)


class Server:
    """Continuous-batching registration server (``lddmm_server``).  Inputs
    are host float64 [N,3] arrays; results come back as numpy arrays."""

    def __init__(self, T: int, precision="fp32c", max_slots: int = 32, max_n: int = 8192,
                 hbm_budget_bytes: int = 1 << 30, device: int = 0, integrator="euler"):
        self.cfg = server_config(T, precision, max_slots, max_n, hbm_budget_bytes, device,
                                 integrator)
        self.precision = precision
        h = _vp()
        rc = lib().lddmm_server_create(ctypes.byref(self.cfg), ctypes.byref(h))
        if rc != OK:
            raise LddmmError(rc, lib().lddmm_server_last_error(None).decode())
        self._h = h
        self._n = {}

    def _err(self, rc):
        raise LddmmError(rc, lib().lddmm_server_last_error(self._h).decode()
                         or lib().lddmm_status_string(rc).decode())

    def submit(self, q0, target, sigma: float, lam: float, p0=None, dim: int = 3,
               **opts) -> int:
        """Queue one registration; ``dim=2`` for a planar job (every z is 0)."""
        import numpy as np
        q0 = np.ascontiguousarray(q0, dtype=np.float64)
        target = np.ascontiguousarray(target, dtype=np.float64)
        n = q0.shape[0]
        prm = make_params(n, self.cfg.T, sigma, lam, self.cfg.precision, dim=dim,
                          integrator=self.cfg.integrator)
        if p0 is not None:
            opts.setdefault("init", 2)
            p0 = np.ascontiguousarray(p0, dtype=np.float64)
        o = solve_opts(self.cfg.precision, **opts)
        jid = ctypes.c_int64(0)
        rc = lib().lddmm_server_submit(self._h, ctypes.byref(prm), ctypes.byref(o),
                                       q0.ctypes.data, target.ctypes.data,
                                       p0.ctypes.data if p0 is not None else None,
                                       ctypes.byref(jid))
        if rc != OK:
            self._err(rc)
        self._n[jid.value] = n
        return jid.value

    def poll(self, job_id: int):
        """None while the job runs; else dict(p0, status, loss, ..., times)."""
        import numpy as np
        n = self._n[job_id]
        p0 = np.empty((n, 3))
        res, tm = SolveResult(), JobTimes()
        rc = lib().lddmm_server_poll(self._h, job_id, p0.ctypes.data, ctypes.byref(res),
                                     ctypes.byref(tm))
        if rc == EBUSY:
            return None
        if rc not in (OK, ENOTCONV, ENONFINITE):
            self._err(rc)
        del self._n[job_id]
        r = {k: getattr(res, k) for k, _ in SolveResult._fields_}
        r.update(p0=p0, submit_s=tm.submit_s, admit_s=tm.admit_s, done_s=tm.done_s)
        return r

    def wait(self, job_id: int, timeout: float | None = None) -> bool:
        rc = lib().lddmm_server_wait(self._h, job_id, -1.0 if timeout is None else float(timeout))
        if rc == EBUSY:
            return False
        if rc != OK:
            self._err(rc)
        return True

    def result(self, job_id: int, timeout: float | None = None):
        if not self.wait(job_id, timeout):
            raise TimeoutError(f"job {job_id} not done")
        return self.poll(job_id)

    def stats(self) -> dict:
        st = ServerStats()
        rc = lib().lddmm_server_stats_get(self._h, ctypes.byref(st))
        if rc != OK:
            self._err(rc)
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().lddmm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def version() -> str:
    return lib().lddmm_version().decode()
