"""Plain FP64 CPU oracle for landmark geodesic shooting (test infrastructure).

A thin ctypes wrapper over ``lddmm_oracle.c``.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg use it; the GPU library and its
Python binding never import it.  Every function takes and returns float64
numpy arrays of shape [N, 3].

Formulas followed (paper Sec. 2.1, eqs. 1-3, Algs. 1-2): see the header of
``lddmm_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB selects another build of the same source (the sanitizer test's).
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


class _Opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("m", ctypes.c_int), ("max_fev", ctypes.c_int),
                ("gtol", ctypes.c_double), ("ftol_rel", ctypes.c_double),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double), ("init", ctypes.c_int)]


class _Result(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_double), ("H0", ctypes.c_double),
                ("mismatch", ctypes.c_double), ("grad_norm", ctypes.c_double),
                ("avg_dist", ctypes.c_double), ("max_dist", ctypes.c_double),
                ("iters", ctypes.c_int), ("fevals", ctypes.c_int), ("status", ctypes.c_int)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_get_threads.restype = ctypes.c_int
        L.oracle_pair_forward.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp, ctypes.c_int]
        L.oracle_pair_adjoint.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp,
                                          ctypes.c_int]
        _ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_pair_forward_rows.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _ip,
                                               ctypes.c_int, _dp, _dp]
        L.oracle_pair_adjoint_rows.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp,
                                               _ip, ctypes.c_int, _dp, _dp]
        L.oracle_hamiltonian.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, ctypes.c_int]
        L.oracle_hamiltonian.restype = ctypes.c_double
        L.oracle_shoot_forward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp,
                                           _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int]
        L.oracle_shoot_forward.restype = ctypes.c_int
        L.oracle_velocity.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp,
                                      _dp, ctypes.c_int]
        L.oracle_flow.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp,
                                  ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int]
        L.oracle_flow.restype = ctypes.c_int
        L.oracle_shoot_grad.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
        L.oracle_shoot_grad.restype = ctypes.c_int
        L.oracle_shoot_grad_all.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                            _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_shoot_grad_all.restype = ctypes.c_int
        L.oracle_solve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   _dp, _dp, _dp, ctypes.POINTER(_Opts), ctypes.POINTER(_Result),
                                   _dp, ctypes.c_int]
        L.oracle_solve.restype = ctypes.c_int
        L.oracle_cubic_step.argtypes = [ctypes.c_double] * 6
        L.oracle_cubic_step.restype = ctypes.c_double
        _lib = L
    return _lib


def _in(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("expected an [N,3] array")
    return a


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def set_threads(k: int) -> None:
    lib().oracle_set_threads(int(k))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def pair_forward(q, p, sigma: float, compensated: bool = False):
    """(Hq, Hp) = (dH/dq, dH/dp) at (q, p): the right-hand side of eq. 2."""
    q, p = _in(q), _in(p)
    Hq, Hp = np.empty_like(q), np.empty_like(q)
    lib().oracle_pair_forward(q.shape[0], float(sigma), _p(q), _p(p), _p(Hq), _p(Hp), int(compensated))
    return Hq, Hp


def pair_adjoint(q, p, a, b, sigma: float, compensated: bool = False):
    """(A, B) of one backward Euler step: a(t) = a + dt A, b(t) = b + dt B."""
    q, p, a, b = _in(q), _in(p), _in(a), _in(b)
    A, B = np.empty_like(q), np.empty_like(q)
    lib().oracle_pair_adjoint(q.shape[0], float(sigma), _p(q), _p(p), _p(a), _p(b), _p(A), _p(B),
                              int(compensated))
    return A, B


def _rows(rows) -> np.ndarray:
    return np.ascontiguousarray(rows, dtype=np.int32)


def pair_forward_rows(q, p, sigma: float, rows):
    """(Hq, Hp) for the listed rows only (each summed over all j)."""
    q, p, rows = _in(q), _in(p), _rows(rows)
    Hq, Hp = np.empty((len(rows), 3)), np.empty((len(rows), 3))
    lib().oracle_pair_forward_rows(q.shape[0], float(sigma), _p(q), _p(p),
                                   rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(rows),
                                   _p(Hq), _p(Hp))
    return Hq, Hp


def pair_adjoint_rows(q, p, a, b, sigma: float, rows):
    """(A, B) for the listed rows only (each summed over all j)."""
    q, p, a, b, rows = _in(q), _in(p), _in(a), _in(b), _rows(rows)
    A, B = np.empty((len(rows), 3)), np.empty((len(rows), 3))
    lib().oracle_pair_adjoint_rows(q.shape[0], float(sigma), _p(q), _p(p), _p(a), _p(b),
                                   rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(rows),
                                   _p(A), _p(B))
    return A, B


def hamiltonian(q, p, sigma: float, compensated: bool = False) -> float:
    """H(q,p) = 1/2 sum_ij g_ij p_i.p_j (eq. 1)."""
    q, p = _in(q), _in(p)
    return float(lib().oracle_hamiltonian(q.shape[0], float(sigma), _p(q), _p(p), int(compensated)))


INTEGRATORS = {"euler": 0, "rk4": 1}


def _integrator(name: str) -> int:
    if name not in INTEGRATORS:
        raise ValueError("integrator must be 'euler' or 'rk4'")
    return INTEGRATORS[name]


def shoot_forward(q0, p0, sigma: float, T: int, traj: bool = False, compensated: bool = False,
                  integrator: str = "euler"):
    """Hamiltonian flow over [0,1] in T explicit Euler steps (Alg. 1, forward
    loop) or, with integrator="rk4", T classical Runge-Kutta steps.

    Returns dict(q1, p1, H0, Hp0[, traj (T+1, 2, N, 3)]).
    """
    q0, p0 = _in(q0), _in(p0)
    n = q0.shape[0]
    q1, p1, Hp0 = np.empty_like(q0), np.empty_like(q0), np.empty_like(q0)
    H0 = ctypes.c_double(0.0)
    tr = np.empty((T + 1, 2, n, 3)) if traj else None
    rc = lib().oracle_shoot_forward(n, int(T), float(sigma), _p(q0), _p(p0), _p(q1), _p(p1),
                                    ctypes.byref(H0), _p(tr), _p(Hp0), int(compensated),
                                    _integrator(integrator))
    if rc != 0:
        raise MemoryError("oracle_shoot_forward")
    out = dict(q1=q1, p1=p1, H0=H0.value, Hp0=Hp0)
    if traj:
        out["traj"] = tr
    return out


def velocity(q, p, x, sigma: float, compensated: bool = False):
    """Velocity field of eq. 4, v(x) = sum_l g(|q_l - x|) p_l, at the points x [M,3]."""
    q, p, x = _in(q), _in(p), _in(x)
    v = np.empty_like(x)
    lib().oracle_velocity(q.shape[0], x.shape[0], float(sigma), _p(q), _p(p), _p(x), _p(v),
                          int(compensated))
    return v


def flow(q0, p0, x0, sigma: float, T: int, compensated: bool = False, integrator: str = "euler"):
    """Points x0 [M,3] carried by the landmark motion from (q0, p0) over T explicit
    Euler steps of eq. 4's velocity (integrator="rk4": Runge-Kutta steps of the
    joint system).  Returns dict(x1, q1)."""
    q0, p0, x0 = _in(q0), _in(p0), _in(x0)
    x1, q1 = np.empty_like(x0), np.empty_like(q0)
    rc = lib().oracle_flow(q0.shape[0], int(T), float(sigma), _p(q0), _p(p0), x0.shape[0], _p(x0),
                           _p(x1), _p(q1), int(compensated), _integrator(integrator))
    if rc != 0:
        raise MemoryError("oracle_flow")
    return dict(x1=x1, q1=q1)


def shoot_grad(q0, p0, x, sigma: float, lam: float, T: int, compensated: bool = False,
               all_grads: bool = False, energy: str = "initial", integrator: str = "euler"):
    """Loss L = H(q0,p0) + lam |q(1)-x|^2 (eq. 3) and dL/dp0 (exact discrete adjoint).

    energy="final" uses H(q(1),p(1)) as the energy term (the loss as Alg. 1
    evaluates it after the forward loop).  integrator="rk4" takes classical
    Runge-Kutta steps and the exact adjoint of their stages.  Returns
    dict(loss, grad, q1, H0 (the energy term), mismatch[, grad_q0, grad_x]).
    """
    if energy not in ("initial", "final"):
        raise ValueError("energy must be 'initial' or 'final'")
    q0, p0, x = _in(q0), _in(p0), _in(x)
    n = q0.shape[0]
    grad, q1 = np.empty_like(q0), np.empty_like(q0)
    gq = np.empty_like(q0) if all_grads else None
    gx = np.empty_like(q0) if all_grads else None
    loss = ctypes.c_double(0.0)
    terms = np.zeros(2)
    rc = lib().oracle_shoot_grad_all(n, int(T), float(sigma), float(lam), _p(q0), _p(p0), _p(x),
                                     ctypes.byref(loss), _p(grad), _p(gq), _p(gx), _p(q1),
                                     _p(terms), int(compensated), int(energy == "final"),
                                     _integrator(integrator))
    if rc != 0:
        raise MemoryError("oracle_shoot_grad")
    out = dict(loss=loss.value, grad=grad, q1=q1, H0=float(terms[0]), mismatch=float(terms[1]))
    if all_grads:
        out.update(grad_q0=gq, grad_x=gx)
    return out


def cubic_step(a0: float, f0: float, d0: float, a1: float, f1: float, d1: float) -> float:
    """The line search's interpolation step: the minimiser of the cubic through
    (a0, f0, f'(a0) = d0) and (a1, f1, f'(a1) = d1), kept inside the middle 80 %
    of the bracket, else the midpoint."""
    return float(lib().oracle_cubic_step(float(a0), float(f0), float(d0), float(a1),
                                         float(f1), float(d1)))


@dataclass
class SolveOpts:
    max_iter: int = 50
    m: int = 5
    max_fev: int = 20
    gtol: float = 1e-8
    ftol_rel: float = 0.0
    c1: float = 1e-4
    c2: float = 0.9
    init: int = 0   # 0: p0 = 0, 1: (x - q0)/T, 2: caller's p0


def solve(q0, x, sigma: float, lam: float, T: int, opts: SolveOpts | None = None, p0=None,
          compensated: bool = False):
    """L-BFGS on p0 (Alg. 1, steps (e)-(f)); own implementation.

    Returns dict(p0, loss, H0, mismatch, grad_norm, avg_dist, max_dist, iters,
    fevals, status, trace [iters+1, 2] of (loss, |g|)).
    """
    opts = opts or SolveOpts()
    q0, x = _in(q0), _in(x)
    n = q0.shape[0]
    p = np.zeros_like(q0) if p0 is None else _in(p0).copy()
    o = _Opts(opts.max_iter, opts.m, opts.max_fev, opts.gtol, opts.ftol_rel, opts.c1, opts.c2,
              opts.init)
    r = _Result()
    trace = np.full((opts.max_iter + 1, 2), np.nan)
    rc = lib().oracle_solve(n, int(T), float(sigma), float(lam), _p(q0), _p(x), _p(p),
                            ctypes.byref(o), ctypes.byref(r), _p(trace), int(compensated))
    if rc == -2:
        raise MemoryError("oracle_solve")
    return dict(p0=p, loss=r.loss, H0=r.H0, mismatch=r.mismatch, grad_norm=r.grad_norm,
                avg_dist=r.avg_dist, max_dist=r.max_dist, iters=r.iters, fevals=r.fevals,
                status=r.status, trace=trace[: r.iters + 1])
