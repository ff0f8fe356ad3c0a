"""torch.autograd access to the shooting loss (eq. 3) and its exact discrete
adjoint gradient.

``ShootLoss.apply(p0, q0, target, cfg)`` returns the scalar FP64 loss
L(p0) = H(q0, p0) + lambda |q(1) - x|^2.  Its forward pass runs one
``lddmm_shoot_grad`` (forward flow, loss and adjoint pass in the HIP
library), so the gradients are ready when the loss is; backward only scales
them.  Gradients flow to p0, and to q0 and the target when they require
them (``lddmm_shoot_grad_all``).

When the whole trajectory (T+1 records of N landmarks) would not fit in the
configured budget, the library keeps every s-th FP64 state and recomputes
each segment of s steps before its backward pass; results are bitwise the
same as with the full trajectory.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import lddmm

_contexts: dict[int, lddmm.Context] = {}


def context(device: int | None = None) -> lddmm.Context:
    """A shared library context per GPU."""
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _contexts:
        _contexts[dev] = lddmm.Context(dev)
    return _contexts[dev]


@dataclass
class ShootConfig:
    T: int
    sigma: float
    lam: float
    precision: str = "fp32c"
    ckpt_every: int | str = "auto"     # int s >= 0, or "auto"
    traj_budget_bytes: int = 2 << 30    # trajectory memory allowed before checkpointing
    energy: str = "initial"             # energy term H(q0,p0) ("initial") or H(q(1),p(1))
    dim: int = 3                        # 2: planar problem (every z component 0)
    integrator: str = "euler"           # "euler" (Alg. 1) or "rk4" (classical Runge-Kutta)

    def resolve_ckpt(self, n: int) -> int:
        if self.ckpt_every != "auto":
            return int(self.ckpt_every)
        rec = 64 if self.precision == "fp64" else 32
        spt = 4 if self.integrator == "rk4" else 1   # records per step
        if (spt * self.T + 1) * n * rec <= self.traj_budget_bytes:
            return 0
        # segment length whose ring of spt s + 1 records fits, at most sqrt(T)
        s = max(1, int(math.ceil(math.sqrt(self.T))))
        while s > 1 and (spt * s + 1) * n * rec > self.traj_budget_bytes:
            s //= 2
        return s


class ShootLoss(torch.autograd.Function):
    @staticmethod
    def forward(actx, p0: torch.Tensor, q0: torch.Tensor, target: torch.Tensor,
                cfg: ShootConfig):
        n = q0.shape[0]
        ctx = context(q0.device.index)
        want_q0, want_x = actx.needs_input_grad[1], actx.needs_input_grad[2]
        r = ctx.shoot_grad(q0.detach().contiguous(), p0.detach().contiguous(),
                           target.detach().contiguous(), cfg.T, cfg.sigma, cfg.lam,
                           precision=cfg.precision, ckpt_every=cfg.resolve_ckpt(n),
                           want_q1=False, want_grad_q0=want_q0, want_grad_x=want_x,
                           energy=cfg.energy, dim=cfg.dim, integrator=cfg.integrator)
        saved = [r.grad] + ([r.grad_q0] if want_q0 else []) + ([r.grad_x] if want_x else [])
        actx.save_for_backward(*saved)
        actx.layout = (want_q0, want_x)
        return r.loss.clone()

    @staticmethod
    def backward(actx, grad_out: torch.Tensor):
        saved = list(actx.saved_tensors)
        want_q0, want_x = actx.layout
        g = saved.pop(0)
        gq = grad_out * saved.pop(0) if want_q0 else None
        gx = grad_out * saved.pop(0) if want_x else None
        return grad_out * g, gq, gx, None


def shoot_loss(p0, q0, target, T: int, sigma: float, lam: float, precision: str = "fp32c",
               ckpt_every: int | str = "auto", energy: str = "initial",
               integrator: str = "euler") -> torch.Tensor:
    """Differentiable loss of eq. 3 (with respect to p0, q0 and target)."""
    return ShootLoss.apply(p0, q0, target,
                           ShootConfig(T, sigma, lam, precision, ckpt_every, energy=energy,
                                       integrator=integrator))
