"""Seeded synthetic landmark workloads.

The paper evaluates on 1847 landmarks sampled from a medial-temporal-lobe
template and warped to 34 subjects (Sec. 3.1).  That data is not available,
so every workload here is synthetic: landmark clouds of the same kind
(surfaces, blobs, uniform boxes) and targets produced by a smooth random
diffeomorphic warp.  This module only draws inputs; it holds none of the
shooting method's arithmetic, and both the GPU path and the CPU oracle are
fed from it.

All arrays are float64, shape [N, 3], C-contiguous.  Randomness comes from
``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


@dataclass
class Problem:
    """One registration problem: template q0, target x, start momentum p0."""

    name: str
    q0: np.ndarray
    target: np.ndarray
    p0: np.ndarray
    sigma: float
    lam: float
    T: int
    iters: int = 0
    precision: str = "fp32c"
    ckpt_every: int = 0
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.q0.shape[0])


# --------------------------------------------------------------------------
# clouds
# --------------------------------------------------------------------------

def uniform_box(rng: np.random.Generator, n: int, lo: float, hi: float) -> np.ndarray:
    return rng.uniform(lo, hi, size=(n, 3))


def ellipsoid(rng: np.random.Generator, n: int, axes, sd: float) -> np.ndarray:
    """Points on a noisy ellipsoid surface: direction uniform on the sphere,
    scaled by the semi-axes, plus isotropic Gaussian noise of std ``sd``."""
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return u * np.asarray(axes, dtype=np.float64)[None, :] + sd * rng.standard_normal((n, 3))


def blobs(rng: np.random.Generator, n: int, centres, sd: float) -> np.ndarray:
    """Isotropic Gaussian blobs of equal size (the last takes the remainder)."""
    centres = np.asarray(centres, dtype=np.float64)
    k = centres.shape[0]
    sizes = [n // k] * k
    sizes[-1] += n - sum(sizes)
    parts = [c[None, :] + sd * rng.standard_normal((m, 3)) for c, m in zip(centres, sizes)]
    return np.concatenate(parts, axis=0)


# --------------------------------------------------------------------------
# smooth random deformations used to make targets
# --------------------------------------------------------------------------

@dataclass
class Bumps:
    centres: np.ndarray  # [K,3]
    amps: np.ndarray     # [K,3]
    width: float

    def field(self, y: np.ndarray) -> np.ndarray:
        """Velocity u(y) = sum_k A_k exp(-|y-c_k|^2 / (2 w^2))."""
        d2 = ((y[:, None, :] - self.centres[None, :, :]) ** 2).sum(-1)
        w = np.exp(-d2 / (2.0 * self.width ** 2))
        return w @ self.amps


def bumps(rng: np.random.Generator, k: int, width: float, sd: float, q: np.ndarray) -> Bumps:
    """K centres uniform in the bounding box of ``q``; amplitudes N(0, sd^2 I)."""
    lo, hi = q.min(axis=0), q.max(axis=0)
    c = lo + (hi - lo) * rng.uniform(0.0, 1.0, size=(k, 3))
    a = sd * rng.standard_normal((k, 3))
    return Bumps(c, a, float(width))


def warp(q: np.ndarray, b: Bumps, steps: int = 20) -> np.ndarray:
    """Flow of dy/dt = u(y) over [0,1] with classical RK4: a diffeomorphic
    image of ``q`` for a smooth u."""
    y = q.copy()
    h = 1.0 / steps
    for _ in range(steps):
        k1 = b.field(y)
        k2 = b.field(y + 0.5 * h * k1)
        k3 = b.field(y + 0.5 * h * k2)
        k4 = b.field(y + h * k3)
        y = y + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def displacement(q: np.ndarray, b: Bumps) -> np.ndarray:
    return q + b.field(q)


def _c(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# the five workload families
# --------------------------------------------------------------------------

def box_displacement(seed: int = 1001, n: int = 64) -> Problem:
    """Uniform cloud in [0,100]^3, target = q0 + sum of 4 bumps (width 30,
    amplitude sd 5); sigma=10, lambda=1, T=10, p0=0, 50 iterations, FP64."""
    rng = np.random.default_rng(seed)
    q0 = uniform_box(rng, n, 0.0, 100.0)
    x = displacement(q0, bumps(rng, 4, 30.0, 5.0, q0))
    return Problem("box64_fp64", _c(q0), _c(x), np.zeros_like(q0), 10.0, 1.0, 10,
                   iters=50, precision="fp64", seed=seed)


def ellipsoid_warp(seed: int = 1002, n: int = 4096, T: int = 40, iters: int = 200) -> Problem:
    """Noisy ellipsoid (semi-axes 60,40,30, noise sd 1); target = RK4 warp by
    8 bumps (width 25, amplitude sd 6); sigma=8, lambda=1, p0=0, FP32 sums."""
    rng = np.random.default_rng(seed)
    q0 = ellipsoid(rng, n, (60.0, 40.0, 30.0), 1.0)
    x = warp(q0, bumps(rng, 8, 25.0, 6.0, q0))
    return Problem(f"ellipsoid{n}_T{T}", _c(q0), _c(x), np.zeros_like(q0), 8.0, 1.0, T,
                   iters=iters, precision="fp32c", seed=seed)


def sphere_autograd(seed: int = 1003, n: int = 16384, T: int = 100, ckpt_every: int = 10) -> Problem:
    """Noisy sphere (radius 80, sd 1), p0 ~ N(0, 0.5^2) i.i.d.; target = RK4
    warp by 8 bumps (width 25, sd 6), lambda=1; sigma=6, T=100, checkpoints
    every 10 steps."""
    rng = np.random.default_rng(seed)
    q0 = ellipsoid(rng, n, (80.0, 80.0, 80.0), 1.0)
    p0 = 0.5 * rng.standard_normal((n, 3))
    x = warp(q0, bumps(rng, 8, 25.0, 6.0, q0))
    return Problem(f"sphere{n}_T{T}", _c(q0), _c(x), _c(p0), 6.0, 1.0, T,
                   precision="fp32c", ckpt_every=ckpt_every, seed=seed)


def serving_job(j: int, n: int | None = None) -> Problem:
    """One job of the serving stream: ellipsoid -> warped ellipsoid as in
    ``ellipsoid_warp`` with a per-job seed; N log-uniform in [500, 8000];
    T=40, 100 iterations, FP32 sums."""
    seed = 40000 + j
    rng = np.random.default_rng(seed)
    if n is None:
        n = int(round(math.exp(rng.uniform(math.log(500.0), math.log(8000.0)))))
    q0 = ellipsoid(rng, n, (60.0, 40.0, 30.0), 1.0)
    x = warp(q0, bumps(rng, 8, 25.0, 6.0, q0))
    return Problem(f"job{j}_n{n}", _c(q0), _c(x), np.zeros_like(q0), 8.0, 1.0, 40,
                   iters=100, precision="fp32c", seed=seed)


def arrivals(n_jobs: int = 512, rate: float = 200.0, seed: int = 49999) -> np.ndarray:
    """Poisson arrival times (seconds) of the serving stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))


def two_blobs(seed: int = 1005, n: int = 65536, T: int = 50) -> Problem:
    """Two Gaussian blobs (centres (+-25,0,0), sd 15); sigma=5, T=50,
    p0 ~ N(0, 0.5^2), target = q0 + 4 bumps (width 30, sd 5), lambda=1."""
    rng = np.random.default_rng(seed)
    q0 = blobs(rng, n, [(-25.0, 0.0, 0.0), (25.0, 0.0, 0.0)], 15.0)
    p0 = 0.5 * rng.standard_normal((n, 3))
    x = displacement(q0, bumps(rng, 4, 30.0, 5.0, q0))
    return Problem(f"blobs{n}_T{T}", _c(q0), _c(x), _c(p0), 5.0, 1.0, T,
                   precision="fp32c", seed=seed)


def random_problem(seed: int, n: int, T: int = 5, sigma: float = 1.5, lam: float = 1.0,
                   p_scale: float = 0.3, spread: float = 3.0) -> Problem:
    """Small generic problem for unit and parity tests."""
    rng = np.random.default_rng(seed)
    q0 = spread * rng.standard_normal((n, 3))
    p0 = p_scale * rng.standard_normal((n, 3))
    x = q0 + 0.5 * rng.standard_normal((n, 3))
    return Problem(f"rand{n}_s{seed}", _c(q0), _c(x), _c(p0), sigma, lam, T, seed=seed)


def subsample(pb: Problem, m: int, seed: int = 7) -> Problem:
    """Seeded row subsample (same rows of q0, target and p0)."""
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(pb.n, size=m, replace=False))
    return Problem(pb.name + f"_sub{m}", _c(pb.q0[idx]), _c(pb.target[idx]), _c(pb.p0[idx]),
                   pb.sigma, pb.lam, pb.T, iters=pb.iters, precision=pb.precision,
                   ckpt_every=pb.ckpt_every, seed=pb.seed, extra={"rows": idx})


CONFIGS = {
    1: box_displacement,
    2: ellipsoid_warp,
    3: sphere_autograd,
    5: two_blobs,
}


# --------------------------------------------------------------------------
# points to deform (flow of eq. 4)
# --------------------------------------------------------------------------

def grid(lo, hi, k: int) -> np.ndarray:
    """Regular k x k x k grid spanning the box [lo, hi], [k^3, 3] (last axis fastest)."""
    ax = [np.linspace(float(lo[d]), float(hi[d]), k) for d in range(3)]
    return _c(np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3))


def ellipsoid_grid(k: int = 64, n: int = 4096, T: int = 40) -> tuple[Problem, np.ndarray]:
    """The ellipsoid registration of ``ellipsoid_warp`` with the momentum
    p0 = (x - q0) / 2, and a k^3 grid over the landmarks' bounding box grown by
    2 sigma on every side: the voxel centres an image warp would carry."""
    pb = ellipsoid_warp(n=n, T=T)
    pb.p0 = _c(0.5 * (pb.target - pb.q0))
    pad = 2.0 * pb.sigma
    pts = grid(pb.q0.min(0) - pad, pb.q0.max(0) + pad, k)
    pb.name = f"ellipsoid{n}_T{T}_grid{k}"
    return pb, pts


# --------------------------------------------------------------------------
# planar problems (every z component 0)
# --------------------------------------------------------------------------

def planar(pb: Problem) -> Problem:
    """The same problem with the z components of q0, target and p0 set to 0."""
    z = lambda a: _c(np.concatenate([a[:, :2], np.zeros((a.shape[0], 1))], axis=1))  # noqa: E731
    return Problem(pb.name + "_planar", z(pb.q0), z(pb.target), z(pb.p0), pb.sigma, pb.lam,
                   pb.T, iters=pb.iters, precision=pb.precision, ckpt_every=pb.ckpt_every,
                   seed=pb.seed)


def ellipse_warp(seed: int = 1006, n: int = 4096, T: int = 40, iters: int = 200) -> Problem:
    """Planar counterpart of ``ellipsoid_warp``: a noisy ellipse (semi-axes 60,
    40, in-plane noise sd 1) in the plane z = 0, matched to its RK4 warp by 8
    in-plane bumps (width 25, amplitude sd 6); sigma 8, lambda 1, p0 = 0."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, 2.0 * math.pi, size=n)
    q0 = np.stack([60.0 * np.cos(t), 40.0 * np.sin(t), np.zeros(n)], axis=1)
    q0[:, :2] += rng.standard_normal((n, 2))
    b = bumps(rng, 8, 25.0, 6.0, q0)
    b.centres[:, 2] = 0.0
    b.amps[:, 2] = 0.0
    x = warp(q0, b)
    return Problem(f"ellipse{n}_T{T}", _c(q0), _c(x), np.zeros_like(q0), 8.0, 1.0, T,
                   iters=iters, precision="fp32c", seed=seed)
