"""Seeded, synthetic initial data for the KGS workloads.

This module only builds inputs: grids, initial fields psi0, u0, v0 and
parameter draws.  It holds none of the scheme's arithmetic, so both the GPU
path and the CPU oracle take their inputs from here.

Grid points are x_j = lo + j*h, j = 0..n-1, h = (hi-lo)/n on every axis (the
paper's x_j = a + (j-1)h re-based to 0, sec. 2).  Arrays have shape (n,)*dim
in C order, axis 0 slowest.  Recipes follow the paper's style of analytic
initial data (sec. 5): Gaussians e^{-|x-c|^2}, sech profiles and plane-wave
phases.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

FP64 = 0
FP32 = 1


@dataclass
class Problem:
    """One KGS initial-value problem on a periodic box [lo, hi)^dim."""

    name: str
    dim: int
    n: int
    lo: float
    hi: float
    tau: float
    steps: int
    kappa1: float = 1.0
    kappa2: float = 1.0
    mu: float = 1.0
    gamma: float = 1.0
    precision: int = FP64
    recipe: object = field(default=None, repr=False)
    psi: Optional[np.ndarray] = field(default=None, repr=False)
    u: Optional[np.ndarray] = field(default=None, repr=False)
    v: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def h(self) -> float:
        return (self.hi - self.lo) / self.n

    @property
    def points(self) -> int:
        return self.n ** self.dim

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def axes(dim: int, n: int, lo: float, hi: float):
    """Coordinate arrays x_0..x_{dim-1}, each of shape (n,)*dim."""
    h = (hi - lo) / n
    x = lo + h * np.arange(n, dtype=np.float64)
    return np.meshgrid(*([x] * dim), indexing="ij")


def _sech(x):
    return 1.0 / np.cosh(x)


def config_1d(n: int = 256, steps: int = 1000) -> Problem:
    """1-D: [-20,20), tau=0.01; psi0 = sech(x) e^{0.5ix}, u0 = 0.5 sech^2(x), v0 = 0."""
    p = Problem("kgs1d", 1, n, -20.0, 20.0, 0.01, steps)
    (x,) = axes(1, n, p.lo, p.hi)
    p.psi = _sech(x) * np.exp(0.5j * x)
    p.u = 0.5 * _sech(x) ** 2
    p.v = np.zeros_like(x)
    return p


def config_2d(n: int = 1024, steps: int = 1000) -> Problem:
    """2-D: [-16,16)^2, tau=0.005; two unit-width Gaussians centred at (-4,0)
    and (4,0) with phases e^{+0.5ix} and e^{-0.5ix} (moving towards each
    other); u0 = e^{-|x|^2}, v0 = 0."""
    p = Problem("kgs2d", 2, n, -16.0, 16.0, 0.005, steps)
    x, y = axes(2, n, p.lo, p.hi)
    left = np.exp(-((x + 4.0) ** 2 + y ** 2)) * np.exp(0.5j * x)
    right = np.exp(-((x - 4.0) ** 2 + y ** 2)) * np.exp(-0.5j * x)
    p.psi = left + right
    p.u = np.exp(-(x ** 2 + y ** 2))
    p.v = np.zeros_like(x)
    return p


def config_3d(n: int = 256, steps: int = 200, precision: int = FP64) -> Problem:
    """3-D: [-8,8)^3, tau=0.002; psi0 = e^{-|x|^2} e^{i(x + 0.5y)} (k=(1,0.5,0)),
    u0 = 0.5 e^{-|x|^2/2}, v0 = 0; kappa1=kappa2=mu=gamma=1."""
    p = Problem("kgs3d", 3, n, -8.0, 8.0, 0.002, steps, precision=precision)
    x, y, z = axes(3, n, p.lo, p.hi)
    r2 = x ** 2 + y ** 2 + z ** 2
    p.psi = np.exp(-r2) * np.exp(1j * (x + 0.5 * y))
    p.u = 0.5 * np.exp(-r2 / 2.0)
    p.v = np.zeros_like(x)
    return p


def accuracy_2d(level: int = 0, precision: int = FP64) -> Problem:
    """The 2-D example of sec. 5.1 (the problem of Tab. conv2d): periodic on
    [-10,10)^2, kappa1 = kappa2 = gamma = mu = 1,
    psi0 = (1+i) e^{-(x^2+y^2)}, u0 = tanh(x^2+y^2),
    v0 = sin(x+y) e^{-2(x^2+y^2)}, up to t = 1.  Level L halves h and tau L
    times from (h, tau) = (5/16, 1/50): n = 64 * 2^L, 50 * 2^L steps."""
    n, steps = 64 << level, 50 << level
    p = Problem(f"accuracy2d_l{level}", 2, n, -10.0, 10.0, 1.0 / steps, steps,
                precision=precision)
    x, y = axes(2, n, p.lo, p.hi)
    r2 = x ** 2 + y ** 2
    p.psi = (1.0 + 1.0j) * np.exp(-r2)
    p.u = np.tanh(r2)
    p.v = np.sin(x + y) * np.exp(-2.0 * r2)
    return p


def timing_2d(n: int = 1024, precision: int = FP64) -> Problem:
    """The 2-D timing example of sec. 5.1 (Tab. time-2d): four Gaussian
    solitons at (0,-3), (3,0), (0,3), (-3,0) on (-10,10)^2,
    psi0 = (1+i) sum_j e^{-|x-x_j|^2}, u0 = sum_j tanh|x-x_j|^2,
    v0 = e^{-|x|^2}; kappa1 = kappa2 = gamma = mu = 0.5, tau = 0.01 up to
    t = 1 (100 steps)."""
    p = Problem("timing2d", 2, n, -10.0, 10.0, 0.01, 100, kappa1=0.5, kappa2=0.5, mu=0.5,
                gamma=0.5, precision=precision)
    x, y = axes(2, n, p.lo, p.hi)
    psi = np.zeros_like(x, dtype=np.complex128)
    u = np.zeros_like(x)
    for cx, cy in ((0.0, -3.0), (3.0, 0.0), (0.0, 3.0), (-3.0, 0.0)):
        r2 = (x - cx) ** 2 + (y - cy) ** 2
        psi += np.exp(-r2)
        u += np.tanh(r2)
    p.psi = (1.0 + 1.0j) * psi
    p.u = u
    p.v = np.exp(-(x ** 2 + y ** 2))
    return p


def timing_3d(n: int = 256, precision: int = FP64) -> Problem:
    """The 3-D example of sec. 5.2 (Tab. gpu3d_list): two Gaussian packets
    at x = -2 and x = 2 with the phase e^{0.01i(x+y+z)},
    u0 = e^{-(x^2+y^2+(z-2)^2)} + sum_{s=+-1} e^{-((x+s sqrt3)^2+y^2+(z+1)^2)},
    v0 = e^{-|x|^2} on (-10,10)^3; kappa1 = -0.4, kappa2 = 0.1,
    gamma = 0.2, mu = 0.1, tau = 0.01 up to t = 1 (100 steps)."""
    p = Problem("timing3d", 3, n, -10.0, 10.0, 0.01, 100, kappa1=-0.4, kappa2=0.1, mu=0.1,
                gamma=0.2, precision=precision)
    x, y, z = axes(3, n, p.lo, p.hi)
    yz = y ** 2 + z ** 2
    phase = np.exp(0.01j * (x + y + z))
    p.psi = (np.exp(-((x + 2.0) ** 2) - yz) + np.exp(-((x - 2.0) ** 2) - yz)) * phase
    r3 = np.sqrt(3.0)
    p.u = (np.exp(-(x ** 2 + y ** 2 + (z - 2.0) ** 2))
           + np.exp(-((x + r3) ** 2 + y ** 2 + (z + 1.0) ** 2))
           + np.exp(-((x - r3) ** 2 + y ** 2 + (z + 1.0) ** 2)))
    p.v = np.exp(-(x ** 2 + yz))
    return p


def random_problem(dim: int, n: int, seed: int, tau: float = 0.01, amp: float = 1.0,
                   precision: int = FP64, steps: int = 1, lo: float = -4.0, hi: float = 4.0,
                   params=None) -> Problem:
    """Independent uniform random fields on every point (a worst case for the
    stencil: no smoothness), seeded; parameters drawn from U[0.5, 2] unless
    given."""
    rng = np.random.default_rng(seed)
    if params is None:
        params = rng.uniform(0.5, 2.0, size=4)
    k1, k2, mu, g = params
    p = Problem(f"random{dim}d", dim, n, lo, hi, tau, steps, k1, k2, mu, g, precision)
    shape = (n,) * dim
    p.psi = amp * (rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape))
    p.u = amp * rng.uniform(-1, 1, shape)
    p.v = amp * rng.uniform(-1, 1, shape)
    return p


def gaussian_problem(dim: int, n: int, seed: int, lo: float, hi: float, tau: float, steps: int,
                     precision: int = FP64, params=None, arrays: bool = True) -> Problem:
    """Gaussian psi0 and u0 with seeded centres in the middle half of the box,
    a seeded plane-wave phase, v0 = 0, parameters ~ U[0.5, 2] unless given.
    With arrays=False only the recipe is drawn (see gaussian_fields_torch)."""
    rng = np.random.default_rng(seed)
    if params is None:
        params = rng.uniform(0.5, 2.0, size=4)
    k1, k2, mu, g = params
    p = Problem(f"gauss{dim}d", dim, n, lo, hi, tau, steps, float(k1), float(k2), float(mu),
                float(g), precision)
    half = 0.25 * (hi - lo)
    c_psi = rng.uniform(-half, half, size=dim)
    c_u = rng.uniform(-half, half, size=dim)
    k = rng.uniform(-1.0, 1.0, size=dim)
    p.recipe = (c_psi, c_u, k)
    if not arrays:
        return p
    X = axes(dim, n, lo, hi)
    r2 = sum((X[a] - c_psi[a]) ** 2 for a in range(dim))
    phase = sum(k[a] * X[a] for a in range(dim))
    p.psi = np.exp(-r2) * np.exp(1j * phase)
    p.u = 0.5 * np.exp(-sum((X[a] - c_u[a]) ** 2 for a in range(dim)))
    p.v = np.zeros_like(X[0])
    return p


def gaussian_fields_torch(p: Problem, device="cuda"):
    """The fields of a gaussian_problem recipe computed on a torch device in
    float64: (psi_re, psi_im, u, v), each of shape (n,)*dim."""
    import torch

    c_psi, c_u, k = p.recipe
    x = p.lo + p.h * torch.arange(p.n, dtype=torch.float64, device=device)
    X = torch.meshgrid(*([x] * p.dim), indexing="ij")
    r2 = sum((X[a] - float(c_psi[a])) ** 2 for a in range(p.dim))
    ph = sum(float(k[a]) * X[a] for a in range(p.dim))
    amp = torch.exp(-r2)
    u = 0.5 * torch.exp(-sum((X[a] - float(c_u[a])) ** 2 for a in range(p.dim)))
    return (amp * torch.cos(ph)).contiguous(), (amp * torch.sin(ph)).contiguous(), u.contiguous(), \
        torch.zeros_like(u)


def random_fields_torch(dim: int, n: int, seed: int, amp: float = 0.5, device="cuda"):
    """I.i.d. uniform fields in [-amp, amp] of shape (n,)*dim, float64,
    generated on a torch device from a seeded generator (for grids too large
    to build in host memory): (psi_re, psi_im, u, v)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    shape = (n,) * dim
    return tuple((2.0 * torch.rand(shape, generator=g, dtype=torch.float64, device=device) - 1.0)
                 * amp for _ in range(4))


def batched_instances(count: int = 64, seed: int = 20250213, steps: int = 500,
                      precision: int = FP64, sizes=None) -> List[Problem]:
    """Batched workload: `count` 2-D instances on [-16,16)^2, tau = 0.005,
    n drawn uniformly from {128, 192, ..., 1024}, (kappa1, kappa2, mu, gamma)
    ~ U[0.5, 2], Gaussian psi0/u0 with seeded centres in [-8, 8]^2."""
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = list(range(128, 1025, 64))
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        out.append(gaussian_problem(2, n, int(rng.integers(1 << 31)), -16.0, 16.0, 0.005, steps,
                                    precision))
        out[-1].name = f"batch{i}"
    return out


def batched3d_instances(count: int = 16, seed: int = 20250213, steps: int = 40,
                        precision: int = FP64, sizes=None) -> List[Problem]:
    """3-D batches: `count` instances on [-8,8)^3, tau = 0.002, n drawn
    uniformly from {64, 96, ..., 256} (the 3-D sizes of the serving mix),
    (kappa1, kappa2, mu, gamma) ~ U[0.5, 2], Gaussian psi0/u0 with seeded
    centres in [-4, 4]^3."""
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = list(range(64, 257, 32))
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        out.append(gaussian_problem(3, n, int(rng.integers(1 << 31)), -8.0, 8.0, 0.002, steps,
                                    precision))
        out[-1].name = f"batch3d{i}"
    return out


@dataclass
class Request:
    """One serving request: a problem and its arrival time in seconds."""

    rid: int
    arrival: float
    problem: Problem


def serving_requests(count: int, rate: float = 50.0, seed: int = 1, max_n=None,
                     max_steps: int = 2000, min_steps: int = 100,
                     arrays: bool = True) -> List[Request]:
    """Poisson arrivals (mean `rate` per second) mixing 1-D n in [256, 8192],
    2-D n in [128, 1024], 3-D n in [64, 256] (n even), steps ~ U[min, max],
    precision a fair coin; domains and tau as in the 1-D/2-D/3-D configs.
    `max_n` optionally caps n per dimension, e.g. {1: 8192, 2: 512, 3: 128}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    ranges = {1: (256, 8192), 2: (128, 1024), 3: (64, 256)}
    boxes = {1: (-20.0, 20.0, 0.01), 2: (-16.0, 16.0, 0.005), 3: (-8.0, 8.0, 0.002)}
    out = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        dim = int(rng.integers(1, 4))
        lo_n, hi_n = ranges[dim]
        if max_n is not None:
            hi_n = min(hi_n, max_n[dim])
        n = 2 * int(rng.integers(lo_n // 2, hi_n // 2 + 1))
        steps = int(rng.integers(min_steps, max_steps + 1))
        prec = int(rng.integers(0, 2))
        lo, hi, tau = boxes[dim]
        p = gaussian_problem(dim, n, int(rng.integers(1 << 31)), lo, hi, tau, steps, prec,
                             arrays=arrays)
        p.name = f"req{rid}"
        out.append(Request(rid, t, p))
    return out
