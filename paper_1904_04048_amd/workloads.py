"""Seeded synthetic inputs for the wave schemes.

This module only samples initial data and draws workload parameters.  It
holds none of the schemes' arithmetic, so both the GPU path and the CPU
oracle can be fed from it.  Everything here is analytic or drawn from a
seeded numpy PCG64 generator in a fixed order.

Grids cover [0, (nx-1) h] x [0, (ny-1) h] with nodes (i h, j h); arrays are
float64 of shape (ny, nx), x (index i) fastest.

The Courant numbers are fractions of the stability limits the paper states
(5-point: sqrt(2)/2, Sec. 6.1.1; 9-point: ~0.796, Sec. 6.2.1, read as
sqrt((3 - sqrt 3)/2); 13-point: 1/sqrt(2), Sec. 6.3).  They are written out
here as part of the workload recipe only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

P5, P9, P13 = 5, 9, 13
SCHEMES = (P5, P9, P13)
STABILITY_LIMIT = {
    P5: math.sqrt(2.0) / 2.0,
    P9: math.sqrt((3.0 - math.sqrt(3.0)) / 2.0),
    P13: 1.0 / math.sqrt(2.0),
}
RADIUS = {P5: 1, P9: 1, P13: 2}

Mode = Tuple[int, int, float, float]  # (p, q, amplitude of u0, amplitude of v0)


def sine_series(nx: int, ny: int, modes: List[Mode]):
    """u0, v0 = sum_m (A_m, B_m) sin(p_m pi i/(nx-1)) sin(q_m pi j/(ny-1))."""
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    u0 = np.zeros((ny, nx))
    v0 = np.zeros((ny, nx))
    for (p, q, A, B) in modes:
        e = np.outer(np.sin(q * math.pi * y / (ny - 1)), np.sin(p * math.pi * x / (nx - 1)))
        if A:
            u0 += A * e
        if B:
            v0 += B * e
    return u0, v0


def sine_series_matmul(nx: int, ny: int, modes: List[Mode]):
    """sine_series as two (ny x m) @ (m x nx) products: the same values up to
    the order of the sums, fast on the host for large batches."""
    p = np.array([m[0] for m in modes], dtype=np.float64)
    q = np.array([m[1] for m in modes], dtype=np.float64)
    a = np.array([m[2] for m in modes], dtype=np.float64)
    b = np.array([m[3] for m in modes], dtype=np.float64)
    sx = np.sin(np.outer(p, np.arange(nx)) * (math.pi / (nx - 1)))  # m x nx
    sy = np.sin(np.outer(np.arange(ny), q) * (math.pi / (ny - 1)))  # ny x m
    return sy @ (a[:, None] * sx), sy @ (b[:, None] * sx)


def sine_series_torch(nx: int, ny: int, modes: List[Mode], device):
    """sine_series sampled on the GPU (float64 tensors of shape (ny, nx))."""
    import torch
    x = torch.arange(nx, dtype=torch.float64, device=device)
    y = torch.arange(ny, dtype=torch.float64, device=device)
    u0 = torch.zeros((ny, nx), dtype=torch.float64, device=device)
    v0 = torch.zeros_like(u0)
    for (p, q, A, B) in modes:
        e = torch.outer(torch.sin(q * math.pi * y / (ny - 1)), torch.sin(p * math.pi * x / (nx - 1)))
        if A:
            u0.add_(e, alpha=A)
        if B:
            v0.add_(e, alpha=B)
    return u0, v0


def smooth_step(t):
    """C-infinity blend from 0 (t <= 0) to 1 (t >= 1)."""
    t = np.clip(np.asarray(t, dtype=np.float64), 0.0, 1.0)
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        a = np.where(t > 0, np.exp(-1.0 / np.where(t > 0, t, 1.0)), 0.0)
        b = np.where(t < 1, np.exp(-1.0 / np.where(t < 1, 1.0 - t, 1.0)), 0.0)
    return a / (a + b)


def gaussian_pulse(n_nodes: int, sigma: float = 0.02, r_in: float = 0.30, r_out: float = 0.45):
    """u0 = exp(-r^2 / (2 sigma^2)) * chi(r) about (0.5, 0.5) on [0,1]^2, v0 = 0.

    chi = 1 for r <= r_in, 0 for r >= r_out, smooth in between."""
    x = np.linspace(0.0, 1.0, n_nodes)
    X, Y = np.meshgrid(x, x)  # Y varies along axis 0 (rows = j)
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2)
    chi = smooth_step((r_out - r) / (r_out - r_in))
    u0 = np.exp(-r * r / (2.0 * sigma * sigma)) * chi
    return u0, np.zeros_like(u0)


def random_modes(rng: np.random.Generator, count: int = 8, kmax: int = 8) -> List[Mode]:
    """`count` distinct (p, q) in [1, kmax]^2, amplitudes N(0,1)/(p^2+q^2)
    drawn independently for u0 and v0."""
    seen = set()
    out = []
    while len(out) < count:
        p, q = (int(v) for v in rng.integers(1, kmax + 1, size=2))
        if (p, q) in seen:
            continue
        seen.add((p, q))
        k2 = float(p * p + q * q)
        A = float(rng.standard_normal()) / k2
        B = float(rng.standard_normal()) / k2
        out.append((p, q, A, B))
    return out


@dataclass
class Problem:
    """One solve: an (nx x ny) grid, spacing h, time step tau, wave speed c,
    scheme, number of time levels after u^0 (steps >= 1), and its data."""
    name: str
    nx: int
    ny: int
    h: float
    tau: float
    c: float
    scheme: int
    steps: int
    modes: List[Mode] = field(default_factory=list)  # empty: data given by `kind`
    kind: str = "sine"

    @property
    def lam(self) -> float:
        return self.c * self.tau / self.h

    @property
    def interior(self) -> int:
        return (self.nx - 2) * (self.ny - 2)

    @property
    def lup(self) -> int:
        """Grid-point updates of the whole solve: interior nodes x levels."""
        return self.interior * self.steps

    def data(self):
        if self.kind == "sine":
            return sine_series(self.nx, self.ny, self.modes)
        if self.kind == "gaussian":
            assert self.nx == self.ny
            return gaussian_pulse(self.nx)
        raise ValueError(self.kind)


def standing_wave(n: int) -> Problem:
    """5-point, 257^2-type benchmark: u0 = sin(pi x) sin(pi y), v0 = 0, tau = h/2."""
    h = 1.0 / n
    return Problem("standing-wave", n + 1, n + 1, h, 0.5 * h, 1.0, P5, 400, [(1, 1, 1.0, 0.0)])


def c1() -> Problem:
    """5-point FP64 on 257x257, h = 1/256, tau = h/2, 400 steps."""
    return standing_wave(256)


def c2(n: int = 4096, steps: int = 2000) -> Problem:
    """9-point on (n+1)^2 (4097^2), tau at 0.9 x the stability limit, 2000 steps;
    u0 = sin(2 pi x) sin(3 pi y), v0 = sin(pi x) sin(pi y)."""
    h = 1.0 / n
    lam = 0.9 * STABILITY_LIMIT[P9]
    return Problem("9pt-4097", n + 1, n + 1, h, lam * h, 1.0, P9, steps,
                   [(2, 3, 1.0, 0.0), (1, 1, 0.0, 1.0)])


def c3(n: int = 8192, steps: int = 3000) -> Problem:
    """13-point on (n+1)^2 (8193^2), lambda = 0.9 x limit, 3000 steps, Gaussian pulse."""
    h = 1.0 / n
    lam = 0.9 * STABILITY_LIMIT[P13]
    return Problem("13pt-gauss", n + 1, n + 1, h, lam * h, 1.0, P13, steps, [], "gaussian")


def draw_instance(rng: np.random.Generator, name: str, side_max: int, steps_max: int) -> Problem:
    """One batched/served instance: side log-uniform in [64, side_max] nodes,
    scheme uniform over {5, 9, 13}, lambda uniform in [0.3, 0.9] x limit,
    steps uniform in [100, steps_max], 8 random modes."""
    side = int(math.floor(math.exp(rng.uniform(math.log(64), math.log(side_max)))))
    side = max(64, min(side, side_max))
    scheme = SCHEMES[int(rng.integers(0, 3))]
    frac = float(rng.uniform(0.3, 0.9))
    steps = int(rng.integers(100, steps_max + 1))
    modes = random_modes(rng)
    n = side - 1
    h = 1.0 / n
    tau = frac * STABILITY_LIMIT[scheme] * h
    return Problem(name, side, side, h, tau, 1.0, scheme, steps, modes)


def c4(count: int = 512, seed: int = 0) -> List[Problem]:
    """Batch: `count` instances, sides in [64, 2048], steps in [100, 2000]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [draw_instance(rng, f"b{k}", 2048, 2000) for k in range(count)]


def c5_requests(count: int, seed: int = 1) -> List[Problem]:
    """Served requests: sides in [64, 4096], steps in [100, 5000]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [draw_instance(rng, f"r{k}", 4096, 5000) for k in range(count)]


def poisson_arrivals(count: int, qps: float, seed: int = 1):
    """Arrival times (s) of a Poisson process of rate qps."""
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


def complete_set(deg: int):
    """The complete monomial set of degree `deg` and its stencil, as inputs
    for a scheme built at run time (Sec. 4, eq. alpha and g): exponent pairs
    (a1, a2) with a1 + a2 <= deg, degree by degree, within a degree in the
    order of eq. g (a1 = a2 first, then a1 - a2 = 1, -1, 2, -2, ...), and
    the node (q(a1), q(a2)) of each, q(a) = (-1)^a floor((a + 1) / 2) being
    the inverse of eq. alpha.  Degree 6 gives the 28 monomials M*_{<=28}
    and their 28 nodes."""
    def q(a: int) -> int:
        return (-1) ** a * ((a + 1) // 2)

    exps: List[Tuple[int, int]] = []
    for d in range(deg + 1):
        pairs = [(a1, d - a1) for a1 in range(d + 1)]
        # position within the degree by eq. g: a1 - a2 for a1 > a2, a2 - a1 + 1 otherwise
        pairs.sort(key=lambda e: e[0] - e[1] if e[1] < e[0] else e[1] - e[0] + 1)
        exps += pairs
    return [(q(a1), q(a2)) for a1, a2 in exps], exps
