"""Seeded synthetic inputs shaped like the paper's test problems.

This module holds initial density fields and workload descriptions only; it
contains none of the step's arithmetic, so the GPU path and the CPU oracle
can both be fed from it.

Shapes follow Sec. IV of Guo, arXiv:2012.11075:
  - a flat liquid slab in vapour (Sec. IV.A) with the tanh profile of Eq. (38);
  - a circular droplet in vapour (Sec. IV.B) with the same radial profile;
  - a seeded uniform perturbation of the density (Sec. IV.A: rho (1 + eps r),
    r ~ U[-1, 1]); the workloads below also use an additive form.
Random numbers come from numpy's PCG64 (``default_rng(seed)``), drawn as one
(ny, nx) array in row-major order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import Optional

import numpy as np


@dataclass(frozen=True)
class Physics:
    """Lattice-unit parameters of one problem (tau: Eq. 2; beta, rho_l, rho_v:
    Eq. 36; kappa: mu = mu0 - kappa lap rho; rho0: Eq. 24)."""
    tau: float
    beta: float
    kappa: float
    rho_l: float
    rho_v: float
    rho0: float = 0.0

    @property
    def rho_ref(self) -> float:
        """Reference density of the shifted FP32 storage, (rho_l + rho_v)/2."""
        return 0.5 * (self.rho_l + self.rho_v)


@dataclass(frozen=True)
class Problem:
    """One initial-value problem on an nx x ny periodic lattice."""
    name: str
    nx: int
    ny: int
    physics: Physics
    shape: str                 # "slab_x", "slab_y" or "droplet"
    width: float = 5.0         # D of Eq. (38) used for the initial profile
    a: float = 0.0             # slab: first interface; droplet: radius
    b: float = 0.0             # slab: second interface
    noise: float = 0.0         # amplitude of the perturbation
    noise_kind: str = "add"    # "add": rho + eps r; "mul": rho (1 + eps r);
                               # "mul_normal": rho (1 + eps r) with r drawn
                               # per position along the slab normal
    seed: int = 0
    steps: int = 0

    def rho(self) -> np.ndarray:
        return initial_density(self)


def tanh_slab(n: int, rho_l: float, rho_v: float, y1: float, y2: float, width: float) -> np.ndarray:
    """Eq. (38): rho_v + (rho_l-rho_v)/2 [tanh(2(y-y1)/D) - tanh(2(y-y2)/D)]
    at y = 0..n-1."""
    y = np.arange(n, dtype=np.float64)
    return rho_v + 0.5 * (rho_l - rho_v) * (np.tanh(2.0 * (y - y1) / width) - np.tanh(2.0 * (y - y2) / width))


def tanh_droplet(nx: int, ny: int, rho_l: float, rho_v: float, radius: float, width: float,
                 cx: Optional[float] = None, cy: Optional[float] = None) -> np.ndarray:
    """Radial tanh profile of a droplet centred at (cx, cy) (default the node
    (nx//2, ny//2)): (rho_l+rho_v)/2 - (rho_l-rho_v)/2 tanh(2(r-R)/D), r the
    Euclidean distance (no wrap)."""
    cx = nx // 2 if cx is None else cx
    cy = ny // 2 if cy is None else cy
    x = np.arange(nx, dtype=np.float64)[None, :] - cx
    y = np.arange(ny, dtype=np.float64)[:, None] - cy
    r = np.sqrt(x * x + y * y)
    return 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (r - radius) / width)


def noise_field(seed: int, ny: int, nx: int) -> np.ndarray:
    """r ~ U[-1, 1] on the lattice, PCG64 seeded, row-major."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (ny, nx))


def initial_density(p: Problem) -> np.ndarray:
    ph = p.physics
    if p.shape == "slab_x":
        prof = tanh_slab(p.nx, ph.rho_l, ph.rho_v, p.a, p.b, p.width)
        rho = np.broadcast_to(prof[None, :], (p.ny, p.nx)).copy()
    elif p.shape == "slab_y":
        prof = tanh_slab(p.ny, ph.rho_l, ph.rho_v, p.a, p.b, p.width)
        rho = np.broadcast_to(prof[:, None], (p.ny, p.nx)).copy()
    elif p.shape == "droplet":
        rho = tanh_droplet(p.nx, p.ny, ph.rho_l, ph.rho_v, p.a, p.width)
    elif p.shape == "uniform":
        rho = np.full((p.ny, p.nx), ph.rho_l)
    else:
        raise ValueError("unknown shape %r" % p.shape)
    if p.noise:
        r = noise_field(p.seed, p.ny, p.nx)
        if p.noise_kind == "add":
            rho = rho + p.noise * r
        elif p.noise_kind == "mul":
            rho = rho * (1.0 + p.noise * r)
        elif p.noise_kind == "mul_normal":
            if p.shape == "slab_y":
                r = np.broadcast_to(noise_field(p.seed, p.ny, 1), (p.ny, p.nx))
            elif p.shape == "slab_x":
                r = np.broadcast_to(noise_field(p.seed, 1, p.nx), (p.ny, p.nx))
            else:
                raise ValueError("mul_normal noise needs a slab")
            rho = rho * (1.0 + p.noise * r)
        else:
            raise ValueError("unknown noise kind %r" % p.noise_kind)
    return np.ascontiguousarray(rho, dtype=np.float64)


# ------------------------------------------------------------------ workloads
BJ_PHYS = Physics(tau=1.0, beta=0.1, kappa=0.02, rho_l=1.0, rho_v=0.1)
THROUGHPUT_PHYS = Physics(tau=0.8, beta=0.1, kappa=0.02, rho_l=1.0, rho_v=0.01)
PAPER_PHYS = Physics(tau=0.85, beta=0.01, kappa=0.0128, rho_l=1.0, rho_v=0.2)
# The free-energy constants of Sec. IV (beta 0.01, kappa 0.0128) at other
# density ratios: the interface stays about 3.2 nodes wide at any ratio.
PAPER_BETA, PAPER_KAPPA = 0.01, 0.0128


def equilibrium_width(ph: Physics) -> float:
    """D of Eq. (38) for the double well, sqrt(8 kappa / beta) / (rho_l - rho_v)."""
    return math.sqrt(8.0 * ph.kappa / ph.beta) / (ph.rho_l - ph.rho_v)

# Flat interface, 200 x 4, slab x in [50, 150), 10,000 steps.
FLAT_200x4 = Problem("flat_200x4", 200, 4, BJ_PHYS, "slab_x", 5.0, 50.0, 150.0,
                     1e-3, "add", 1, 10_000)
# Stationary droplet, 256 x 256, radius 64 at the centre, 20,000 steps.
DROPLET_256 = Problem("droplet_256", 256, 256, BJ_PHYS, "droplet", 5.0, 64.0, 0.0,
                      1e-3, "add", 2, 20_000)
# Throughput grid: droplet of radius 1024 on 4096 x 4096, density ratio 100.
DROPLET_4096 = Problem("droplet_4096", 4096, 4096, THROUGHPUT_PHYS, "droplet", 5.0,
                       1024.0, 0.0, 1e-3, "mul", 3, 2_000)
# The same grid and droplet with the free-energy constants of Sec. IV: the
# state stays finite for the whole run (the configured constants give an
# interface 1.3 nodes wide, and the step diverges within ~100 steps).
FINITE_PHYS = Physics(tau=0.8, beta=PAPER_BETA, kappa=PAPER_KAPPA, rho_l=1.0, rho_v=0.01)
DROPLET_4096_FINITE = Problem("droplet_4096_finite", 4096, 4096, FINITE_PHYS, "droplet",
                              equilibrium_width(FINITE_PHYS), 1024.0, 0.0, 1e-3, "mul", 3, 2_000)
# The Sec. IV.B droplet constants (density ratio 5) on the 4096 x 4096 grid:
# a full-size case on which the standard LBE stays finite (at density ratio
# 100 it goes to negative densities within a few steps), used for the
# forcing-term comparison of Sec. II.
PAPER_DROPLET_4096 = Problem("paper_droplet_4096", 4096, 4096, PAPER_PHYS, "droplet", 4.0,
                             1024.0, 0.0, 1e-3, "mul", 5, 2_000)
# The same physics on a 512 x 512 crop (radius scaled), for parity at moderate size.
DROPLET_512_RATIO100 = Problem("droplet_512_ratio100", 512, 512, THROUGHPUT_PHYS, "droplet",
                               5.0, 128.0, 0.0, 1e-3, "mul", 3, 1_000)
# The paper's own runs (Sec. IV.A, IV.B).
# Sec. IV.A puts the liquid on the rows 25 <= y <= 75: the interfaces of
# Eq. (38) sit half-way between the last liquid and the first vapour row,
# y1 = 24.5 and y2 = 75.5.  It writes the perturbed profile as
# rho(y) = (1 + eps r) rho_0(y): one random number per row.
PAPER_FLAT = Problem("paper_flat_21x101", 21, 101, PAPER_PHYS, "slab_y", 4.0, 24.5, 75.5,
                     1e-2, "mul_normal", 11, 0)
PAPER_DROPLET = Problem("paper_droplet_100", 100, 100, PAPER_PHYS, "droplet", 4.0, 25.0, 0.0,
                        1e-2, "mul", 12, 0)

PROBLEMS = {p.name: p for p in [FLAT_200x4, DROPLET_256, DROPLET_4096, DROPLET_4096_FINITE,
                                PAPER_DROPLET_4096, DROPLET_512_RATIO100,
                                PAPER_FLAT, PAPER_DROPLET]}


def separable_density(nx: int, ny: int, seed: int) -> np.ndarray:
    """rho(y, x) = a(y) + b(x) for lattices too large for the tanh profiles:
    smooth periodic profiles plus per-row and per-column noise, so the field
    has grid-scale structure in both directions; values in [0.16, 0.94]."""
    rng = np.random.default_rng(seed)
    a = 0.55 + 0.35 * np.sin(2 * np.pi * 3 * np.arange(ny) / ny) + 0.01 * rng.uniform(-1, 1, ny)
    b = 0.02 * np.sin(2 * np.pi * 5 * np.arange(nx) / nx) + 0.01 * rng.uniform(-1, 1, nx)
    return a[:, None] + b[None, :]


def batch_instances(count: int = 512, seed: int = 4, side_lo: int = 32, side_hi: int = 512,
                    steps: int = 5_000) -> list:
    """Uneven independent problems for one batched launch: side log-uniform on
    [side_lo, side_hi]; droplet (radius 0.15-0.35 of the side) or a slab of
    half the side with probability 1/2; density ratio 10 or 100; tau uniform
    on [0.6, 1.2]; the free-energy constants of Sec. IV (beta 0.01, kappa
    0.0128); tanh profile of the equilibrium width; multiplicative noise 1e-3.
    The WB step has a growing grid-scale mode in bulk liquid for tau below
    about 0.8, so the instances drawn there diverge whatever the ratio."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        side = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
        ratio = 10.0 if rng.uniform() < 0.5 else 100.0
        tau = float(rng.uniform(0.6, 1.2))
        ph = Physics(tau=tau, beta=PAPER_BETA, kappa=PAPER_KAPPA, rho_l=1.0, rho_v=1.0 / ratio)
        w = equilibrium_width(ph)
        if rng.uniform() < 0.5:
            radius = float(rng.uniform(0.15, 0.35)) * side
            prob = Problem("batch%03d" % k, side, side, ph, "droplet", w, radius, 0.0,
                           1e-3, "mul", seed * 100_000 + k, steps)
        else:
            prob = Problem("batch%03d" % k, side, side, ph, "slab_x", w, side / 4.0,
                           3.0 * side / 4.0, 1e-3, "mul", seed * 100_000 + k, steps)
        out.append(prob)
    return out


@dataclass(frozen=True)
class Request:
    """One run-to-equilibrium request of a served stream."""
    rid: int
    arrival: float             # seconds after the stream starts
    problem: Problem
    precision: str             # "fp32s" or "fp64"
    tol: float                 # retire when max|u| < tol
    step_cap: int
    scheme: str = "well_balanced"  # the scheme the request is stepped with
    force_stencil: int = 0         # 1: the fourth-order gradients of the force


def request_stream(n: int, rate_hz: float, seed: int = 5, side_lo: int = 64,
                   side_hi: int = 2048, step_cap: int = 50_000, fp64_fraction: float = 0.1) -> list:
    """Poisson arrivals at rate_hz; side log-uniform on [side_lo, side_hi];
    droplet or slab; density ratio log-uniform on [10, 1000]; tau 1 and the
    free-energy constants of Sec. IV; tanh profile of the equilibrium width;
    FP32-shifted by default (tolerance 1e-6) and FP64 with probability
    fp64_fraction (tolerance 1e-10)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += float(rng.exponential(1.0 / rate_hz))
        side = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
        ratio = math.exp(rng.uniform(math.log(10.0), math.log(1000.0)))
        ph = Physics(tau=1.0, beta=PAPER_BETA, kappa=PAPER_KAPPA, rho_l=1.0, rho_v=1.0 / ratio)
        w = equilibrium_width(ph)
        if rng.uniform() < 0.5:
            prob = Problem("req%05d" % k, side, side, ph, "droplet", w,
                           float(rng.uniform(0.15, 0.35)) * side, 0.0, 1e-3, "mul", seed * 1_000_000 + k)
        else:
            prob = Problem("req%05d" % k, side, side, ph, "slab_x", w, side / 4.0, 3.0 * side / 4.0,
                           1e-3, "mul", seed * 1_000_000 + k)
        fp64 = rng.uniform() < fp64_fraction
        out.append(Request(k, t, prob, "fp64" if fp64 else "fp32s", 1e-10 if fp64 else 1e-6, step_cap))
    return out


def droplet3_density(nx: int, ny: int, nz: int, ph: Physics, radius: float, width: float,
                     noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """3-D droplet: the radial tanh profile of Eq. (38) about the node
    (nx//2, ny//2, nz//2), shape (nz, ny, nx), with an optional
    multiplicative perturbation (1 + noise r), r ~ U[-1, 1] (PCG64, seeded)."""
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - nx // 2) ** 2 + (y - ny // 2) ** 2 + (z - nz // 2) ** 2)
    rho = 0.5 * (ph.rho_l + ph.rho_v) - 0.5 * (ph.rho_l - ph.rho_v) * np.tanh(2.0 * (r - radius) / width)
    if noise:
        rho = rho * (1.0 + noise * np.random.default_rng(seed).uniform(-1.0, 1.0, (nz, ny, nx)))
    return np.ascontiguousarray(rho)


@dataclass(frozen=True)
class Problem3:
    """One 3-D initial-value problem: a droplet of the given radius about the
    node (nx//2, ny//2, nz//2) of an nx x ny x nz periodic lattice, on the
    D3Q19 (q3 = 19) or D3Q27 (q3 = 27) lattice."""
    name: str
    nx: int
    ny: int
    nz: int
    physics: Physics
    radius: float
    width: float
    noise: float = 0.0
    seed: int = 0
    q3: int = 19

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def rho(self) -> np.ndarray:
        return droplet3_density(self.nx, self.ny, self.nz, self.physics, self.radius, self.width,
                                self.noise, self.seed)


def request_stream3(n: int, rate_hz: float, seed: int = 7, side_lo: int = 16, side_hi: int = 96,
                    step_cap: int = 2_000) -> list:
    """3-D requests: Poisson arrivals at rate_hz; cubic side log-uniform on
    [side_lo, side_hi]; a droplet (radius 0.2-0.3 of the side) on D3Q19 or
    D3Q27 with equal probability; density ratio 10, tau 1 and the
    free-energy constants of Sec. IV; FP32-shifted (tolerance 1e-6) or FP64
    (1e-10) with equal probability; multiplicative noise 1e-3."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += float(rng.exponential(1.0 / rate_hz))
        side = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
        ph = Physics(tau=1.0, beta=PAPER_BETA, kappa=PAPER_KAPPA, rho_l=1.0, rho_v=0.1)
        q3 = 27 if rng.uniform() < 0.5 else 19
        prob = Problem3("req3d%05d" % k, side, side, side, ph,
                        float(rng.uniform(0.2, 0.3)) * side, equilibrium_width(ph), 1e-3,
                        seed * 1_000_000 + k, q3)
        fp64 = rng.uniform() < 0.5
        out.append(Request(k, t, prob, "fp64" if fp64 else "fp32s", 1e-10 if fp64 else 1e-6,
                           step_cap))
    return out


# 3-D throughput lattice: 256^3 D3Q19 droplet of radius 64, the free-energy
# constants of Sec. IV at density ratio 10, tau 1 (a finite, relaxing state).
PHYS3 = Physics(tau=1.0, beta=PAPER_BETA, kappa=PAPER_KAPPA, rho_l=1.0, rho_v=0.1)
DROPLET3_SIDE, DROPLET3_RADIUS = 256, 64.0


def with_size(p: Problem, nx: int, ny: int, **kw) -> Problem:
    """The same problem on another lattice (interfaces scaled with the side)."""
    sx = nx / p.nx
    return replace(p, nx=nx, ny=ny, a=p.a * sx, b=p.b * sx, **kw)
