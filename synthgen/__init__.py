"""Seeded synthetic inputs shared by the oracle and the GPU library's callers.

This module only draws random numbers and describes workloads: it holds none of
the tiling method's arithmetic and none of the per-point operations.  Both the
oracle (``oracle/``) and the product callers (``bench.py``, tests) take their
inputs from here, so the two sides see identical data.

Generator: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  The n-th output (n >= 1) of a
stream with state ``s0`` is ``mix(s0 + n * GAMMA)``, so the same stream can be
drawn sequentially (structure) or vectorised by counter (bulk data).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
DATA_SALT = 0xD1B54A32D192ED03  # data stream state = seed ^ DATA_SALT


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * M1) & MASK
    z = ((z ^ (z >> 27)) * M2) & MASK
    return z ^ (z >> 31)


class SplitMix64:
    """Sequential SplitMix64 stream."""

    def __init__(self, seed: int):
        self.state = seed & MASK

    def next(self) -> int:
        self.state = (self.state + GAMMA) & MASK
        return _mix(self.state)

    def unit(self) -> float:
        """Uniform double in [0,1): top 53 bits times 2^-53."""
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)

    def uniform(self, a: float, b: float) -> float:
        return a + (b - a) * self.unit()

    def randint(self, n: int) -> int:
        return self.next() % n


def splitmix_block(state0: int, first: int, count: int) -> np.ndarray:
    """Outputs number first+1 .. first+count of the stream with state ``state0``
    (vectorised counter form), as uint64."""
    with np.errstate(over="ignore"):
        n = np.arange(first + 1, first + count + 1, dtype=np.uint64)
        z = np.uint64(state0 & MASK) + n * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        return z ^ (z >> np.uint64(31))


def uniform_block(state0: int, first: int, count: int, a: float, b: float) -> np.ndarray:
    u = (splitmix_block(state0, first, count) >> np.uint64(11)).astype(np.float64)
    u *= 1.0 / 9007199254740992.0
    return a + (b - a) * u


# --------------------------------------------------------------------------
# Stencils (offsets listed in the order weights are drawn and applied)
# --------------------------------------------------------------------------

def star(ndim: int, radius: int) -> List[Tuple[int, ...]]:
    """Centre, then for each axis (x, y, z) and each distance 1..radius the
    points -r, +r.  5/9 points in 2D, 7/13 points in 3D."""
    pts = [tuple([0] * ndim)]
    for ax in range(ndim):
        for r in range(1, radius + 1):
            for s in (-r, r):
                p = [0] * ndim
                p[ax] = s
                pts.append(tuple(p))
    return pts


# --------------------------------------------------------------------------
# Synthetic loop chains (2D and 3D weighted-sum chains)
# --------------------------------------------------------------------------

@dataclass
class ChainInput:
    dat: int
    stencil: List[Tuple[int, ...]]


@dataclass
class ChainLoop:
    out: int
    inputs: List[ChainInput]
    weights: List[float]  # input-major, stencil point order


@dataclass
class SyntheticChain:
    ndim: int
    n: int
    halo: int
    ndat: int
    loops: List[ChainLoop]
    seed: int
    reduce_last: bool = False

    @property
    def shape_alloc(self) -> Tuple[int, ...]:
        """Padded array shape, slowest axis first (z, y, x)."""
        return tuple([self.n + 2 * self.halo] * self.ndim)

    def last_written(self) -> int:
        return self.loops[-1].out

    def cell_updates(self) -> int:
        return len(self.loops) * self.n ** self.ndim


def make_chain(ndim: int, n: int, ndat: int, nloops: int, seed: int,
               halo: int = 2, reduce_last: bool = False) -> SyntheticChain:
    """Chain structure drawn from SplitMix64(seed), per loop in this order:
    output = randint(ndat); k = min(2 + randint(3), ndat - 1) distinct inputs != output
    (partial Fisher-Yates over the remaining datasets); per input a stencil
    (radius 1 star if randint(2) == 0 else radius 2 star); then one weight per
    (input, stencil point) uniform in [-0.25, 0.25)."""
    rng = SplitMix64(seed)
    loops = []
    for _ in range(nloops):
        o = rng.randint(ndat)
        k = min(2 + rng.randint(3), ndat - 1)
        pool = [d for d in range(ndat) if d != o]
        for i in range(k):
            j = i + rng.randint(len(pool) - i)
            pool[i], pool[j] = pool[j], pool[i]
        ins = []
        for i in range(k):
            radius = 1 if rng.randint(2) == 0 else 2
            ins.append(ChainInput(pool[i], star(ndim, radius)))
        w = []
        for ci in ins:
            for _p in ci.stencil:
                w.append(rng.uniform(-0.25, 0.25))
        loops.append(ChainLoop(o, ins, w))
    return SyntheticChain(ndim, n, halo, ndat, loops, seed, reduce_last)


def chain_data(ch: SyntheticChain, dtype=np.float64) -> List[np.ndarray]:
    """Initial dataset values, halos included: uniform [-1,1) from the data
    stream (state seed ^ DATA_SALT), dataset-major then row-major (x fastest)."""
    shape = ch.shape_alloc
    size = int(np.prod(shape))
    state0 = (ch.seed ^ DATA_SALT) & MASK
    out = []
    for d in range(ch.ndat):
        a = uniform_block(state0, d * size, size, -1.0, 1.0).reshape(shape)
        out.append(np.ascontiguousarray(a.astype(dtype)))
    return out


# Workload presets (sizes of the paper-shaped synthetic workloads)
def chain_2d(n: int = 4096, seed: int = 1, ndat: int = 12, nloops: int = 40) -> SyntheticChain:
    return make_chain(2, n, ndat, nloops, seed)


def chain_3d(n: int = 384, seed: int = 2, ndat: int = 25, nloops: int = 60) -> SyntheticChain:
    return make_chain(3, n, ndat, nloops, seed, reduce_last=True)


# --------------------------------------------------------------------------
# Heat-conduction (TeaLeaf-style) problem inputs
# --------------------------------------------------------------------------

@dataclass
class HeatProblem:
    ndim: int
    n: int
    seed: int
    halo: int = 2
    dt: float = 0.004
    density: np.ndarray = field(default=None, repr=False)  # interior, (y,x) or (z,y,x)
    energy: np.ndarray = field(default=None, repr=False)

    @property
    def dx(self) -> float:
        return 1.0 / self.n

    @property
    def rx(self) -> float:
        return self.dt / (self.dx * self.dx)


def heat_problem(n: int = 256, seed: int = 0, ndim: int = 2) -> HeatProblem:
    """Density uniform [0.1,1.0) for every interior cell, then energy uniform
    [1,2) for every interior cell, from one sequential counter stream
    (state = seed), row-major with x fastest."""
    cells = n ** ndim
    shape = tuple([n] * ndim)
    rho = uniform_block(seed, 0, cells, 0.1, 1.0).reshape(shape)
    e = uniform_block(seed, cells, cells, 1.0, 2.0).reshape(shape)
    return HeatProblem(ndim, n, seed, density=np.ascontiguousarray(rho),
                       energy=np.ascontiguousarray(e))


def batch_sizes(count: int = 512, seed: int = 3, lo: int = 64, hi: int = 1024) -> List[Tuple[int, int]]:
    """(n, instance seed) per batched solve: n = round(exp(U[ln lo, ln hi)))."""
    rng = SplitMix64(seed)
    out = []
    for _ in range(count):
        u = rng.uniform(math.log(lo), math.log(hi))
        out.append((int(round(math.exp(u))), rng.next()))
    return out


@dataclass
class Request:
    arrival: float
    ndim: int
    n: int
    seed: int


def serving_requests(rate: float = 200.0, duration: float = 60.0, seed: int = 4) -> List[Request]:
    """Poisson arrivals (exponential gaps of mean 1/rate), each a 2D
    (n log-uniform 128..2048) or 3D (n log-uniform 64..256) solve, 50/50."""
    rng = SplitMix64(seed)
    t = 0.0
    out = []
    while True:
        t += -math.log(1.0 - rng.unit()) / rate
        if t >= duration:
            break
        if rng.randint(2) == 0:
            nd, lo, hi = 2, 128, 2048
        else:
            nd, lo, hi = 3, 64, 256
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append(Request(t, nd, n, rng.next()))
    return out


# --------------------------------------------------------------------------
# Compressible Euler (Taylor-Green vortex) initial state
# --------------------------------------------------------------------------

def taylor_green(n: int, halo: int = 2, gamma: float = 1.4, mach: float = 0.1) -> List[np.ndarray]:
    """Conserved variables (rho, rho u, rho v, rho w, E) of the Taylor-Green
    vortex on [0, 2pi)^3 at cell centres (i + 1/2) h, evaluated on the padded
    array (ghost cells take the same formula at their own coordinates).
    Arrays are (z, y, x)."""
    h = 2.0 * math.pi / n
    c = (np.arange(-halo, n + halo, dtype=np.float64) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = 1.0 / (gamma * mach * mach) + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    rho = np.ones_like(u)
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return [np.ascontiguousarray(a) for a in (rho, rho * u, rho * v, rho * w, E)]


# --------------------------------------------------------------------------
# Jacobi iteration of the 2D heat equation (the paper's baseline benchmark)
# --------------------------------------------------------------------------

# One explicit heat-equation step u' = u + nu (sum of the four neighbours - 4u)
# with nu = 1/5: every one of the five points weighs 0.2 (the centre weight
# 1 - 4 nu is 0.2 as well).  Points: centre, then -x, +x, -y, +y.
JACOBI_POINTS = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
JACOBI_WEIGHTS = [0.2] * 5


def jacobi_field(n: int, seed: int = 5) -> np.ndarray:
    """(n + 2)^2 values (y, x), the one-cell Dirichlet layer included: uniform
    [0, 1) from the data stream (state seed ^ DATA_SALT), row-major with x
    fastest.  The layer keeps these values for the whole run."""
    state0 = (seed ^ DATA_SALT) & MASK
    size = (n + 2) * (n + 2)
    return np.ascontiguousarray(uniform_block(state0, 0, size, 0.0, 1.0).reshape(n + 2, n + 2))


def jacobi_mode(n: int, k: int, l: int) -> np.ndarray:
    """(n + 2)^2 values (y, x): sin(pi k (x+1)/(n+1)) sin(pi l (y+1)/(n+1))
    on the interior x, y in [0, n), and exactly 0 on the Dirichlet layer
    (x or y = -1 or n)."""
    c = np.arange(-1, n + 1, dtype=np.float64) + 1.0
    sx = np.sin(math.pi * k * c / (n + 1))
    sy = np.sin(math.pi * l * c / (n + 1))
    a = np.outer(sy, sx)
    a[0, :] = a[-1, :] = 0.0
    a[:, 0] = a[:, -1] = 0.0
    return np.ascontiguousarray(a)
