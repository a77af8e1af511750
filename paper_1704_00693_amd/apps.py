"""Workload drivers written against the tilechain ABI (user code of the library,
as the paper's applications are user code of OPS): the synthetic
weighted-sum chains, the Jacobi heat-equation iteration, the heat-conduction
PPCG solve, the compressible-Euler step and the request-serving loop.

Nothing here computes on the host beyond the scalar recurrences of the solver
(CG's alpha and beta, the Chebyshev coefficients); every loop is recorded with
``tc_par_loop`` (or several at once with ``tc_par_loops``) and runs in the
library's HIP kernels.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import (TC_F32, TC_F64, TC_RED_MAX, TC_RED_SUM, Context, LoopBatch)


# ---------------------------------------------------------------------------
# synthetic weighted-sum chains
# ---------------------------------------------------------------------------
class ChainRunner:
    """Declares a chain's datasets and stencils once; ``record()`` enqueues
    its loops (and the final sum reduction if the chain has one)."""

    def __init__(self, ctx: Context, chain, data: Optional[Sequence[np.ndarray]] = None, dtype: int = TC_F64):
        self.ctx, self.chain = ctx, chain
        nd, n, h = chain.ndim, chain.n, chain.halo
        self.blk = ctx.tc_decl_block(nd, "chain")
        self.dats = []
        for d in range(chain.ndat):
            init = None if data is None else data[d]
            self.dats.append(ctx.tc_decl_dat(self.blk, [n] * nd, [h] * nd, [h] * nd, init, dtype, f"d{d}"))
        self.stencils: Dict[Tuple, int] = {}
        self.centre = self.stencil([tuple([0] * nd)])
        self.red = ctx.tc_decl_reduction(TC_RED_SUM, "sum") if chain.reduce_last else None
        self.range = [v for _ in range(nd) for v in (0, n)]

    def stencil(self, pts) -> int:
        key = tuple(tuple(p) for p in pts)
        if key not in self.stencils:
            self.stencils[key] = self.ctx.tc_decl_stencil(list(key))
        return self.stencils[key]

    def record(self):
        for i, lp in enumerate(self.chain.loops):
            args = [(self.dats[lp.out], self.centre, "W")]
            args += [(self.dats[ci.dat], self.stencil(ci.stencil), "R") for ci in lp.inputs]
            self.ctx.tc_par_loop("WSUM", self.blk, self.range, args, lp.weights, name=f"loop{i}")
        if self.red is not None:
            self.ctx.tc_par_loop("SUM", self.blk, self.range,
                                 [(self.dats[self.chain.last_written()], self.centre, "R"), ("red", self.red)],
                                 name="sum")

    def run(self) -> Optional[float]:
        """Record the chain and execute it (the reduction fetch flushes)."""
        self.record()
        if self.red is not None:
            return self.ctx.tc_reduction_result(self.red)
        self.ctx.tc_flush()
        return None

    def read(self, d: int) -> np.ndarray:
        return self.ctx.tc_dat_read(self.dats[d])


# ---------------------------------------------------------------------------
# Jacobi iteration of the 2D heat equation
# ---------------------------------------------------------------------------
class JacobiRunner:
    """The Jacobi benchmark of the paper (Section 5; measured in Section 6.2):
    a five-point weighted stencil applied over the interior of an n^2 field
    whose one-cell Dirichlet layer is never written.

    Two datasets a and b, both holding the initial field (layer included).
    ``record(iters)`` enqueues iterations without executing them:

    * copy variant: b = stencil(a), then a second loop copies b into a;
    * non-copy variant: a -> b and b -> a alternately, no copy.

    The copy is recorded as a one-point weighted sum with weight 1, so that it
    can share a fused group with the stencil loops: fma(1, v, 0) is v for
    every value except -0, which becomes +0.

    ``points`` are the stencil's (x, y) offsets, ``weights`` one weight per
    point, applied in that order."""

    def __init__(self, ctx: Context, u0: np.ndarray, points: Sequence[Sequence[int]], weights: Sequence[float],
                 copy: bool, dtype: int = TC_F64):
        self.ctx, self.copy = ctx, copy
        self.n = n = u0.shape[0] - 2
        if u0.shape != (n + 2, n + 2):
            raise ValueError(f"u0 must be (n+2, n+2), got {u0.shape}")
        self.blk = ctx.tc_decl_block(2, "jacobi")
        self.a = ctx.tc_decl_dat(self.blk, [n, n], [1, 1], [1, 1], u0, dtype, "a")
        self.b = ctx.tc_decl_dat(self.blk, [n, n], [1, 1], [1, 1], u0, dtype, "b")
        self.S = ctx.tc_decl_stencil([tuple(p) for p in points])
        self.S_c = ctx.tc_decl_stencil([(0, 0)])
        self.w = [float(v) for v in weights]
        self.range = [0, n, 0, n]
        self.done = 0  # iterations recorded so far (the non-copy variant alternates across calls)

    def record(self, iters: int):
        c = self.ctx
        for _ in range(iters):
            t = self.done
            if self.copy:
                c.tc_par_loop("WSUM", self.blk, self.range, [(self.b, self.S_c, "W"), (self.a, self.S, "R")],
                              self.w, name="jacobi")
                c.tc_par_loop("WSUM", self.blk, self.range, [(self.a, self.S_c, "W"), (self.b, self.S_c, "R")],
                              [1.0], name="copy")
            else:
                src, dst = (self.a, self.b) if t % 2 == 0 else (self.b, self.a)
                c.tc_par_loop("WSUM", self.blk, self.range, [(dst, self.S_c, "W"), (src, self.S, "R")], self.w,
                              name="jacobi")
            self.done += 1

    def run(self, iters: int):
        """Record ``iters`` iterations and execute them as one chain."""
        self.record(iters)
        self.ctx.tc_flush()

    def current(self) -> int:
        """The dataset that holds the latest field."""
        return self.a if self.copy or self.done % 2 == 0 else self.b

    def result(self) -> np.ndarray:
        """The latest field, (n + 2)^2 with the layer (flushes pending loops)."""
        return self.ctx.tc_dat_read(self.current())


# ---------------------------------------------------------------------------
# heat conduction, PPCG
# ---------------------------------------------------------------------------
def chebyshev_coefs(lmin: float, lmax: float, steps: int):
    """Chebyshev iteration scalars for the spectrum [lmin, lmax]:
    theta, delta, and (alpha_j, beta_j) for j = 1..steps-1 with rho_0 =
    1/sigma, rho_j = 1/(2 sigma - rho_{j-1}), alpha_j = rho_j rho_{j-1},
    beta_j = 2 rho_j / delta."""
    theta = (lmax + lmin) / 2.0
    delta = (lmax - lmin) / 2.0
    sigma = theta / delta
    r_old = 1.0 / sigma
    al, be = [], []
    for _ in range(1, steps):
        r_new = 1.0 / (2.0 * sigma - r_old)
        al.append(r_new * r_old)
        be.append(2.0 * r_new / delta)
        r_old = r_new
    return theta, delta, al, be


class HeatSolver:
    """Implicit heat-conduction step solved with PPCG (CG preconditioned by a
    fixed number of Chebyshev steps), every loop through the tilechain ABI.

    The per-iteration chain between two reduction fetches is what the
    library tiles: chain A = p update, ghost fill of p, w = A p with p.w;
    chain B = x, r update, preconditioner (ghost fill of sd, P1, P2 per
    inner step), r.z and r.r."""

    FIELDS = ("rho", "e", "u0", "u", "kx", "ky", "kz", "r", "p", "w", "z", "rt", "sd")

    def __init__(self, ctx: Context, density: np.ndarray, energy: np.ndarray, dt: float = 0.004, halo: int = 2,
                 dtype: int = TC_F64):
        self.ctx = ctx
        self.D = density.ndim
        self.n = n = density.shape[0]
        self.h = halo
        self.rx = dt * n * n
        D = self.D
        self.blk = ctx.tc_decl_block(D, "heat")
        shape = tuple([n + 2 * halo] * D)
        inner = tuple([slice(halo, halo + n)] * D)
        self.f: Dict[str, int] = {}
        names = [k for k in self.FIELDS if not (k == "kz" and D < 3)]
        for k in names:
            init = None
            if k in ("rho", "e"):
                init = np.zeros(shape)
                init[inner] = density if k == "rho" else energy
            self.f[k] = ctx.tc_decl_dat(self.blk, [n] * D, [halo] * D, [halo] * D, init, dtype, k)
        z = [0] * D

        def unit(d, s):
            p = [0] * D
            p[d] = s
            return tuple(p)

        self.S_c = ctx.tc_decl_stencil([tuple(z)])
        self.S_star = ctx.tc_decl_stencil([tuple(z)] + [unit(d, s) for d in range(D) for s in (-1, 1)])
        self.S_kface = [ctx.tc_decl_stencil([tuple(z), unit(d, 1)]) for d in range(D)]
        self.S_rho = ctx.tc_decl_stencil([tuple(z)] + [unit(d, -1) for d in range(D)])
        self.S_reflect = {}
        for axis in range(D):
            for side in (0, 1):
                sgn = 1 if side == 0 else -1
                self.S_reflect[(axis, side)] = ctx.tc_decl_stencil(
                    [tuple(z), unit(axis, sgn * 1), unit(axis, sgn * 3)])
        self.r_sum = [ctx.tc_decl_reduction(TC_RED_SUM, f"s{i}") for i in range(3)]
        self.r_max = ctx.tc_decl_reduction(TC_RED_MAX, "lmax")
        self.interior = [v for _ in range(D) for v in (0, n)]
        self._batches: Dict[tuple, LoopBatch] = {}

    # -- loop helpers --------------------------------------------------------
    def K(self):
        return [(self.f[k], self.S_kface[d], "R") for d, k in enumerate(["kx", "ky", "kz"][: self.D])]

    def halo_fill(self, name: str):
        n, h, D = self.n, self.h, self.D
        for axis in range(D):
            for side in (0, 1):
                rng = []
                for d in range(D):
                    if d == axis:
                        rng += [-h, 0] if side == 0 else [n, n + h]
                    elif d < axis:
                        rng += [-h, n + h]
                    else:
                        rng += [0, n]
                self.ctx.tc_par_loop("HALO_REFLECT", self.blk, rng,
                                     [(self.f[name], self.S_reflect[(axis, side)], "RW")], [axis, side, n],
                                     name=f"halo_{name}_{axis}{side}")

    def loop(self, op, args, params=(), rng=None, name=""):
        self.ctx.tc_par_loop(op, self.blk, rng or self.interior, args, params, name=name or op)

    def F(self, k, acc, st=None):
        return (self.f[k], self.S_c if st is None else st, acc)

    # -- solver ---------------------------------------------------------------
    def setup(self) -> float:
        D = self.D
        self.halo_fill("rho")
        self.loop("TEA_INIT", [self.F("rho", "R"), self.F("e", "R"), self.F("u0", "W"), self.F("u", "W")])
        kout = [self.F(k, "W") for k in ["kx", "ky", "kz"][:D]]
        self.loop("TEA_K", [self.F("rho", "R", self.S_rho)] + kout, [self.rx],
                  rng=[v for _ in range(D) for v in (0, self.n + 1)])
        self.loop("TEA_GERSH", self.K() + [("red", self.r_max)])
        return self.ctx.tc_reduction_result(self.r_max)

    def dot(self, a, b, red):
        self.loop("DOT", [self.F(a, "R"), self.F(b, "R"), ("red", red)], name=f"dot_{a}{b}")

    def precondition(self, theta, al, be, steps):
        self.loop("TEA_PRECON_INIT", [self.F("r", "R"), self.F("rt", "W"), self.F("sd", "W"), self.F("z", "W")],
                  [theta])
        for j in range(1, steps + 1):
            self.halo_fill("sd")
            self.loop("TEA_P1", self.K() + [self.F("sd", "R", self.S_star), self.F("rt", "RW"), self.F("z", "RW")])
            if j < steps:
                self.loop("TEA_P2", [self.F("sd", "RW"), self.F("rt", "R")], [al[j - 1], be[j - 1]])

    def solve(self, outer: int = 50, inner: int = 10, tol: Optional[float] = None, max_iter: int = 10000):
        """Same sequence of loops and reductions as the FP64 reference PPCG:
        exactly ``outer`` iterations when tol is None, else stop at
        sqrt(r.r) <= tol ||b||.  Returns a dict of scalars and histories."""
        ctx = self.ctx
        lmax = self.setup()
        theta, delta, al, be = chebyshev_coefs(1.0, lmax, inner)
        s0, s1, s2 = self.r_sum
        self.dot("u0", "u0", s0)
        bnorm = math.sqrt(ctx.tc_reduction_result(s0))
        self.halo_fill("u")
        self.loop("TEA_RESID", self.K() + [self.F("u", "R", self.S_star), self.F("u0", "R"), self.F("r", "W")])
        self.precondition(theta, al, be, inner)
        self.loop("COPY", [self.F("p", "W"), self.F("z", "R")])
        self.dot("r", "z", s0)
        rz = ctx.tc_reduction_result(s0)
        hist = {"rr": [], "rz": [], "pw": []}
        it = 0
        limit = outer if tol is None else max_iter

        def cg_p():
            self.loop("TEA_CG_P", [self.F("p", "RW"), self.F("z", "R")], [0.0])

        def matvec():
            self.halo_fill("p")
            self.loop("TEA_MATVEC_DOT", self.K() + [self.F("p", "R", self.S_star), self.F("w", "W"), ("red", s0)])

        def update():
            self.loop("TEA_CG_UPDATE", [self.F("u", "RW"), self.F("r", "RW"), self.F("p", "R"), self.F("w", "R")],
                      [0.0])
            self.precondition(theta, al, be, inner)
            self.dot("r", "z", s1)
            self.dot("r", "r", s2)

        # the loops between two reduction fetches are the same every
        # iteration: each chain is recorded with one call, only the CG scalar
        # (beta of the p update, alpha of the x, r update) changing
        chain_a0 = self._batch(("a0",), matvec)
        chain_a = self._batch(("a",), lambda: (cg_p(), matvec()))
        chain_b = self._batch(("b", inner, theta, tuple(al), tuple(be)), update)
        beta = None
        while it < limit:
            if beta is None:
                chain_a0.record()
            else:
                chain_a.params[chain_a.first_param[0]] = beta
                chain_a.record()
            pw = ctx.tc_reduction_result(s0)
            alpha = rz / pw
            chain_b.params[chain_b.first_param[0]] = alpha
            chain_b.record()
            rz_new = ctx.tc_reduction_result(s1)
            rr = ctx.tc_reduction_result(s2)
            it += 1
            hist["rr"].append(rr)
            hist["rz"].append(rz_new)
            hist["pw"].append(pw)
            if tol is not None and math.sqrt(rr) <= tol * bnorm:
                beta = None
                break
            beta = rz_new / rz
            rz = rz_new
        if beta is not None:  # the last p update, as the plain iteration makes it
            self.loop("TEA_CG_P", [self.F("p", "RW"), self.F("z", "R")], [beta])
        ctx.tc_flush()
        return {"iterations": it, "lmax": lmax, "bnorm": bnorm, **hist}

    def _batch(self, key, record) -> LoopBatch:
        """The loops ``record`` enqueues, captured once per key and then
        recorded with one tc_par_loops call each time."""
        b = self._batches.get(key)
        if b is None:
            with self.ctx.capture() as loops:
                record()
            b = self._batches[key] = LoopBatch(self.ctx, loops)
        return b

    def field(self, name: str) -> np.ndarray:
        a = self.ctx.tc_dat_read(self.f[name])
        h, n = self.h, self.n
        return a[tuple([slice(h, h + n)] * self.D)]


# ---------------------------------------------------------------------------
# mixed precision: FP32 stencil sweeps, FP64 reductions, FP64 refinement
# ---------------------------------------------------------------------------
class MixedHeatSolver:
    """Heat-conduction solve to a true FP64 relative residual.

    Iterative refinement: the solution x, the right-hand side b and the true
    residual r = b - A x live in FP64; every correction A d = r is solved by
    PPCG with FP32 storage and FP32 stencil sweeps (operator coefficients,
    directions, preconditioner state), while its dot products and norms
    accumulate in FP64 (the library's reductions always do).  x += d in FP64.
    """

    F64 = ("rho", "e", "u0", "u", "kx", "ky", "kz", "r", "d")
    F32 = ("kx", "ky", "kz", "r", "p", "w", "z", "rt", "sd", "d")

    def __init__(self, ctx: Context, density: np.ndarray, energy: np.ndarray, dt: float = 0.004, halo: int = 2):
        self.ctx = ctx
        self.D = density.ndim
        self.n = n = density.shape[0]
        self.h = halo
        self.rx = dt * n * n
        D = self.D
        self.blk = ctx.tc_decl_block(D, "heat")
        shape = tuple([n + 2 * halo] * D)
        inner = tuple([slice(halo, halo + n)] * D)
        self.f64: Dict[str, int] = {}
        self.f32: Dict[str, int] = {}
        for k in self.F64:
            if k == "kz" and D < 3:
                continue
            init = None
            if k in ("rho", "e"):
                init = np.zeros(shape)
                init[inner] = density if k == "rho" else energy
            self.f64[k] = ctx.tc_decl_dat(self.blk, [n] * D, [halo] * D, [halo] * D, init, TC_F64, k)
        for k in self.F32:
            if k == "kz" and D < 3:
                continue
            self.f32[k] = ctx.tc_decl_dat(self.blk, [n] * D, [halo] * D, [halo] * D, None, TC_F32, k + "32")
        # the FP64 driver shares stencils and helpers with HeatSolver
        self.H = HeatSolver.__new__(HeatSolver)
        H = self.H
        H.ctx, H.D, H.n, H.h, H.rx, H.blk = ctx, D, n, halo, self.rx, self.blk
        H.f = self.f64
        z = [0] * D

        def unit(d, s):
            p = [0] * D
            p[d] = s
            return tuple(p)

        H.S_c = ctx.tc_decl_stencil([tuple(z)])
        H.S_star = ctx.tc_decl_stencil([tuple(z)] + [unit(d, s) for d in range(D) for s in (-1, 1)])
        H.S_kface = [ctx.tc_decl_stencil([tuple(z), unit(d, 1)]) for d in range(D)]
        H.S_rho = ctx.tc_decl_stencil([tuple(z)] + [unit(d, -1) for d in range(D)])
        H.S_reflect = {}
        for axis in range(D):
            for side in (0, 1):
                sgn = 1 if side == 0 else -1
                H.S_reflect[(axis, side)] = ctx.tc_decl_stencil([tuple(z), unit(axis, sgn * 1), unit(axis, sgn * 3)])
        H.r_sum = [ctx.tc_decl_reduction(TC_RED_SUM, f"s{i}") for i in range(3)]
        H.r_max = ctx.tc_decl_reduction(TC_RED_MAX, "lmax")
        H.interior = [v for _ in range(D) for v in (0, n)]

    def _with(self, fields):
        self.H.f = fields

    def solve(self, tol: float = 1e-8, inner_tol: float = 1e-4, inner: int = 10, max_refine: int = 50,
              max_inner_iter: int = 500):
        """Refine until ||b - A x|| <= tol ||b|| (FP64); each correction runs
        PPCG in FP32 until its recursive residual falls by ``inner_tol``."""
        ctx, H = self.ctx, self.H
        D = self.D
        self._with(self.f64)
        lmax = H.setup()
        theta, delta, al, be = chebyshev_coefs(1.0, lmax, inner)
        s0, s1, s2 = H.r_sum
        H.dot("u0", "u0", s0)
        bnorm = math.sqrt(ctx.tc_reduction_result(s0))
        # FP32 operator coefficients
        for k in ["kx", "ky", "kz"][:D]:
            H.loop("COPY", [(self.f32[k], H.S_c, "W"), (self.f64[k], H.S_c, "R")],
                   rng=[v for _ in range(D) for v in (0, self.n + 1)], name=f"{k}32")
        history = []
        inner_total = 0
        for it in range(max_refine + 1):
            # true residual in FP64
            self._with(self.f64)
            H.halo_fill("u")
            H.loop("TEA_RESID", H.K() + [H.F("u", "R", H.S_star), H.F("u0", "R"), H.F("r", "W")])
            H.dot("r", "r", s0)
            rnorm = math.sqrt(ctx.tc_reduction_result(s0))
            history.append(rnorm / bnorm)
            if rnorm <= tol * bnorm or it == max_refine:
                break
            # correction solve in FP32 sweeps: A d = r, d0 = 0
            H.loop("COPY", [(self.f32["r"], H.S_c, "W"), (self.f64["r"], H.S_c, "R")], name="r32")
            self._with(self.f32)
            H.loop("AXPBY", [H.F("d", "RW"), H.F("r", "R")], [0.0, 0.0], name="d=0")
            H.precondition(theta, al, be, inner)
            H.loop("COPY", [H.F("p", "W"), H.F("z", "R")])
            H.dot("r", "z", s0)
            rz = ctx.tc_reduction_result(s0)
            r0 = rnorm
            k = 0
            while k < max_inner_iter:
                H.halo_fill("p")
                H.loop("TEA_MATVEC_DOT", H.K() + [H.F("p", "R", H.S_star), H.F("w", "W"), ("red", s0)])
                pw = ctx.tc_reduction_result(s0)
                alpha = rz / pw
                H.loop("TEA_CG_UPDATE", [H.F("d", "RW"), H.F("r", "RW"), H.F("p", "R"), H.F("w", "R")], [alpha])
                H.precondition(theta, al, be, inner)
                H.dot("r", "z", s1)
                H.dot("r", "r", s2)
                rz_new = ctx.tc_reduction_result(s1)
                rr = ctx.tc_reduction_result(s2)
                k += 1
                if math.sqrt(rr) <= inner_tol * r0:
                    break
                beta = rz_new / rz
                rz = rz_new
                H.loop("TEA_CG_P", [H.F("p", "RW"), H.F("z", "R")], [beta])
            inner_total += k
            # x += d in FP64
            self._with(self.f64)
            H.loop("COPY", [(self.f64["d"], H.S_c, "W"), (self.f32["d"], H.S_c, "R")], name="d64")
            H.loop("AXPBY", [H.F("u", "RW"), H.F("d", "R")], [1.0, 1.0], name="x+=d")
        ctx.tc_flush()
        self._with(self.f64)
        return {"refinements": len(history) - 1, "inner_iterations": inner_total, "history": history,
                "lmax": lmax, "bnorm": bnorm}

    def field(self, name: str) -> np.ndarray:
        a = self.ctx.tc_dat_read(self.f64[name])
        h, n = self.h, self.n
        return a[tuple([slice(h, h + n)] * self.D)]


# ---------------------------------------------------------------------------
# serving: a request trace replayed against a batch engine in real time
# ---------------------------------------------------------------------------
def serve(ctx: Context, requests, mixed: bool = False, tol: float = 1e-8, max_instances: int = 256,
          hbm_budget: int = 64 << 30, max_cells: int = 1 << 27, horizon: Optional[float] = None,
          drain: float = 120.0, keep_x: Sequence[int] = (), replays_per_step: int = 2):
    """Submit request i when the wall clock passes its arrival time; the
    engine (``tc_batch_step``) admits solves into free slots as memory frees
    up, advances every resident solve, and retires finished ones (continuous
    batching).  Arrivals after `horizon` seconds are not submitted; resident
    and queued work is then drained for at most `drain` seconds.  Returns a
    dict with per-request latency (completion - arrival, seconds, None if
    unfinished), engine results, and the solutions of the requests listed in
    `keep_x`."""
    import time
    from . import Batch, TC_SOLVE_DONE
    keep = set(keep_x)
    b = Batch(ctx, mixed=mixed, max_instances=max_instances, max_cells=max_cells, hbm_budget=hbm_budget,
              replays_per_step=replays_per_step)
    try:
        t0 = time.perf_counter()
        nxt = 0
        sub = {}  # request index -> (ticket, submit time since t0)
        horizon = requests[-1].arrival + 1e-9 if horizon is None and requests else horizon
        while True:
            now = time.perf_counter() - t0
            while nxt < len(requests) and requests[nxt].arrival <= now and requests[nxt].arrival <= horizon:
                q = requests[nxt]
                tk = b.tc_batch_submit(q.ndim, q.n, q.seed, tol=tol, keep_x=nxt in keep)
                sub[nxt] = (tk, time.perf_counter() - t0)
                nxt += 1
            left = b.tc_batch_step()
            arrivals_left = nxt < len(requests) and requests[nxt].arrival <= horizon
            if not arrivals_left and left == 0:
                break
            if now > horizon + drain:
                break
            if left == 0 and arrivals_left:
                time.sleep(max(0.0, min(requests[nxt].arrival - (time.perf_counter() - t0), 0.01)))
        b.tc_batch_step()
        wall = time.perf_counter() - t0
        out = {"latency": [None] * len(requests), "results": [None] * len(requests), "x": {}, "wall_s": wall,
               "submitted": len(sub)}
        for i, (tk, ts) in sub.items():
            r = b.tc_batch_poll(tk)
            out["results"][i] = r
            if r["state"] == TC_SOLVE_DONE:
                out["latency"][i] = ts + r["seconds"] - requests[i].arrival
                if i in keep:
                    out["x"][i] = b.tc_batch_read_x(tk)
        return out
    finally:
        b.close()


# ---------------------------------------------------------------------------
# compressible Euler: one SSP-RK3 step with fourth-order central differences
# ---------------------------------------------------------------------------
class EulerRunner:
    """Q = (rho, rho u_1..rho u_D, E) on a block with halo `halo` whose ghost
    cells hold fixed boundary values; ``record_step(dt)`` enqueues one RK3
    step: Q0 = Q, then per stage the primitive variables over the padded grid,
    one right-hand-side loop per component and one Runge-Kutta update per
    component over the interior."""

    RK3 = [(0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0)]

    def __init__(self, ctx: Context, q: Sequence[np.ndarray], n: int, h: float, gamma: float = 1.4, halo: int = 2,
                 dtype: int = TC_F64):
        self.ctx, self.n, self.h, self.halo = ctx, n, h, halo
        D = self.D = q[0].ndim
        self.gm1 = gamma - 1.0
        self.blk = ctx.tc_decl_block(D, "euler")
        size, hh = [n] * D, [halo] * D

        def dat(init, name):
            return ctx.tc_decl_dat(self.blk, size, hh, hh, init, dtype, name)

        self.Q = [dat(q[c], f"q{c}") for c in range(D + 2)]
        self.Q0 = [dat(q[c], f"q0_{c}") for c in range(D + 2)]
        self.R = [dat(None, f"r{c}") for c in range(D + 2)]
        self.vel = [dat(None, f"u{d}") for d in range(D)]
        self.p = dat(None, "p")
        z = [0] * D
        pts = [tuple(z)]
        for d in range(D):
            for o in (-1, 1, -2, 2):
                e = list(z)
                e[d] = o
                pts.append(tuple(e))
        self.S_c = ctx.tc_decl_stencil([tuple(z)])
        self.S_x = ctx.tc_decl_stencil(pts)
        self.red = ctx.tc_decl_reduction(TC_RED_SUM, "energy")
        self.interior = [v for _ in range(D) for v in (0, n)]
        self.padded = [v for _ in range(D) for v in (-halo, n + halo)]

    def record_step(self, dt: float):
        ctx, D = self.ctx, self.D
        for c in range(D + 2):
            ctx.tc_par_loop("COPY", self.blk, self.interior, [(self.Q0[c], self.S_c, "W"), (self.Q[c], self.S_c, "R")],
                            name=f"q0_{c}")
        s = 1.0 / (12.0 * self.h)
        for st, (a, b) in enumerate(self.RK3):
            ctx.tc_par_loop("EULER_PRIM", self.blk, self.padded,
                            [(q, self.S_c, "R") for q in self.Q] + [(u, self.S_c, "W") for u in self.vel] +
                            [(self.p, self.S_c, "W")], [self.gm1], name=f"prim{st}")
            for c in range(D + 2):
                ctx.tc_par_loop("EULER_RHS", self.blk, self.interior,
                                [(self.R[c], self.S_c, "W"), (self.Q[c], self.S_x, "R")] +
                                [(u, self.S_x, "R") for u in self.vel] + [(self.p, self.S_x, "R")],
                                [float(c), s], name=f"rhs{st}_{c}")
            for c in range(D + 2):
                ctx.tc_par_loop("RK_STAGE", self.blk, self.interior,
                                [(self.Q0[c], self.S_c, "R"), (self.Q[c], self.S_c, "RW"), (self.R[c], self.S_c, "R")],
                                [a, b, dt], name=f"rk{st}_{c}")

    def step(self, dt: float) -> float:
        """One RK3 step; returns the sum of E over the interior (the flush)."""
        self.record_step(dt)
        self.ctx.tc_par_loop("SUM", self.blk, self.interior, [(self.Q[self.D + 1], self.S_c, "R"), ("red", self.red)],
                             name="sumE")
        return self.ctx.tc_reduction_result(self.red)

    def loops_per_step(self) -> int:
        return (self.D + 2) + 3 * (1 + 2 * (self.D + 2)) + 1
