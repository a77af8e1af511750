"""Heat-conduction solve with polynomially preconditioned CG (PPCG).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper evaluates tiling on TeaLeaf's PPCG solver (Section 5 and Section 6.4:
CG with a Chebyshev polynomial preconditioner whose two key loops touch five
datasets and contain no reductions).  TeaLeaf's own source is not part of the
paper, so the solve is written from the textbook methods it names:

* preconditioned CG (Saad, Iterative Methods for Sparse Linear Systems, 2nd
  ed., Algorithm 9.1);
* Chebyshev iteration as the preconditioner z = M^{-1} r (Saad, Algorithm
  12.1), a fixed number of steps from z = 0, so M^{-1} is a fixed polynomial
  in A and PCG stays valid.

Operator (implicit backward-Euler heat step, unit square, dx = 1/n):
``(A v)_c = (1 + sum of the cell's face coefficients) v_c - sum over faces of
K_face * v_neighbour`` with ``K = (dt/dx^2) * 2 / (rho_left + rho_right)``
(harmonic mean of the conductivity 1/rho) and reflective ghost cells, so the
boundary flux cancels and the smallest eigenvalue is exactly 1.  The largest
eigenvalue is bounded by the Gershgorin bound ``max_c 1 + 2 * sum K``.

Every loop runs over its whole range in program order (the plain definition
that a tiled execution must reproduce).  Reductions are exactly rounded.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import Grid, OV, lib, exact_dot_terms


@dataclass
class Cheb:
    theta: float
    delta: float
    alpha: List[float]  # alpha_j, j = 1..steps-1 (used after inner step j)
    beta: List[float]


def chebyshev_coefs(lmin: float, lmax: float, steps: int) -> Cheb:
    """rho_0 = 1/sigma, rho_j = 1/(2 sigma - rho_{j-1}); after step j the new
    direction is rho_j rho_{j-1} d + (2 rho_j / delta) r (Saad, Alg. 12.1)."""
    theta = (lmax + lmin) / 2.0
    delta = (lmax - lmin) / 2.0
    sigma = theta / delta
    rho_old = 1.0 / sigma
    al, be = [], []
    for _ in range(1, steps):
        rho_new = 1.0 / (2.0 * sigma - rho_old)
        al.append(rho_new * rho_old)
        be.append(2.0 * rho_new / delta)
        rho_old = rho_new
    return Cheb(theta, delta, al, be)


class HeatOracle:
    """Field storage and loops of the heat solve on one block."""

    FIELDS = ("rho", "e", "u0", "u", "kx", "ky", "kz", "r", "p", "w", "z", "rt", "sd")

    def __init__(self, density: np.ndarray, energy: np.ndarray, dt: float = 0.004, halo: int = 2):
        self.ndim = density.ndim
        self.n = density.shape[0]
        self.halo = halo
        self.grid = Grid(self.ndim, self.n, halo)
        shape = tuple([self.n + 2 * halo] * self.ndim)
        self.f: Dict[str, np.ndarray] = {k: np.zeros(shape) for k in self.FIELDS}
        h, n = halo, self.n
        inner = tuple([slice(h, h + n)] * self.ndim)
        self.f["rho"][inner] = density
        self.f["e"][inner] = energy
        self.rx = dt * n * n  # dt / dx^2 with dx = 1/n
        self.L = lib()
        self.log: List[str] = []

    # -- helpers -----------------------------------------------------------
    def v(self, name) -> OV:
        return self.grid.view(self.f[name])

    def kv(self):
        names = ["kx", "ky", "kz"][: self.ndim]
        return (OV * 3)(*[self.v(k) for k in names] + [self.v("kx")] * (3 - self.ndim))

    def box(self, lo, hi):
        return self.grid.box(lo, hi)

    def interior(self):
        return [0] * self.ndim, [self.n] * self.ndim

    # -- loops (each over its whole range) --------------------------------
    def halo_ranges(self):
        """Reflective fill of both ghost layers, one loop per side: x sides over
        the interior of the other axes; later axes over the full padded extent
        of the earlier axes (corners included)."""
        n, h, D = self.n, self.halo, self.ndim
        out = []
        for axis in range(D):
            for side in (0, 1):
                lo, hi = [], []
                for d in range(D):
                    if d == axis:
                        lo.append(-h if side == 0 else n)
                        hi.append(0 if side == 0 else n + h)
                    elif d < axis:
                        lo.append(-h)
                        hi.append(n + h)
                    else:
                        lo.append(0)
                        hi.append(n)
                out.append((axis, side, lo, hi))
        return out

    def fill_halo(self, name):
        for axis, side, lo, hi in self.halo_ranges():
            l, h = self.box(lo, hi)
            self.L.orc_halo_reflect(l, h, self.v(name), axis, side, ctypes.c_int64(self.n))

    def setup(self) -> float:
        """Ghost-fill rho, u0 = u = e*rho, face coefficients, Gershgorin bound."""
        self.fill_halo("rho")
        l, h = self.box(*self.interior())
        self.L.orc_tea_init(l, h, self.v("rho"), self.v("e"), self.v("u0"), self.v("u"))
        l, h = self.box([0] * self.ndim, [self.n + 1] * self.ndim)
        self.L.orc_tea_k(self.ndim, l, h, self.v("rho"), self.kv(), ctypes.c_double(self.rx))
        l, h = self.box(*self.interior())
        return float(self.L.orc_tea_gersh(self.ndim, l, h, self.kv()))

    def resid(self):
        self.fill_halo("u")
        l, h = self.box(*self.interior())
        self.L.orc_tea_resid(self.ndim, l, h, self.kv(), self.v("u"), self.v("u0"), self.v("r"))

    def precondition(self, cheb: Cheb, steps: int):
        l, h = self.box(*self.interior())
        self.L.orc_tea_precon_init(l, h, self.v("r"), self.v("rt"), self.v("sd"), self.v("z"),
                                   ctypes.c_double(cheb.theta))
        for j in range(1, steps + 1):
            self.fill_halo("sd")
            self.L.orc_tea_p1(self.ndim, l, h, self.kv(), self.v("sd"), self.v("rt"), self.v("z"))
            if j < steps:
                self.L.orc_tea_p2(l, h, self.v("sd"), self.v("rt"),
                                  ctypes.c_double(cheb.alpha[j - 1]), ctypes.c_double(cheb.beta[j - 1]))

    def dot(self, a, b) -> float:
        cells = self.n ** self.ndim
        c = np.empty(2 * cells)
        l, h = self.box(*self.interior())
        self.L.orc_dot_terms(l, h, self.v(a), self.v(b), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return exact_dot_terms(c)

    def matvec_dot(self) -> float:
        self.fill_halo("p")
        cells = self.n ** self.ndim
        c = np.empty(2 * cells)
        l, h = self.box(*self.interior())
        self.L.orc_tea_matvec_dot(self.ndim, l, h, self.kv(), self.v("p"), self.v("w"),
                                  c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return exact_dot_terms(c)

    def copy(self, dst, src):
        l, h = self.box(*self.interior())
        self.L.orc_copy(l, h, self.v(dst), self.v(src))

    def cg_update(self, alpha):
        l, h = self.box(*self.interior())
        self.L.orc_tea_cg_update(l, h, self.v("u"), self.v("r"), self.v("p"), self.v("w"), ctypes.c_double(alpha))

    def cg_p(self, beta):
        l, h = self.box(*self.interior())
        self.L.orc_tea_cg_p(l, h, self.v("p"), self.v("z"), ctypes.c_double(beta))

    def apply_A(self, name: str) -> np.ndarray:
        """A applied to a field (ghosts reflected first), returned as a new
        interior array; used by tests and for the true residual."""
        self.fill_halo(name)
        keep = self.f["r"].copy()
        l, h = self.box(*self.interior())
        zero = np.zeros_like(self.f["r"])
        self.f["_zero"] = zero
        self.L.orc_tea_resid(self.ndim, l, h, self.kv(), self.v(name), self.grid.view(zero), self.v("r"))
        out = -self.inner("r")
        self.f["r"][...] = keep
        del self.f["_zero"]
        return out

    def inner(self, name) -> np.ndarray:
        h, n = self.halo, self.n
        return self.f[name][tuple([slice(h, h + n)] * self.ndim)].copy()


@dataclass
class SolveResult:
    x: np.ndarray
    iterations: int
    rr: List[float]
    rz: List[float]
    pw: List[float]
    lmax: float
    bnorm: float
    true_rel_resid: float


def ppcg_solve(density, energy, outer: int = 50, inner: int = 10, tol: Optional[float] = None,
               dt: float = 0.004, max_iter: int = 10000, oracle: Optional[HeatOracle] = None) -> SolveResult:
    """PPCG for A x = b, b = x0 = e * rho.  With ``tol`` None, exactly
    ``outer`` iterations; otherwise stop when sqrt(r.r)/||b|| <= tol."""
    H = oracle or HeatOracle(density, energy, dt)
    lmax = H.setup()
    cheb = chebyshev_coefs(1.0, lmax, inner)
    bnorm = math.sqrt(H.dot("u0", "u0"))
    H.resid()
    H.precondition(cheb, inner)
    H.copy("p", "z")
    rz = H.dot("r", "z")
    rr_hist, rz_hist, pw_hist = [], [], []
    it = 0
    limit = outer if tol is None else max_iter
    while it < limit:
        pw = H.matvec_dot()
        alpha = rz / pw
        H.cg_update(alpha)
        H.precondition(cheb, inner)
        rz_new = H.dot("r", "z")
        rr = H.dot("r", "r")
        it += 1
        rr_hist.append(rr)
        rz_hist.append(rz_new)
        pw_hist.append(pw)
        if tol is not None and math.sqrt(rr) <= tol * bnorm:
            break
        beta = rz_new / rz
        rz = rz_new
        H.cg_p(beta)
    x = H.inner("u")
    Ax = H.apply_A("u")
    b = H.inner("u0")
    true = math.sqrt(math.fsum(((b - Ax) ** 2).ravel().tolist())) / bnorm
    return SolveResult(x, it, rr_hist, rz_hist, pw_hist, lmax, bnorm, true)
