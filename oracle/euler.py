"""Compressible Euler step: three-stage SSP Runge-Kutta with fourth-order
central differences.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper tiles OpenSBLI's Taylor-Green vortex solver (Section 5, Section 6.4):
a chain of explicit Runge-Kutta stages, each a sweep of pointwise and
central-difference loops.  OpenSBLI's generated code is not part of the paper,
so the step is written from textbook definitions:

* conservative Euler equations, Q = (rho, rho u, rho v, rho w, E), ideal gas
  p = (gamma - 1)(E - rho |u|^2 / 2);
* the right-hand side L(Q) = -sum_d dF_d/dx_d with the fourth-order central
  difference df/dx = (8 (f_{+1} - f_{-1}) - (f_{+2} - f_{-2})) / (12 h),
  differences taken first (a constant field gives exactly zero);
* SSP-RK3 (Shu and Osher, J. Comput. Phys. 77, 1988):
  Q1 = Q0 + dt L(Q0);  Q2 = 3/4 Q0 + 1/4 (Q1 + dt L(Q1));
  Q3 = 1/3 Q0 + 2/3 (Q2 + dt L(Q2)).

Per stage the loops are, in program order: primitive variables over the whole
padded grid (ghost cells hold fixed boundary values), one right-hand-side loop
per component over the interior, then one Runge-Kutta update per component
over the interior.  Point arithmetic is in ``csrc/oracle.c``.
"""
from __future__ import annotations

import ctypes
from typing import Callable, List, Optional

import numpy as np

from . import OV, Grid, lib

RK3 = [(0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0)]


class EulerOracle:
    def __init__(self, q: List[np.ndarray], n: int, h: float, gamma: float = 1.4, halo: int = 2):
        self.ndim = q[0].ndim
        self.n, self.h, self.halo = n, h, halo
        self.gm1 = gamma - 1.0
        self.grid = Grid(self.ndim, n, halo)
        self.q = [np.array(a, dtype=np.float64, copy=True) for a in q]
        self.q0 = [a.copy() for a in self.q]
        self.vel = [np.zeros_like(self.q[0]) for _ in range(self.ndim)]
        self.p = np.zeros_like(self.q[0])
        self.r = [np.zeros_like(self.q[0]) for _ in range(self.ndim + 2)]
        self.L = lib()

    def _views(self, arrs):
        return (OV * len(arrs))(*[self.grid.view(a) for a in arrs])

    def prim(self):
        h, n = self.halo, self.n
        lo, hi = self.grid.box([-h] * self.ndim, [n + h] * self.ndim)
        self.L.orc_euler_prim(self.ndim, lo, hi, self._views(self.q), self._views(self.vel), self.grid.view(self.p),
                              ctypes.c_double(self.gm1))

    def rhs(self):
        lo, hi = self.grid.box(*self.grid.interior())
        s = 1.0 / (12.0 * self.h)
        for c in range(self.ndim + 2):
            self.L.orc_euler_rhs(self.ndim, lo, hi, c, self.grid.view(self.r[c]), self.grid.view(self.q[c]),
                                 self._views(self.vel), self.grid.view(self.p), ctypes.c_double(s))

    def rk_stage(self, a: float, b: float, dt: float):
        lo, hi = self.grid.box(*self.grid.interior())
        for c in range(self.ndim + 2):
            self.L.orc_rk_stage(lo, hi, self.grid.view(self.q0[c]), self.grid.view(self.q[c]),
                                self.grid.view(self.r[c]), ctypes.c_double(a), ctypes.c_double(b),
                                ctypes.c_double(dt))

    def step(self, dt: float, rhs: Optional[Callable[["EulerOracle"], None]] = None):
        """One RK3 step from the current state (which becomes Q0)."""
        for c in range(self.ndim + 2):
            self.q0[c][...] = self.q[c]
        for a, b in RK3:
            if rhs is None:
                self.prim()
                self.rhs()
            else:
                rhs(self)
            self.rk_stage(a, b, dt)

    def interior(self, a: np.ndarray) -> np.ndarray:
        h, n = self.halo, self.n
        return a[tuple([slice(h, h + n)] * self.ndim)]
