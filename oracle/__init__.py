"""Oracle for the run-time loop-chain tiling workloads.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1704_00693_amd``) and never imports it.

What it computes (Reguly, Mudalige, Giles, "Loop Tiling in Large-Scale Stencil
Codes at Run-time with OPS"):

* ``chain``     -- the plain definition of a loop chain: every loop executed in
                   program order over its whole iteration range (Section 3 and
                   the delayed-execution description, Section 4.1).  Tiling
                   only reorders this computation.
* ``skewed``    -- the tiling plan of Algorithm 1 (Section 4.2) and the tiled
                   execution order of Algorithm 2, in the paper's notation.
* ``stamps``    -- a brute-force dependency check: every read in a tiled
                   schedule must see the same writer as in program order
                   (the condition stated with the 1D example, Section 4.2).
* ``reduce``    -- reductions as exactly rounded sums (``math.fsum``).
* ``tealeaf``   -- the heat-conduction PPCG solve used as the workload of the
                   TeaLeaf experiment (Section 5/6.4), written from textbook
                   CG and Chebyshev iterations.
* ``euler``     -- a compressible-Euler Runge-Kutta step with fourth-order
                   central differences, the stand-in for the OpenSBLI
                   Taylor-Green experiment (Section 5/6.4).

Point arithmetic runs in ``csrc/oracle.c`` (plain C, explicit fma, FP64).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import List, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "oracle.c")
_LIB = os.path.join(_HERE, "csrc", "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C point operations (plain gcc, no fp contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-shared", "-fPIC",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OV(ctypes.Structure):
    _fields_ = [("p", ctypes.POINTER(ctypes.c_double)), ("origin", ctypes.c_int64),
                ("sx", ctypes.c_int64), ("sy", ctypes.c_int64), ("sz", ctypes.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        I64A = ctypes.POINTER(ctypes.c_int64)
        for name in ("orc_wsum", "orc_copy", "orc_axpby", "orc_halo_reflect", "orc_tea_init",
                     "orc_tea_k", "orc_tea_resid", "orc_tea_matvec_dot", "orc_tea_p1", "orc_tea_p2",
                     "orc_tea_precon_init", "orc_tea_cg_update", "orc_tea_cg_p", "orc_dot_terms",
                     "orc_euler_prim", "orc_euler_rhs", "orc_rk_stage"):
            getattr(L, name).restype = ctypes.c_int
        L.orc_tea_gersh.restype = ctypes.c_double
        _lib = L
    return _lib


class Grid:
    """Datasets of one block: numpy arrays (z, y, x) padded by ``halo`` on every
    side; logical coordinate c maps to array index c + halo."""

    def __init__(self, ndim: int, n: int, halo: int):
        self.ndim, self.n, self.halo = ndim, n, halo

    def view(self, a: np.ndarray) -> OV:
        assert a.dtype == np.float64 and a.flags.c_contiguous
        h = self.halo
        if a.ndim == 1:
            sx, sy, sz = 1, 0, 0
            origin = h
        elif a.ndim == 2:
            sx, sy, sz = 1, a.shape[1], 0
            origin = h * a.shape[1] + h
        else:
            sx, sy, sz = 1, a.shape[2], a.shape[1] * a.shape[2]
            origin = h * sz + h * sy + h
        return OV(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), origin, sx, sy, sz)

    def box(self, lo: Sequence[int], hi: Sequence[int]):
        l3 = list(lo) + [0] * (3 - len(lo))
        h3 = list(hi) + [1] * (3 - len(hi))
        return (ctypes.c_int64 * 3)(*l3), (ctypes.c_int64 * 3)(*h3)

    def interior(self):
        return [0] * self.ndim, [self.n] * self.ndim


def _off3(p):
    p = list(p) + [0] * (3 - len(p))
    return p


def wsum(grid: Grid, lo, hi, out: np.ndarray, inputs: List[np.ndarray], stencils, weights) -> None:
    """One weighted-sum loop over [lo, hi): out = sum_a sum_q w_aq * in_a[x + q]."""
    L = lib()
    nin = len(inputs)
    views = (OV * nin)(*[grid.view(a) for a in inputs])
    npts = (ctypes.c_int * nin)(*[len(s) for s in stencils])
    flat = [c for s in stencils for p in s for c in _off3(p)]
    offs = (ctypes.c_int * len(flat))(*flat)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    assert len(w) == sum(len(s) for s in stencils)
    l, h = grid.box(lo, hi)
    L.orc_wsum(l, h, grid.view(out), nin, views, npts, offs,
               w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))


def exact_sum(values) -> float:
    """Correctly rounded sum of all values (Shewchuk / math.fsum)."""
    return math.fsum(np.asarray(values, dtype=np.float64).ravel().tolist())


def exact_dot_terms(c: np.ndarray) -> float:
    """Correctly rounded sum of (prod, err) pairs, i.e. of the exact dot product."""
    return math.fsum(c.tolist())


def run_chain(chain, data: List[np.ndarray]) -> List[np.ndarray]:
    """Plain definition of a synthetic weighted-sum chain: loops in program
    order, each over the whole interior [0, n)^D.  Returns new arrays; the
    inputs are not modified.  If the chain ends with a reduction, the exactly
    rounded sum of the last-written dataset's interior is returned as well."""
    grid = Grid(chain.ndim, chain.n, chain.halo)
    arrs = [np.array(a, dtype=np.float64, copy=True) for a in data]
    lo, hi = grid.interior()
    for lp in chain.loops:
        wsum(grid, lo, hi, arrs[lp.out], [arrs[ci.dat] for ci in lp.inputs],
             [ci.stencil for ci in lp.inputs], lp.weights)
    return arrs


def interior(grid: Grid, a: np.ndarray) -> np.ndarray:
    h, n = grid.halo, grid.n
    sl = tuple([slice(h, h + n)] * a.ndim)
    return a[sl]
