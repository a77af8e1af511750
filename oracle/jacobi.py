"""Jacobi iteration of the 2D heat equation: the tiling benchmark the paper
uses to set a baseline (Section 5, first application; measured in Section
6.2 on an 8192^2 mesh with one extra Dirichlet layer on every side, 250
iterations, FP64).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may use this module.  It shares no
code with the GPU library and never imports it.

One iteration applies a five-point weighted stencil to the current field over
the interior and writes the result to the other array; the boundary layer
(one cell wide) is never written.  Section 5 names two ways to run the time
loop, and both are written out here in the plain order:

* copy: b = stencil(a), then a second loop copies b back into a;
* non-copy: the time loop unrolled by two, a -> b on even iterations and
  b -> a on odd ones, with no copy.

Both produce the same values.  After T iterations the copy variant's result
is in a; the non-copy variant's is in a for even T and in b for odd T.

The stencil's point arithmetic is the oracle's weighted sum (``oracle.wsum``,
plain C, explicit fma in point order); the copy is a plain element copy.
Pins: a closed-form eigenmode decay, a brute-force evaluation with exactly
rounded fma on tiny grids, and the invariants of a fixed boundary layer and
of equal copy / non-copy results.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import Grid, lib, wsum


def _copy_interior(grid: Grid, lo, hi, dst: np.ndarray, src: np.ndarray) -> None:
    l, h = grid.box(lo, hi)
    lib().orc_copy(l, h, grid.view(dst), grid.view(src))


def jacobi(u0: np.ndarray, iters: int, points: Sequence[Sequence[int]], weights: Sequence[float],
           copy: bool) -> np.ndarray:
    """Run ``iters`` Jacobi iterations on a field with a one-cell boundary
    layer.  ``u0`` is (ny + 2, nx + 2) (y, x), the layer included; the
    interior is x in [0, nx), y in [0, ny).  ``points`` are (x, y) offsets of
    the stencil and ``weights`` one weight per point, applied in that order.
    Returns a new array holding the field after the last iteration."""
    ny, nx = u0.shape[0] - 2, u0.shape[1] - 2
    grid = Grid(2, max(nx, ny), 1)
    lo, hi = [0, 0], [nx, ny]
    a = np.array(u0, dtype=np.float64, copy=True)
    b = a.copy()
    pts = [tuple(p) for p in points]
    w = list(weights)
    for t in range(iters):
        if copy:
            wsum(grid, lo, hi, b, [a], [pts], w)
            _copy_interior(grid, lo, hi, a, b)
        elif t % 2 == 0:
            wsum(grid, lo, hi, b, [a], [pts], w)
        else:
            wsum(grid, lo, hi, a, [b], [pts], w)
    return a if copy or iters % 2 == 0 else b
