"""Pins of the Jacobi heat-equation oracle (the paper's baseline benchmark,
Sections 5 and 6.2): the closed-form decay of a discrete sine mode, a
brute-force evaluation with exactly rounded fma on tiny grids, the fixed
Dirichlet layer, equal copy and non-copy results, and the window oracle used
for full-size checks."""
import math
import sys
from fractions import Fraction

import numpy as np
import pytest

from oracle.jacobi import jacobi
from synthgen import JACOBI_POINTS, JACOBI_WEIGHTS, jacobi_field, jacobi_mode

sys.path.insert(0, "tests")
from windows import jacobi_window  # noqa: E402


def _fma(a, b, c):
    """fma(a, b, c) rounded once: exact rational arithmetic, then Python's
    correctly rounded int / int division."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _brute(u0, iters, points, weights):
    """Jacobi iterations with pure-Python loops (non-copy order)."""
    cur = [list(map(float, row)) for row in u0]
    ny, nx = len(cur) - 2, len(cur[0]) - 2
    for _ in range(iters):
        nxt = [row[:] for row in cur]
        for y in range(ny):
            for x in range(nx):
                acc = 0.0
                for (dx, dy), w in zip(points, weights):
                    acc = _fma(w, cur[y + 1 + dy][x + 1 + dx], acc)
                nxt[y + 1][x + 1] = acc
        cur = nxt
    return np.array(cur)


@pytest.mark.parametrize("n,k,l,iters", [(37, 3, 5, 40), (24, 1, 2, 31), (16, 7, 2, 9)])
@pytest.mark.parametrize("copy", [False, True])
def test_sine_mode_decays_by_the_eigenvalue(n, k, l, iters, copy):
    """sin(a (x+1)) sin(b (y+1)), a = pi k/(n+1), b = pi l/(n+1), vanishes on
    the layer and is an eigenvector of the stencil: one iteration scales it
    by 0.2 (1 + 2 cos a + 2 cos b)."""
    u0 = jacobi_mode(n, k, l)
    lam = 0.2 * (1.0 + 2.0 * math.cos(math.pi * k / (n + 1)) + 2.0 * math.cos(math.pi * l / (n + 1)))
    got = jacobi(u0, iters, JACOBI_POINTS, JACOBI_WEIGHTS, copy)
    exact = lam ** iters * u0
    bound = 8 * iters * np.finfo(float).eps
    assert np.abs(got - exact).max() <= bound, (np.abs(got - exact).max(), bound)
    assert np.all(got[0, :] == 0) and np.all(got[-1, :] == 0)
    assert np.all(got[:, 0] == 0) and np.all(got[:, -1] == 0)


@pytest.mark.parametrize("shape,iters", [((7, 7), 3), ((6, 9), 4), ((9, 5), 2)])
def test_brute_force_tiny(shape, iters):
    """Bit-exact against pure-Python loops with exactly rounded fma, on
    square and non-square fields, with asymmetric weights so that a swapped
    axis or offset shows."""
    u0 = jacobi_field(max(shape), seed=9)[:shape[0], :shape[1]].copy()
    weights = [0.3, 0.11, 0.17, 0.13, 0.29]
    for copy in (False, True):
        got = jacobi(u0, iters, JACOBI_POINTS, weights, copy)
        assert np.array_equal(got, _brute(u0, iters, JACOBI_POINTS, weights))


@pytest.mark.parametrize("iters", [6, 7])
def test_copy_and_non_copy_agree_and_layer_is_fixed(iters):
    u0 = jacobi_field(30, seed=3)
    a = jacobi(u0, iters, JACOBI_POINTS, JACOBI_WEIGHTS, True)
    b = jacobi(u0, iters, JACOBI_POINTS, JACOBI_WEIGHTS, False)
    assert np.array_equal(a, b)
    for got in (a, b):
        assert np.array_equal(got[0, :], u0[0, :]) and np.array_equal(got[-1, :], u0[-1, :])
        assert np.array_equal(got[:, 0], u0[:, 0]) and np.array_equal(got[:, -1], u0[:, -1])
    # weights sum to 1 and are positive: values stay within the initial range
    assert a.min() >= u0.min() - 1e-15 and a.max() <= u0.max() + 1e-15


@pytest.mark.parametrize("y0,x0,s", [(0, 0, 6), (20, 13, 5), (34, 34, 6), (0, 27, 9)])
@pytest.mark.parametrize("copy", [False, True])
def test_window_equals_full(y0, x0, s, copy):
    n, iters = 40, 9
    u0 = jacobi_field(n, seed=11)
    full = jacobi(u0, iters, JACOBI_POINTS, JACOBI_WEIGHTS, copy)
    win = jacobi_window(u0, iters, JACOBI_POINTS, JACOBI_WEIGHTS, copy, y0, x0, s)
    assert np.array_equal(win, full[y0 + 1:y0 + 1 + s, x0 + 1:x0 + 1 + s])


@pytest.mark.parametrize("copy", [False, True])
@pytest.mark.parametrize("tile", [[8, 5], [30, 3], [4, 11]])
def test_skewed_tiles_reproduce_program_order(copy, tile):
    """The skewed tiling of Algorithms 1 and 2 applied to the Jacobi chain on
    the CPU (every tile in order, every loop over its skewed range) gives the
    program-order values bit for bit: the copy variant's write-after-read
    dependencies included."""
    from oracle import Grid, wsum
    from oracle.jacobi import _copy_interior
    from oracle.skewed import Arg, Loop, execute_tiled, skewed_plan
    n, iters = 23, 9
    u0 = jacobi_field(n, seed=21)
    pts = [tuple(p) for p in JACOBI_POINTS]
    loops, ops = [], []
    for t in range(iters):
        if copy:
            loops += [Loop([0, 0], [n, n], [Arg(1, [(0, 0)], "W"), Arg(0, pts, "R")]),
                      Loop([0, 0], [n, n], [Arg(0, [(0, 0)], "W"), Arg(1, [(0, 0)], "R")])]
            ops += [("stencil", 0, 1), ("copy", 1, 0)]
        else:
            src, dst = (0, 1) if t % 2 == 0 else (1, 0)
            loops.append(Loop([0, 0], [n, n], [Arg(dst, [(0, 0)], "W"), Arg(src, pts, "R")]))
            ops.append(("stencil", src, dst))
    arrs = [u0.copy(), u0.copy()]
    grid = Grid(2, n, 1)

    def run_loop(l, lo, hi):
        kind, src, dst = ops[l]
        if kind == "stencil":
            wsum(grid, lo, hi, arrs[dst], [arrs[src]], [pts], JACOBI_WEIGHTS)
        else:
            _copy_interior(grid, lo, hi, arrs[dst], arrs[src])

    execute_tiled(skewed_plan(loops, 2, tile), len(loops), run_loop)
    ref = jacobi(u0, iters, JACOBI_POINTS, JACOBI_WEIGHTS, copy)
    got = arrs[0] if copy or iters % 2 == 0 else arrs[1]
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("mutation", ["moved point", "dropped term", "swapped weight"])
def test_closed_form_catches_a_planted_stencil_mistake(mutation):
    """Negative control of the eigenmode pin: the oracle run with a wrong
    stencil (a point moved one cell further, a point left out, or two weights
    exchanged on an asymmetric stencil) misses the closed-form decay by far
    more than the rounding bound."""
    n, k, l, iters = 37, 3, 5, 40
    u0 = jacobi_mode(n, k, l)
    lam = 0.2 * (1.0 + 2.0 * math.cos(math.pi * k / (n + 1)) + 2.0 * math.cos(math.pi * l / (n + 1)))
    pts = [tuple(p) for p in JACOBI_POINTS]
    w = list(JACOBI_WEIGHTS)
    if mutation == "moved point":
        i = pts.index((1, 0))
        pts[i] = (2, 0)
    elif mutation == "dropped term":
        i = pts.index((0, 1))
        del pts[i], w[i]
    else:
        # an x/y-asymmetric mode, so exchanging an x weight with a y weight shows
        k, l = 2, 7
        u0 = jacobi_mode(n, k, l)
        w = [0.2, 0.25, 0.25, 0.15, 0.15]
        lam = 0.2 + 0.5 * math.cos(math.pi * k / (n + 1)) + 0.3 * math.cos(math.pi * l / (n + 1))
        ix, iy = pts.index((1, 0)), pts.index((0, 1))
        w[ix], w[iy] = w[iy], w[ix]
    got = jacobi(u0, iters, pts, w, False)
    err = np.abs(got - lam ** iters * u0).max()
    assert err > 1e4 * 8 * iters * np.finfo(float).eps, err


def test_skewed_plan_without_skew_breaks_program_order():
    """Negative control of the skewed-schedule pin: the same tiles with every
    loop cut at the same rows (the skew of Algorithm 1 removed) let a later
    iteration read rows of the next tile that an earlier iteration has not
    produced yet, and the result differs from program order."""
    from oracle import Grid, wsum
    from oracle.skewed import Arg, Loop, Plan, execute_tiled, skewed_plan
    n, iters, rows = 23, 9, 5
    u0 = jacobi_field(n, seed=21)
    pts = [tuple(p) for p in JACOBI_POINTS]
    loops = []
    for t in range(iters):
        src, dst = (0, 1) if t % 2 == 0 else (1, 0)
        loops.append(Loop([0, 0], [n, n], [Arg(dst, [(0, 0)], "W"), Arg(src, pts, "R")]))
    good = skewed_plan(loops, 2, [0, rows])
    T = good.num_tiles[1]
    flat_end = [[[min(n, (t + 1) * rows) for _ in loops] for t in range(T)]]
    flat_start = [[[t * rows for _ in loops] for t in range(T)]]
    flat = Plan(2, good.num_tiles, [good.start[0], flat_start[0]], [good.end[0], flat_end[0]])
    assert flat.num_tiles == [1, T] and T > 2

    def run(plan):
        arrs = [u0.copy(), u0.copy()]
        grid = Grid(2, n, 1)

        def run_loop(l, lo, hi):
            src, dst = (0, 1) if l % 2 == 0 else (1, 0)
            wsum(grid, lo, hi, arrs[dst], [arrs[src]], [pts], JACOBI_WEIGHTS)

        execute_tiled(plan, len(loops), run_loop)
        return arrs[1] if iters % 2 else arrs[0]

    ref = jacobi(u0, iters, JACOBI_POINTS, JACOBI_WEIGHTS, False)
    assert np.array_equal(run(good), ref)
    assert not np.array_equal(run(flat), ref)
