"""Pins of the oracle's Algorithm 1 / Algorithm 2 (skewed tiling plan).

* the paper's 1D worked example, exactly (tests/golden/paper_1d_example.json);
* brute-force version stamps on random tiny chains (every read sees the same
  writer as in program order; every point of every loop runs exactly once);
* a planted mistake in a plan is caught by the stamp check;
* the CPU tiled schedule of a weighted-sum chain is bit-exact to program order;
* wavefront-parallel skewed tiles: the tiles of one wavefront (equal tile
  index sums) touch disjoint data wherever one of them writes, over the whole
  chain, so any interleaving of them is program order; the stamp check agrees
  for interleaved and reversed orders, and rejects a grouping that puts
  dependent tiles in one wavefront.
"""
import json
import os
import random

import numpy as np
import pytest

import oracle
from oracle.skewed import READ, WRITE, Arg, Loop, skewed_plan, execute_tiled, max_skew, wavefront_schedule, wavefronts
from oracle.stamps import check_schedule, tiled_schedule
from randchains import random_chain, to_oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_1d_example.json")


def test_paper_1d_example():
    g = json.load(open(GOLD))
    n = g["points"]
    loops = []
    for spec in g["loops"]:
        args = [Arg(r["dat"], [(o,) for o in r["stencil"]], READ) for r in spec["reads"]]
        args += [Arg(w, [(0,)], WRITE) for w in spec["writes"]]
        loops.append(Loop([0], [n], args, spec["name"]))
    plan = skewed_plan(loops, 1, [g["tilesize"]])
    assert plan.num_tiles == [2]
    for l, spec in enumerate(g["loops"]):
        got = [[plan.start[0][t][l], plan.end[0][t][l]] for t in range(2)]
        assert got == g["expected_half_open"][spec["name"]]
        incl = [[a, b - 1] for a, b in got]
        assert incl == g["expected_inclusive"][spec["name"]]
    check_schedule(loops, tiled_schedule(plan, len(loops)))


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_random_chains_stamps(ndim):
    rng = random.Random(1000 + ndim)
    for _ in range(250 if ndim < 3 else 120):
        ch = random_chain(rng, ndim)
        loops = to_oracle(ch)
        ts = [rng.randint(1, 5) for _ in range(ndim)]
        plan = skewed_plan(loops, ndim, ts)
        check_schedule(loops, tiled_schedule(plan, len(loops)))


def test_untiled_dimension_is_one_tile():
    rng = random.Random(7)
    ch = random_chain(rng, 2)
    loops = to_oracle(ch)
    plan = skewed_plan(loops, 2, [0, 2])
    assert plan.num_tiles[0] == 1
    check_schedule(loops, tiled_schedule(plan, len(loops)))


def test_planted_mistake_is_caught():
    """Shrinking one interior tile end of a producer loop (a dropped skew)
    must be reported by the stamp check."""
    loops = [
        Loop([0], [12], [Arg(0, [(0,)], READ), Arg(1, [(0,)], WRITE)]),
        Loop([0], [12], [Arg(1, [(-1,), (0,), (1,)], READ), Arg(2, [(0,)], WRITE)]),
        Loop([0], [12], [Arg(2, [(-2,), (0,), (2,)], READ), Arg(0, [(0,)], WRITE)]),
    ]
    plan = skewed_plan(loops, 1, [4])
    check_schedule(loops, tiled_schedule(plan, 3))
    assert plan.end[0][0][0] > plan.end[0][0][1] > plan.end[0][0][2]  # skewed
    plan.end[0][0][0] -= 1
    plan.start[0][1][0] -= 1
    with pytest.raises(AssertionError):
        check_schedule(loops, tiled_schedule(plan, 3))


def test_skew_matches_stencil_radii():
    """A chain of k loops each reading the previous output with radius r: the
    tile boundary of loop i (0-based) sits (k-1-i)*r beyond the last loop's."""
    k, r = 5, 2
    loops = []
    for i in range(k):
        loops.append(Loop([0], [64], [Arg(i, [(-r,), (0,), (r,)], READ), Arg(i + 1, [(0,)], WRITE)]))
    plan = skewed_plan(loops, 1, [16])
    for t in range(plan.num_tiles[0] - 1):
        base = plan.end[0][t][k - 1]
        for i in range(k):
            assert plan.end[0][t][i] == base + (k - 1 - i) * r
    assert max_skew(plan, 0) == (k - 1) * r


@pytest.mark.parametrize("ndim,n,tile", [(2, 13, [5, 4]), (3, 7, [3, 4, 2])])
def test_cpu_tiled_chain_bit_exact(ndim, n, tile):
    from synthgen import make_chain, chain_data
    ch = make_chain(ndim, n, 5, 8, seed=11)
    data = chain_data(ch)
    ref = oracle.run_chain(ch, data)
    loops = [Loop([0] * ndim, [n] * ndim,
                  [Arg(ci.dat, ci.stencil, READ) for ci in lp.inputs] + [Arg(lp.out, [tuple([0] * ndim)], WRITE)])
             for lp in ch.loops]
    plan = skewed_plan(loops, ndim, tile)
    check_schedule(loops, tiled_schedule(plan, len(loops)))
    grid = oracle.Grid(ndim, n, ch.halo)
    arrs = [a.copy() for a in data]

    def run_loop(l, lo, hi):
        lp = ch.loops[l]
        oracle.wsum(grid, lo, hi, arrs[lp.out], [arrs[c.dat] for c in lp.inputs],
                    [c.stencil for c in lp.inputs], lp.weights)

    execute_tiled(plan, len(loops), run_loop)
    for a, b in zip(arrs, ref):
        assert np.array_equal(a, b)


def _footprint(plan, loops, t):
    """Points a tile reads and writes over the whole chain, as (dataset, point)."""
    import itertools
    reads, writes = set(), set()
    for l, lp in enumerate(loops):
        lo, hi = plan.box(t, l)
        for x in itertools.product(*[range(a, b) for a, b in zip(lo, hi)]):
            for a in lp.args:
                if a.reads():
                    for q in a.stencil:
                        reads.add((a.dat, tuple(xi + qi for xi, qi in zip(x, q))))
                if a.writes():
                    writes.add((a.dat, x))
    return reads, writes


@pytest.mark.parametrize("ndim", [2, 3])
def test_wavefront_parallel_tiles(ndim):
    import itertools
    rng = random.Random(7000 + ndim)
    pairs = 0
    col_conflicts = [0]
    for _ in range(60 if ndim == 2 else 30):
        ch = random_chain(rng, ndim)
        loops = to_oracle(ch)
        plan = skewed_plan(loops, ndim, [rng.randint(1, 5) for _ in range(ndim)])
        for wave in wavefronts(plan):
            fp = [_footprint(plan, loops, t) for t in wave]
            for (ra, wa), (rb, wb) in itertools.combinations(fp, 2):
                assert not (wa & (rb | wb)) and not (wb & ra)
                pairs += 1
        for interleave, reverse in ((True, False), (True, True), (False, True)):
            check_schedule(loops, wavefront_schedule(plan, len(loops), interleave, reverse))
        # the same check finds conflicts when a column of tiles (one x index,
        # consecutive y indices, which depend on each other) is grouped instead
        cols = {}
        for t in plan.tiles():
            cols.setdefault(t[0], []).append(t)
        for col in cols.values():
            fp = [_footprint(plan, loops, t) for t in col]
            for (ra, wa), (rb, wb) in itertools.combinations(fp, 2):
                col_conflicts[0] += bool((wa & (rb | wb)) or (wb & ra))
    assert pairs > 100 and col_conflicts[0] > 0


def test_wavefront_check_rejects_dependent_tiles():
    n = 12
    # a 1D chain whose tiles depend on each other in sequence: its tiles form
    # one wavefront each; put all of them in one wavefront, run one after the
    # other in reverse order, and program order breaks
    loops = [Loop([0], [n], [Arg(0, [(-1,), (0,), (1,)], READ), Arg(1, [(0,)], WRITE)]),
             Loop([0], [n], [Arg(1, [(-1,), (0,), (1,)], READ), Arg(2, [(0,)], WRITE)]),
             Loop([0], [n], [Arg(2, [(-1,), (0,), (1,)], READ), Arg(0, [(0,)], WRITE)])]
    plan = skewed_plan(loops, 1, [3])
    check_schedule(loops, wavefront_schedule(plan, len(loops)))
    assert len(wavefronts(plan)) == plan.num_tiles[0] > 1
    together = [(l, *plan.box((t,), l)) for t in reversed(range(plan.num_tiles[0])) for l in range(len(loops))
                if plan.box((t,), l)[1][0] > plan.box((t,), l)[0][0]]
    with pytest.raises(AssertionError):
        check_schedule(loops, together)
