"""Skewed tiling plan (Algorithm 1), tiled execution order (Algorithm 2) and
the wavefront-parallel order of the same tiles (future work, end of Section
4.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Written from Section 4.2 of Reguly, Mudalige, Giles, "Loop Tiling in
Large-Scale Stencil Codes at Run-time with OPS": the seven-step description and
Algorithm 1 (plan), Algorithm 2 (execution).  Notation follows the paper:
``loop_l.start_d / end_d``, ``tile_{t_d}.loop_l.start_d / end_d``,
``read_dep_a.tile_t.start_d / end_d``, ``write_dep_a.tile_t.start_d / end_d``.

Readings of passages that are garbled or ambiguous in the printed algorithm
(each one is listed with its reason in the design notes):

* ranges are half-open [start, end); the paper's 1D example is inclusive;
* a tile's start is the previous tile's END for the same loop (the prose of
  step 3 says so; the printed line repeats "start");
* the default end is ``min(loop_l.end_d, start_d + (t_d + 1) * tilesize_d)``
  with 0-based tile index (with the printed ``t * tilesize`` the first tile
  would be empty);
* the start, the read-after-write end, the write-after-read/write end and the
  default end are all computed in ONE pass over the tiles in increasing order,
  because the next tile's start needs this tile's final end;
* "last non-empty tile in d" is the last tile index; ends are clipped to the
  loop's range so a loop's trailing tiles may be empty;
* an end below the start is raised to the start (empty tile for that loop);
* "largest negative / positive stencil point in d" are the minimum and
  maximum stencil offsets along d;
* the write-dependency update uses tile index t (printed subscript "l");
* dependencies are kept per dimension (separable), indexed by t_d, and never
  shrink (monotone union);
* multi-dimensional tiles run in lexicographic order, slowest dimension
  outermost (x innermost).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

INF = float("inf")

READ, WRITE, RW, INC = "R", "W", "RW", "INC"


@dataclass
class Arg:
    dat: int
    stencil: List[Tuple[int, ...]]
    access: str

    def reads(self) -> bool:
        return self.access in (READ, RW, INC)

    def writes(self) -> bool:
        return self.access in (WRITE, RW, INC)

    def lo(self, d: int) -> int:
        return min(p[d] for p in self.stencil)

    def hi(self, d: int) -> int:
        return max(p[d] for p in self.stencil)


@dataclass
class Loop:
    start: List[int]
    end: List[int]
    args: List[Arg]
    name: str = ""


@dataclass
class Plan:
    ndim: int
    num_tiles: List[int]
    # start[d][t][l], end[d][t][l]
    start: List[List[List[int]]]
    end: List[List[List[int]]]

    def tiles(self):
        """Tile index tuples (t_0, ..., t_{D-1}) in execution order: slowest
        dimension outermost, dimension 0 (x) innermost."""
        ranges = [range(self.num_tiles[d]) for d in reversed(range(self.ndim))]
        for rev in itertools.product(*ranges):
            yield tuple(reversed(rev))

    def box(self, t: Sequence[int], l: int):
        lo = [self.start[d][t[d]][l] for d in range(self.ndim)]
        hi = [self.end[d][t[d]][l] for d in range(self.ndim)]
        return lo, hi


def skewed_plan(loops: List[Loop], ndim: int, tilesize: Sequence[int]) -> Plan:
    """Algorithm 1.  ``tilesize[d] <= 0`` leaves dimension d untiled."""
    L = len(loops)
    # union of the index sets and the number of tiles per dimension (steps 1-6)
    start_u = [min(lp.start[d] for lp in loops) for d in range(ndim)]
    end_u = [max(lp.end[d] for lp in loops) for d in range(ndim)]
    ts = []
    num_tiles = []
    for d in range(ndim):
        size = end_u[d] - start_u[d]
        t = tilesize[d] if tilesize[d] > 0 else max(size, 1)
        ts.append(t)
        num_tiles.append(max((size - 1) // t + 1, 1))

    start = [[[0] * L for _ in range(num_tiles[d])] for d in range(ndim)]
    end = [[[0] * L for _ in range(num_tiles[d])] for d in range(ndim)]
    # read_dep[a][d][t] = [start, end]; write_dep likewise
    read_dep: Dict[int, List[List[List[float]]]] = {}
    write_dep: Dict[int, List[List[List[float]]]] = {}

    def dep(table, a):
        if a not in table:
            table[a] = [[[INF, -INF] for _ in range(num_tiles[d])] for d in range(ndim)]
        return table[a]

    # loops backward, each dimension separately (steps 2-7)
    for l in reversed(range(L)):
        lp = loops[l]
        for d in range(ndim):
            T = num_tiles[d]
            for t in range(T):
                # start index: first tile starts at the loop's start, others
                # at the previous tile's end for this loop
                s = lp.start[d] if t == 0 else end[d][t - 1][l]
                e = -INF
                if t == T - 1:
                    e = lp.end[d]
                else:
                    # read-after-write: cover what later loops of this tile
                    # read from the datasets this loop writes
                    for a in lp.args:
                        if a.writes():
                            rd = dep(read_dep, a.dat)[d][t]
                            e = min(lp.end[d], max(e, rd[1]))
                    # write-after-read / write-after-write: the next tile of
                    # this loop must not touch what later loops of this tile
                    # already overwrote
                    for a in lp.args:
                        m = a.lo(d)
                        wd = dep(write_dep, a.dat)[d][t]
                        e = min(lp.end[d], max(e, wd[1] - m))
                # no dependency: default tile size
                if e == -INF:
                    e = min(lp.end[d], start_u[d] + (t + 1) * ts[d])
                e = max(int(e), s)
                start[d][t][l] = s
                end[d][t][l] = e
                # update the dependencies with this loop's stencils
                for a in lp.args:
                    if a.reads():
                        rd = dep(read_dep, a.dat)[d][t]
                        rd[1] = max(rd[1], e + a.hi(d))
                        rd[0] = min(rd[0], s + a.lo(d))
                for a in lp.args:
                    if a.writes():
                        wd = dep(write_dep, a.dat)[d][t]
                        wd[1] = max(wd[1], e)
                        wd[0] = min(wd[0], s)
    return Plan(ndim, num_tiles, start, end)


def execute_tiled(plan: Plan, n_loops: int, run_loop) -> None:
    """Algorithm 2: for every tile in order, for every loop, call the loop on
    the tile's bounds; loops with an empty range in the tile are skipped."""
    for t in plan.tiles():
        for l in range(n_loops):
            lo, hi = plan.box(t, l)
            if all(h > o for o, h in zip(lo, hi)):
                run_loop(l, lo, hi)


def wavefronts(plan: Plan):
    """Skewed tiles grouped for wavefront-parallel execution, the alternative
    to in-order tile execution that the end of Section 4.2 names as future
    work: wavefront w holds the tiles whose indices sum to w, in the order of
    Plan.tiles().  Wavefronts run in increasing order; the tiles of one
    wavefront are meant to run at the same time."""
    waves = {}
    for t in plan.tiles():
        waves.setdefault(sum(t), []).append(t)
    return [waves[w] for w in sorted(waves)]


def wavefront_schedule(plan: Plan, n_loops: int, interleave: bool = True, reverse: bool = False):
    """(loop, lo, hi) steps of the wavefront-parallel schedule.  Within a
    wavefront the tiles either advance together, loop by loop (interleave:
    every tile runs loop l before any runs loop l + 1, as one launch per
    loop and wavefront would), or one after another; reverse flips the
    order of the tiles of each wavefront."""
    out = []
    for wave in wavefronts(plan):
        ts = wave[::-1] if reverse else wave
        order = ([(l, t) for l in range(n_loops) for t in ts] if interleave
                 else [(l, t) for t in ts for l in range(n_loops)])
        for l, t in order:
            lo, hi = plan.box(t, l)
            if all(h > o for o, h in zip(lo, hi)):
                out.append((l, lo, hi))
    return out


def max_skew(plan: Plan, d: int) -> int:
    """Largest difference over interior tile boundaries between the loops'
    ends, i.e. the skew between the bottom and top of a tile along d."""
    best = 0
    for t in range(plan.num_tiles[d] - 1):
        ends = plan.end[d][t]
        best = max(best, max(ends) - min(ends))
    return best
