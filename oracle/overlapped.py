"""Overlapped tiles (Section 4.4) executed on the CPU.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 4.4 replaces the sequential skewed tiles by tiles that run
independently: a tile owns a box of the iteration space and, besides its own
points, computes redundantly the points of earlier loops that its later loops
read.  Only read dependencies shape a tile (every tile works on its own copy
of the data, so write-after-read and write-after-write hazards between tiles
cannot arise).

Written from that description:

* ``need_boxes``: walking the chain backwards from the owned box, a loop is
  computed wherever a later loop of the chain, or the final state on the
  owned box, needs a value it writes (clipped to the loop's range); the
  points it reads there, grown by its read stencils, are then needed from the
  loops before it, and a dataset a loop writes is needed before that loop
  only outside the loop's box or where the loop itself reads it.  Needed
  points are exact sets; a loop computes the hull (bounding box) of the
  needed points inside its range, which may be more than the least set but
  never less.
* ``execute_overlapped``: every tile starts from a snapshot of the chain-start
  state, runs the loops in program order over its need boxes, and writes back
  the owned box of every dataset the chain writes.

Bit-exactness against program order follows because every computed point
reads the same values in the same arithmetic as in program order.
"""
from __future__ import annotations

import copy
import itertools
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from .skewed import Loop

Box = Tuple[List[int], List[int]]  # (lo, hi), half-open per dimension


def written_datasets(loops: List[Loop]) -> List[int]:
    out = []
    for lp in loops:
        for a in lp.args:
            if a.writes() and a.dat not in out:
                out.append(a.dat)
    return out


def _box_points(b: Box):
    return itertools.product(*[range(l, h) for l, h in zip(b[0], b[1])])


def _hull_of(points) -> Optional[Box]:
    pts = list(points)
    if not pts:
        return None
    nd = len(pts[0])
    return ([min(p[d] for p in pts) for d in range(nd)], [max(p[d] for p in pts) + 1 for d in range(nd)])


def need_boxes(loops: List[Loop], own: Box) -> Tuple[List[Optional[Box]], Dict[int, Box]]:
    """Per loop, the box a tile owning ``own`` computes (None: nothing), and
    per dataset the hull of the chain-start values the tile reads or keeps.

    Needed points are kept as exact point sets (tiny grids only): the points
    of each dataset whose value at the current position of the backward walk
    some later loop, or the final state on the owned box, uses."""
    need: Dict[int, set] = {d: set(_box_points(own)) for d in written_datasets(loops)}
    comp: List[Optional[Box]] = [None] * len(loops)
    for l in reversed(range(len(loops))):
        lp = loops[l]
        rng = (lp.start, lp.end)
        want = set()
        for a in lp.args:
            if a.writes():
                want |= {p for p in need.get(a.dat, ()) if all(s <= x < e for x, s, e in zip(p, *rng))}
        box = _hull_of(want)
        comp[l] = box
        if box is None:
            continue
        inside = set(_box_points(box))
        # the loop produces its written datasets on its box: their earlier
        # values are needed there only where the loop reads them (below)
        for a in lp.args:
            if a.writes() and a.dat in need:
                need[a.dat] -= inside
        for a in lp.args:
            if a.reads():
                tgt = need.setdefault(a.dat, set())
                for q in a.stencil:
                    tgt |= {tuple(x + o for x, o in zip(p, q)) for p in inside}
    return comp, {d: _hull_of(s) for d, s in need.items() if s}


def owned_partition(lo: Sequence[int], hi: Sequence[int], tile: Sequence[int]) -> List[Box]:
    """Owned boxes of ``tile`` points per dimension covering [lo, hi) once."""
    axes = []
    for d in range(len(lo)):
        t = tile[d] if tile[d] > 0 else max(hi[d] - lo[d], 1)
        axes.append([(s, min(s + t, hi[d])) for s in range(lo[d], hi[d], t)])
    return [([r[0] for r in c], [r[1] for r in c]) for c in itertools.product(*axes)]


def union_range(loops: List[Loop]) -> Box:
    """Bounding box of the loops' iteration spaces (loops with an empty range
    have no points and do not count)."""
    live = [lp for lp in loops if all(e > s for s, e in zip(lp.start, lp.end))] or loops
    nd = len(live[0].start)
    return ([min(lp.start[d] for lp in live) for d in range(nd)],
            [max(lp.end[d] for lp in live) for d in range(nd)])


def execute_overlapped(loops: List[Loop], tiles: List[Box], state,
                       run_loop: Callable[[object, int, List[int], List[int]], None],
                       write_back: Callable[[object, object, int, Box], None]):
    """Run every tile from a snapshot of ``state`` (deep-copied), loops in
    program order over their need boxes, then ``write_back(out, private,
    dataset, owned box)`` for every written dataset.  Returns the new state."""
    out = copy.deepcopy(state)
    written = written_datasets(loops)
    for own in tiles:
        comp, _ = need_boxes(loops, own)
        priv = copy.deepcopy(state)
        for l, box in enumerate(comp):
            if box is not None:
                run_loop(priv, l, box[0], box[1])
        for d in written:
            write_back(out, priv, d, own)
    return out
