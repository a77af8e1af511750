"""Brute-force dependency check of a tiled schedule (version stamps).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 4.2 states the condition a tiling must satisfy: a block of a later loop
may only contain iterations whose inputs were already computed by the blocks
executed before it, and a later loop's write must not be seen by an earlier
loop's read that, in program order, came first.  Equivalently: every read in
the tiled schedule sees exactly the writer (loop index) it sees in program
order.  This module simulates both orders on tiny grids with per-point write
stamps and compares every read.
"""
from __future__ import annotations

import itertools
from typing import Callable, Dict, Iterable, List, Sequence, Tuple

from .skewed import Loop


def _points(lo: Sequence[int], hi: Sequence[int]):
    return itertools.product(*[range(a, b) for a, b in zip(lo, hi)])


def _run(loops: List[Loop], schedule: Iterable[Tuple[int, Sequence[int], Sequence[int]]]):
    stamp: Dict[Tuple[int, Tuple[int, ...]], int] = {}
    seen: Dict[Tuple, int] = {}
    writes: Dict[int, List[Tuple[int, ...]]] = {}
    done = set()
    for l, lo, hi in schedule:
        lp = loops[l]
        for x in _points(lo, hi):
            if (l, x) in done:
                raise AssertionError(f"loop {l} point {x} executed twice")
            done.add((l, x))
            for ai, a in enumerate(lp.args):
                if a.reads():
                    for qi, q in enumerate(a.stencil):
                        y = tuple(xi + qi_ for xi, qi_ in zip(x, q))
                        key = (l, x, ai, qi)
                        seen[key] = stamp.get((a.dat, y), -1)
            for a in lp.args:
                if a.writes():
                    stamp[(a.dat, x)] = l
                    writes.setdefault(l, []).append(x)
    return seen, stamp, done


def program_order(loops: List[Loop]):
    return [(l, lp.start, lp.end) for l, lp in enumerate(loops)]


def check_schedule(loops: List[Loop], schedule) -> None:
    """Raise AssertionError if the schedule's reads or final state differ from
    program order, or if a loop's points are not each executed exactly once."""
    ref_seen, ref_stamp, ref_done = _run(loops, program_order(loops))
    got_seen, got_stamp, got_done = _run(loops, schedule)
    if ref_done != got_done:
        raise AssertionError("executed points differ from the loops' ranges")
    if ref_seen.keys() != got_seen.keys():
        missing = set(ref_seen) - set(got_seen)
        extra = set(got_seen) - set(ref_seen)
        raise AssertionError(f"coverage differs: missing {sorted(missing)[:5]} extra {sorted(extra)[:5]}")
    for k, v in ref_seen.items():
        if got_seen[k] != v:
            raise AssertionError(f"read {k} saw writer {got_seen[k]}, program order saw {v}")
    if ref_stamp != got_stamp:
        raise AssertionError("final writers differ")


def tiled_schedule(plan, n_loops: int):
    out = []
    for t in plan.tiles():
        for l in range(n_loops):
            lo, hi = plan.box(t, l)
            if all(h > o for o, h in zip(lo, hi)):
                out.append((l, lo, hi))
    return out


def check_overlapped(loops: List[Loop], tiles, compute_boxes) -> None:
    """Version-stamp check of overlapped tiles (Section 4.4).  Every tile
    starts from the chain-start state (all stamps -1) and runs every loop over
    ``compute_boxes(own)[l]`` (a (lo, hi) box or None).  Every read it makes
    must see the writer program order gives that read, and on the owned box
    every dataset's last writer must be program order's.  Raise
    AssertionError otherwise, or if the owned boxes do not cover the union of
    the loops' ranges exactly once."""
    ref_seen, ref_stamp, _ = _run(loops, program_order(loops))
    nd = len(loops[0].start)
    live = [lp for lp in loops if all(e > s for s, e in zip(lp.start, lp.end))] or loops
    lo = [min(lp.start[d] for lp in live) for d in range(nd)]
    hi = [max(lp.end[d] for lp in live) for d in range(nd)]
    owner: Dict[Tuple[int, ...], int] = {}
    for i, (olo, ohi) in enumerate(tiles):
        for x in _points(olo, ohi):
            if x in owner:
                raise AssertionError(f"point {x} owned by tiles {owner[x]} and {i}")
            owner[x] = i
    if set(owner) != set(_points(lo, hi)):
        raise AssertionError("owned boxes do not cover the union of the loop ranges")
    dats = {a.dat for lp in loops for a in lp.args}
    for i, own in enumerate(tiles):
        boxes = compute_boxes(own)
        sched = []
        for l, b in enumerate(boxes):
            if b is None:
                continue
            blo, bhi = b
            if any(bl < s or bh > e for bl, bh, s, e in zip(blo, bhi, loops[l].start, loops[l].end)):
                raise AssertionError(f"tile {i}: loop {l} box {b} leaves the loop's range")
            sched.append((l, blo, bhi))
        seen, stamp, _ = _run(loops, sched)
        for k, v in seen.items():
            if ref_seen[k] != v:
                raise AssertionError(f"tile {i}: read {k} saw writer {v}, program order saw {ref_seen[k]}")
        for x in _points(*own):
            for d in dats:
                if stamp.get((d, x), -1) != ref_stamp.get((d, x), -1):
                    raise AssertionError(f"tile {i}: dataset {d} at {x} last written by "
                                         f"{stamp.get((d, x), -1)}, program order {ref_stamp.get((d, x), -1)}")
