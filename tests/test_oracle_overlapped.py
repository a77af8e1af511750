"""Pins of the oracle's overlapped tiles (Section 4.4).

* version stamps on random tiny chains in 1D-3D: every read of every tile
  sees the writer program order gives it, and the owned boxes end with
  program order's last writers;
* closed form: in a chain where each loop reads the previous one's output
  through a radius-r stencil, loop j of L computes r (L - 1 - j) points
  beyond the owned box on each side (clipped to its range);
* planted mistakes (a need box one point short, no overlap at all) are
  caught by the stamp check;
* the CPU overlapped execution of random weighted-sum / axpby chains is
  bit-identical to program order;
* the library's fused analysis (its per-loop recomputed extents) passes the
  same stamp check and never computes less than the oracle's need boxes.
"""
import random

import numpy as np
import pytest

from oracle.overlapped import execute_overlapped, need_boxes, owned_partition, union_range
from oracle.skewed import READ, WRITE, Arg, Loop
from oracle.stamps import check_overlapped
from randchains import op_chain_data, random_chain, random_op_chain, run_op_chain_oracle, to_oracle


def oracle_boxes(loops):
    return lambda own: need_boxes(loops, own)[0]


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_random_chains_stamps(ndim):
    rng = random.Random(4400 + ndim)
    for _ in range(200 if ndim < 3 else 60):
        loops = to_oracle(random_chain(rng, ndim))
        lo, hi = union_range(loops)
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        tiles = owned_partition(lo, hi, [rng.randint(1, 5) for _ in range(ndim)])
        check_overlapped(loops, tiles, oracle_boxes(loops))


def _pipeline(L, r, n):
    # dataset j -> loop j writes dataset j + 1 from dataset j through a radius-r stencil
    sten = [(o,) for o in range(-r, r + 1)]
    return [Loop([0], [n], [Arg(j, sten, READ), Arg(j + 1, [(0,)], WRITE)], f"l{j}") for j in range(L)]


@pytest.mark.parametrize("L,r", [(1, 1), (4, 1), (5, 2), (7, 1)])
def test_closed_form_extension(L, r):
    n = 60
    loops = _pipeline(L, r, n)
    own = ([20], [30])
    comp, live = need_boxes(loops, own)
    for j, b in enumerate(comp):
        e = r * (L - 1 - j)
        assert b == ([20 - e], [30 + e]), (j, b)
    assert live[0] == ([20 - r * L], [30 + r * L])
    # at the range boundary the boxes are clipped to the loop's range
    comp0, _ = need_boxes(loops, ([0], [10]))
    for j, b in enumerate(comp0):
        assert b == ([0], [10 + r * (L - 1 - j)])
    check_overlapped(loops, owned_partition([0], [n], [7]), oracle_boxes(loops))


def test_planted_short_box_is_caught():
    loops = _pipeline(3, 1, 30)
    tiles = owned_partition([0], [30], [6])

    def short(own):
        comp = need_boxes(loops, own)[0]
        b = comp[0]
        if b is not None and b[0][0] > 0:
            comp[0] = ([b[0][0] + 1], list(b[1]))
        return comp

    with pytest.raises(AssertionError):
        check_overlapped(loops, tiles, short)


def test_planted_no_overlap_is_caught():
    rng = random.Random(77)
    caught = 0
    for _ in range(40):
        loops = to_oracle(random_chain(rng, 2))
        lo, hi = union_range(loops)
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        tiles = owned_partition(lo, hi, [3, 3])

        def no_overlap(own):
            out = []
            for lp in loops:
                b = ([max(a, s) for a, s in zip(own[0], lp.start)], [min(a, e) for a, e in zip(own[1], lp.end)])
                out.append(None if any(h <= l for l, h in zip(*b)) else b)
            return out

        try:
            check_overlapped(loops, tiles, no_overlap)
        except AssertionError:
            caught += 1
    assert caught >= 10


def _run_op_loop(chain, arrs, l, lo, hi):
    import ctypes
    import oracle
    lp = chain["loops"][l]
    grid = oracle.Grid(chain["ndim"], 0, chain["halo"])
    args = lp["args"]
    if lp["op"] == "WSUM":
        oracle.wsum(grid, lo, hi, arrs[args[0]["dat"]], [arrs[a["dat"]] for a in args[1:]],
                    [a["stencil"] for a in args[1:]], lp["params"])
    else:
        l3, h3 = grid.box(lo, hi)
        oracle.lib().orc_axpby(l3, h3, grid.view(arrs[args[0]["dat"]]), grid.view(arrs[args[1]["dat"]]),
                               ctypes.c_double(lp["params"][0]), ctypes.c_double(lp["params"][1]))


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_overlapped_execution_bit_exact(ndim):
    rng = random.Random(900 + ndim)
    for trial in range(25 if ndim < 3 else 10):
        ch = random_op_chain(rng, ndim)
        data = op_chain_data(ch, seed=trial)
        ref = run_op_chain_oracle(ch, data)
        loops = to_oracle(ch)
        lo, hi = union_range(loops)
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        h = ch["halo"]

        def write_back(out, priv, d, own):
            sl = tuple(slice(own[0][k] + h, own[1][k] + h) for k in reversed(range(ndim)))
            out[d][sl] = priv[d][sl]

        got = execute_overlapped(loops, owned_partition(lo, hi, [rng.randint(1, 4) for _ in range(ndim)]),
                                 [np.array(a, copy=True) for a in data],
                                 lambda st, l, blo, bhi: _run_op_loop(ch, st, l, blo, bhi), write_back)
        for d in range(ch["ndat"]):
            assert np.array_equal(got[d], ref[d]), (trial, d)


def test_library_fused_extents_pass_stamps():
    """The library's fused groups (random 2D weighted-sum chains over one
    range, analysed on a host-only context) compute, per loop, the owned
    block grown by the reported extents within the range.  As overlapped
    tiles of their group those boxes pass the stamp check, and they contain
    the oracle's need boxes."""
    import paper_1704_00693_amd as tc
    from randchains import record_op_chain, star_pts
    rng = random.Random(31)
    checked = 0
    for trial in range(30):
        n = [rng.randint(12, 18), rng.randint(10, 16)]
        ndat = rng.randint(3, 6)
        loops = []
        for _ in range(rng.randint(2, 6)):
            dats = list(range(ndat))
            rng.shuffle(dats)
            ins = []
            for a in dats[1:1 + rng.randint(1, min(3, ndat - 1))]:
                sten = star_pts(2, rng.randint(1, 2)) if rng.random() < 0.6 else \
                    [(0, 0)] + [(rng.randint(-2, 2), rng.randint(-2, 2)) for _ in range(rng.randint(1, 3))]
                ins.append({"dat": a, "stencil": sten, "access": "R"})
            loops.append({"op": "WSUM", "start": [0, 0], "end": list(n), "params": [0.1] * sum(len(a["stencil"]) for a in ins),
                          "args": [{"dat": dats[0], "stencil": [(0, 0)], "access": "W"}] + ins})
        ch = {"ndim": 2, "ndat": ndat, "n": n, "halo": 4, "loops": loops}
        with tc.Context(host_only=True) as c:
            record_op_chain(c, ch)
            try:
                groups, per = c.tc_fused_plan((8, 0, 0))
            except tc.TcError:
                continue
        ol = to_oracle(ch)
        for g0, g1 in groups:
            sub = ol[g0:g1]

            def lib_boxes(own, g0=g0, g1=g1, sub=sub):
                out = []
                for l in range(g0, g1):
                    computed, left, right, below, above = per[l][:5]
                    if computed != 1:
                        out.append(None)
                        continue
                    lp = sub[l - g0]
                    b = ([max(own[0][0] - left, lp.start[0]), max(own[0][1] - below, lp.start[1])],
                         [min(own[1][0] + right, lp.end[0]), min(own[1][1] + above, lp.end[1])])
                    out.append(None if b[1][0] <= b[0][0] or b[1][1] <= b[0][1] else b)
                return out

            tiles = owned_partition([0, 0], n, [5, 4])
            check_overlapped(sub, tiles, lib_boxes)
            for own in tiles:
                need = need_boxes(sub, own)[0]
                got = lib_boxes(own)
                for nb, gb in zip(need, got):
                    if nb is None:
                        continue
                    assert gb is not None
                    assert all(a >= b for a, b in zip(nb[0], gb[0])) and all(a <= b for a, b in zip(nb[1], gb[1]))
            checked += 1
    assert checked >= 10
