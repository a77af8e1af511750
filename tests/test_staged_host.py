"""Host-side checks of the library's staged groups (overlapped tiles staged in
LDS, Section 4.4): analysed on host-only contexts, no GPU.

* On random op chains in 1D-3D (weighted sums and axpby over random
  sub-ranges, dot products), every tile's computed boxes, as the library
  reports them, pass the oracle's version-stamp check of overlapped tiles:
  every read sees the writer program order gives it, the owned boxes end
  with program order's last writers, and the owned boxes cover the union
  of the loop ranges exactly once.  They also contain the oracle's need
  boxes for the same owned box.
* The heat-conduction PPCG chain between two reduction fetches (update, ten
  Chebyshev steps with their ghost fills, two dot products) is one staged
  group, and its interior tile recomputes ten points around the owned box
  for the first loops (one per Chebyshev step).
"""
import random

import numpy as np
import pytest

import paper_1704_00693_amd as tc
from oracle.overlapped import need_boxes
from oracle.skewed import READ, Arg, Loop
from oracle.stamps import check_overlapped
from randchains import random_op_chain, record_op_chain, to_oracle


def with_dots(rng, ch):
    """Insert dot-product loops (reads only, one reduction) at random places."""
    ndim = ch["ndim"]
    loops = list(ch["loops"])
    for _ in range(rng.randint(0, 2)):
        a, b = rng.randrange(ch["ndat"]), rng.randrange(ch["ndat"])
        st = [rng.randint(-1, 1) for _ in range(ndim)]
        en = [max(ch["n"][d] + rng.randint(-1, 1), st[d]) for d in range(ndim)]
        c = [tuple([0] * ndim)]
        loops.insert(rng.randint(0, len(loops)),
                     {"op": "DOT", "start": st, "end": en, "params": [],
                      "args": [{"dat": a, "stencil": c, "access": "R"}, {"dat": b, "stencil": c, "access": "R"},
                               {"red": True}]})
    return dict(ch, loops=loops)


def record(c, ch):
    ndim, h = ch["ndim"], ch["halo"]
    blk = c.tc_decl_block(ndim)
    dats = [c.tc_decl_dat(blk, ch["n"], [h] * ndim, [h] * ndim, None) for _ in range(ch["ndat"])]
    red = c.tc_decl_reduction(tc.TC_RED_SUM, "r")
    cache = {}
    for i, lp in enumerate(ch["loops"]):
        rng = [v for d in range(ndim) for v in (lp["start"][d], lp["end"][d])]
        args = []
        for a in lp["args"]:
            if a.get("red"):
                args.append(("red", red))
                continue
            key = tuple(tuple(p) for p in a["stencil"])
            if key not in cache:
                cache[key] = c.tc_decl_stencil(list(key))
            args.append((dats[a["dat"]], cache[key], a["access"]))
        c.tc_par_loop(lp["op"], blk, rng, args, lp["params"], name=f"l{i}")


def oracle_loops(ch):
    out = []
    for lp in ch["loops"]:
        args = [Arg(a["dat"], [tuple(p) for p in a["stencil"]], a["access"]) for a in lp["args"] if not a.get("red")]
        out.append(Loop(list(lp["start"]), list(lp["end"]), args))
    return out


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_staged_tiles_pass_stamps(ndim, monkeypatch):
    # every group the analysis accepts is taken, whatever its modelled cost
    monkeypatch.setenv("TC_STAGED", "2")
    rng = random.Random(6100 + ndim)
    groups_checked = 0
    for trial in range(40 if ndim < 3 else 25):
        ch = with_dots(rng, random_op_chain(rng, ndim, max_loops=7))
        with tc.Context(host_only=True) as c:
            record(c, ch)
            try:
                groups, per = c.tc_fused_plan()
            except tc.TcError:
                continue
            staged = []
            for gi in range(len(groups)):
                g0, g1, ext, tiles = c.tc_staged_tiles(gi)
                if tiles:
                    staged.append((g0, g1, tiles))
        loops = oracle_loops(ch)
        for g0, g1, tiles in staged:
            sub = loops[g0:g1]
            cut = lambda b: None if b is None else (list(b[0][:ndim]), list(b[1][:ndim]))
            by_own = {(tuple(o[0][:ndim]), tuple(o[1][:ndim])): [cut(b) for b in boxes] for o, boxes in tiles}
            owned = [(list(k[0]), list(k[1])) for k in by_own]
            # the stamp check uses dataset loops; a dot loop reads only
            check_overlapped(sub, owned, lambda own: by_own[(tuple(own[0]), tuple(own[1]))])
            for own in owned:
                need = need_boxes(sub, own)[0]
                got = by_own[(tuple(own[0]), tuple(own[1]))]
                for l, (nb, gb) in enumerate(zip(need, got)):
                    if nb is None or not sub[l].args or not any(a.writes() for a in sub[l].args):
                        continue
                    assert gb is not None, (trial, l)
                    assert all(a >= b for a, b in zip(nb[0], gb[0])) and all(a <= b for a, b in zip(nb[1], gb[1]))
            groups_checked += 1
    assert groups_checked >= 10


def test_ppcg_chain_is_one_staged_group(monkeypatch):
    # without the dedicated Chebyshev-step groups
    monkeypatch.setenv("TC_CHEB", "0")
    from paper_1704_00693_amd.apps import HeatSolver, chebyshev_coefs
    n = 256
    with tc.Context(host_only=True) as c:
        hs = HeatSolver(c, np.full((n, n), 0.5), np.full((n, n), 1.5))
        theta, delta, al, be = chebyshev_coefs(1.0, 100.0, 10)
        hs.loop("TEA_CG_UPDATE", [hs.F("u", "RW"), hs.F("r", "RW"), hs.F("p", "R"), hs.F("w", "R")], [0.3])
        hs.precondition(theta, al, be, 10)
        hs.dot("r", "z", hs.r_sum[1])
        hs.dot("r", "r", hs.r_sum[2])
        L = c.tc_pending()
        groups, per = c.tc_fused_plan()
        g0, g1, ext, tiles = c.tc_staged_tiles(0)
    # one staged group holds the preconditioner and the dot products (the
    # x, r update before it joins or runs alone, as the cost model prefers)
    assert len(groups) == 1 and groups[0][0] <= 1 and groups[0][1] == L
    assert all(p[0] == 2 for p in per[1:])
    # preconditioner set-up: one point per Chebyshev step on every side
    assert per[1][1:5] == (10, 10, 10, 10)
    if groups[0][0] == 0:
        assert per[0][1:5] == (10, 10, 10, 10)
    # the last preconditioner step and the dot products: the owned box only
    assert per[-1][1:5] == (0, 0, 0, 0) and per[-3][1:5] == (0, 0, 0, 0)
    assert tiles and (g0, g1) == groups[0]


@pytest.mark.parametrize("inner", [1, 3, 4, 10, 12])
def test_ppcg_chebyshev_steps_become_chebyshev_groups(inner):
    """The preconditioner's Chebyshev steps (four ghost fills of sd, TEA_P1,
    TEA_P2) form runs of at most five steps, each one Chebyshev group (plan
    code 4); the last step, without TEA_P2, ends the last group; the first
    group takes the CG update and the preconditioner's set-up; the dot
    products after them run on their own."""
    from paper_1704_00693_amd.apps import HeatSolver, chebyshev_coefs
    n = 256
    with tc.Context(host_only=True) as c:
        hs = HeatSolver(c, np.full((n, n), 0.5), np.full((n, n), 1.5))
        theta, delta, al, be = chebyshev_coefs(1.0, 100.0, inner)
        hs.loop("TEA_CG_UPDATE", [hs.F("u", "RW"), hs.F("r", "RW"), hs.F("p", "R"), hs.F("w", "R")], [0.3])
        hs.precondition(theta, al, be, inner)
        hs.dot("r", "z", hs.r_sum[1])
        hs.dot("r", "r", hs.r_sum[2])
        L = c.tc_pending()
        groups, per = c.tc_fused_plan()
    # the update is loop 0, the set-up loop 1, the steps occupy loops
    # [2, L - 2): 6 loops each, the last one 5; the first group takes the
    # update and the set-up
    assert 2 + 6 * inner - 1 == L - 2
    assert len(groups) >= (inner + 4) // 5
    assert groups[0][0] == 0 and groups[-1][1] == L - 2
    for (a0, a1), (b0, b1) in zip(groups, groups[1:]):
        assert a1 == b0
    for g0, g1 in groups[:-1]:
        g0 += 2 if g0 == 0 else 0
        assert (g1 - g0) % 6 == 0 and (g1 - g0) // 6 <= 5
    last0 = groups[-1][0] + (2 if groups[-1][0] == 0 else 0)
    assert (groups[-1][1] - last0 + 1) % 6 == 0 and (groups[-1][1] - last0 + 1) // 6 <= 5
    for g0, g1 in groups:
        assert all(per[i][0] == 4 for i in range(g0, g1))
    assert [p[0] for p in per[-2:]] == [-1, -1]


def test_chebyshev_run_needs_the_recorded_fill_pattern():
    from paper_1704_00693_amd.apps import HeatSolver, chebyshev_coefs
    n = 64
    with tc.Context(host_only=True) as c:
        hs = HeatSolver(c, np.full((n, n), 0.5), np.full((n, n), 1.5))
        theta, delta, al, be = chebyshev_coefs(1.0, 100.0, 3)
        hs.loop("TEA_PRECON_INIT", [hs.F("r", "R"), hs.F("rt", "W"), hs.F("sd", "W"), hs.F("z", "W")], [theta])
        hs.halo_fill("sd")
        hs.loop("TEA_P1", hs.K() + [hs.F("sd", "R", hs.S_star), hs.F("rt", "RW"), hs.F("z", "RW")])
        hs.loop("TEA_P2", [hs.F("sd", "RW"), hs.F("rt", "R")], [al[0], be[0]])
        # the second step fills only three sides: no run through it
        for axis, side in ((0, 0), (0, 1), (1, 0)):
            rng = [-2, 0, 0, n] if (axis, side) == (0, 0) else [n, n + 2, 0, n] if axis == 0 else [-2, n + 2, -2, 0]
            c.tc_par_loop("HALO_REFLECT", hs.blk, rng, [(hs.f["sd"], hs.S_reflect[(axis, side)], "RW")],
                          [axis, side, n])
        hs.loop("TEA_P1", hs.K() + [hs.F("sd", "R", hs.S_star), hs.F("rt", "RW"), hs.F("z", "RW")])
        groups, per = c.tc_fused_plan()
    assert (0, 7) in groups  # with the set-up
    assert all(per[i][0] != 4 for i in range(7, len(per)))


def test_chebyshev_runs_need_twice_the_ghost_depth():
    """A grid narrower than twice the ghost depth has cells that mirror ghosts
    on both sides: no Chebyshev group takes it (n = 3, depth 2); n = 4 does."""
    from paper_1704_00693_amd.apps import HeatSolver, chebyshev_coefs
    for n, want in ((3, False), (4, True)):
        with tc.Context(host_only=True) as c:
            hs = HeatSolver(c, np.full((n, n), 0.5), np.full((n, n), 1.5))
            theta, delta, al, be = chebyshev_coefs(1.0, 100.0, 4)
            hs.loop("TEA_PRECON_INIT", [hs.F("r", "R"), hs.F("rt", "W"), hs.F("sd", "W"), hs.F("z", "W")], [theta])
            hs.precondition(theta, al, be, 4)
            groups, per = c.tc_fused_plan()
        assert any(p[0] == 4 for p in per) == want, n
