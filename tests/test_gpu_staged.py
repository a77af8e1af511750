"""GPU parity of staged groups (overlapped tiles with the group's written
datasets staged in LDS, Section 4.4) against the oracle.

* Random op chains in 1D-3D (weighted sums and axpby over random sub-ranges
  with random stencils, dot products between them), ragged sizes, every
  group the analysis accepts taken as a staged group: in the
  fused mode the datasets are identical to the oracle's program-order
  execution and to the untiled GPU run, bit for bit; reduction values agree
  with the untiled run within 1e-14 relative (double-double partials summed
  in another order).
* The heat-conduction PPCG solve (2D and 3D, ghost fills, Chebyshev steps,
  dot products inside the groups) in the fused mode against the oracle's
  FP64 solve, 1e-12 relative, with staged groups in the plan.
"""
import random
import sys

import numpy as np
import pytest

from randchains import op_chain_data, random_op_chain, run_op_chain_oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1704_00693_amd as tcm
    tcm.lib()
    return tcm


def with_dots(rng, ch):
    ndim = ch["ndim"]
    loops = list(ch["loops"])
    for _ in range(rng.randint(1, 2)):
        a, b = rng.randrange(ch["ndat"]), rng.randrange(ch["ndat"])
        st = [rng.randint(-1, 1) for _ in range(ndim)]
        en = [max(ch["n"][d] + rng.randint(-1, 1), st[d] + 1) for d in range(ndim)]
        c = [tuple([0] * ndim)]
        loops.insert(rng.randint(0, len(loops)),
                     {"op": "DOT", "start": st, "end": en, "params": [],
                      "args": [{"dat": a, "stencil": c, "access": "R"}, {"dat": b, "stencil": c, "access": "R"},
                               {"red": True}]})
    return dict(ch, loops=loops)


def run(tc, ch, data, mode):
    ndim, h = ch["ndim"], ch["halo"]
    with tc.Context() as c:
        c.tc_set_tiling(mode, (0, 0, 0))
        blk = c.tc_decl_block(ndim)
        dats = [c.tc_decl_dat(blk, ch["n"], [h] * ndim, [h] * ndim, data[d]) for d in range(ch["ndat"])]
        reds = []
        cache = {}
        for i, lp in enumerate(ch["loops"]):
            rng = [v for d in range(ndim) for v in (lp["start"][d], lp["end"][d])]
            args = []
            for a in lp["args"]:
                if a.get("red"):
                    reds.append(c.tc_decl_reduction(tc.TC_RED_SUM, f"r{len(reds)}"))
                    args.append(("red", reds[-1]))
                    continue
                key = tuple(tuple(p) for p in a["stencil"])
                if key not in cache:
                    cache[key] = c.tc_decl_stencil(list(key))
                args.append((dats[a["dat"]], cache[key], a["access"]))
            c.tc_par_loop(lp["op"], blk, rng, args, lp["params"], name=f"l{i}")
        vals = [c.tc_reduction_result(r) for r in reds]
        st = c.tc_get_stats()
        out = [c.tc_dat_read(d) for d in dats]
    return out, vals, st


@pytest.mark.parametrize("threads", ["256", "1024"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_staged_random_chains(tc, ndim, threads, monkeypatch):
    # every group the analysis accepts is taken, whatever its modelled cost,
    # with workgroups of either size
    monkeypatch.setenv("TC_STAGED", "2")
    monkeypatch.setenv("TC_STAGED_THREADS", threads)
    rng = random.Random(7300 + ndim)
    staged_runs = 0
    for it in range(14 if ndim < 3 else 10):
        ch = with_dots(rng, random_op_chain(rng, ndim, max_loops=8))
        data = op_chain_data(ch, seed=100 + it)
        plain = dict(ch, loops=[lp for lp in ch["loops"] if lp["op"] != "DOT"])
        ref = run_op_chain_oracle(plain, data)
        say(f"staged random chain ndim={ndim} threads={threads} it={it} n={ch['n']} loops={len(ch['loops'])}")
        base, vb, _ = run(tc, ch, data, tc.TC_TILING_NONE)
        got, vg, st = run(tc, ch, data, tc.TC_TILING_FUSED)
        staged_runs += st["last_groups"] > 0
        for d in range(ch["ndat"]):
            assert np.array_equal(base[d], ref[d]), (it, d)
            assert np.array_equal(got[d], ref[d]), (it, d)
        for a, b in zip(vg, vb):
            assert abs(a - b) <= 1e-14 * max(abs(b), 1e-300) + 1e-300, (a, b)
    assert staged_runs >= 5


@pytest.mark.parametrize("n,outer,ndim", [(32, 6, 2), (45, 3, 2), (12, 3, 3)])
def test_staged_ppcg(tc, n, outer, ndim):
    from oracle.tealeaf import ppcg_solve
    from paper_1704_00693_amd.apps import HeatSolver
    from synthgen import heat_problem
    hp = heat_problem(n, seed=5, ndim=ndim)
    ref = ppcg_solve(hp.density, hp.energy, outer=outer)
    say(f"staged ppcg n={n} ndim={ndim} outer={outer}")
    with tc.Context() as c:
        c.tc_set_tiling(tc.TC_TILING_FUSED, (0, 0, 0))
        s = HeatSolver(c, hp.density, hp.energy)
        info = s.solve(outer=outer, inner=10)
        x = s.field("u")
        # the solve's last flush holds one loop; a ghost fill and matvec
        # with its dot product run as a staged group
        s.halo_fill("p")
        s.loop("TEA_MATVEC_DOT", s.K() + [s.F("p", "R", s.S_star), s.F("w", "W"), ("red", s.r_sum[0])])
        c.tc_reduction_result(s.r_sum[0])
        st = c.tc_get_stats()
    assert st["last_groups"] >= 1
    assert abs(info["lmax"] - ref.lmax) <= 1e-15 * ref.lmax
    assert float(np.abs(x - ref.x).max() / np.abs(ref.x).max()) <= 1e-12
    for a, b in zip(info["rr"], ref.rr):
        assert abs(a - b) <= 1e-10 * abs(b)
