"""GPU parity of loop chains: the HIP path (untiled and skewed-tiled) against
the oracle's program-order execution, element by element.

Tolerance: 1e-12 relative to the largest magnitude of the reference dataset
(the FP64 bound the workloads fix).  Both sides evaluate every point with the
same fma order, so the values are expected to agree exactly; tiled and
untiled GPU runs must agree bit for bit (tiling only reorders points)."""
import random
import sys

import numpy as np
import pytest

import oracle
from randchains import op_chain_data, random_op_chain, record_op_chain, run_op_chain_oracle
from synthgen import chain_data, make_chain
from windows import window_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1704_00693_amd as tcm
    tcm.lib()  # raises if the library was not built
    return tcm


def rel_err(got, ref):
    scale = max(np.abs(ref).max(), 1e-300)
    return float(np.abs(got - ref).max() / scale)


def run_gpu_op_chain(tc, ch, data, mode, tile=(0, 0, 0)):
    with tc.Context() as c:
        c.tc_set_tiling(mode, tile)
        blk, dats = record_op_chain(c, ch, data)
        c.tc_flush()
        out = [c.tc_dat_read(d) for d in dats]
        st = c.tc_get_stats()
    return out, st


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_random_op_chains(tc, ndim):
    rng = random.Random(500 + ndim)
    for it in range(12):
        ch = random_op_chain(rng, ndim)
        data = op_chain_data(ch, seed=it)
        ref = run_op_chain_oracle(ch, data)
        say(f"random op chain ndim={ndim} it={it} n={ch['n']} loops={len(ch['loops'])} untiled")
        got, _ = run_gpu_op_chain(tc, ch, data, tc.TC_TILING_NONE)
        for g, r in zip(got, ref):
            assert rel_err(g, r) <= TOL
        tile = [rng.randint(1, 5) for _ in range(ndim)] + [0] * (3 - ndim)
        say(f"  skewed tile={tile}")
        got_t, st = run_gpu_op_chain(tc, ch, data, tc.TC_TILING_SKEWED, tile)
        for g, gt in zip(got, got_t):
            assert np.array_equal(g, gt)
        hseg = rng.choice([0, 3, 5, 16])
        say(f"  fused rows per wavefront segment={hseg}")
        got_f, st = run_gpu_op_chain(tc, ch, data, tc.TC_TILING_FUSED, (hseg, 0, 0))
        for g, gf in zip(got, got_f):
            assert np.array_equal(g, gf)


@pytest.mark.parametrize("ndim", [2, 3])
def test_centre_only_weighted_sums(tc, ndim):
    """Weighted sums whose inputs are all read at their centre (1 to 4
    inputs; the Jacobi copy loop is one of them) run in their own kernel,
    four rows per lane: ragged ranges, ranges reaching into the halo, one-row
    ranges (the generic kernel) and two-row ones, and boxes of the skewed
    schedule, against the oracle."""
    rng = random.Random(900 + ndim)
    h = 2
    n = [70, 37] if ndim == 2 else [45, 13, 9]
    centre = [tuple([0] * ndim)]
    loops = []
    ranges = [([0] * ndim, list(n)),
              ([-2] * ndim, [v + 2 for v in n]),
              ([3] + [1] * (ndim - 1), [n[0] - 5, 2] + list(n[2:])),
              ([0] + [5] * (ndim - 1), [n[0], 7] + [6] * (ndim - 2)),
              ([1] * ndim, [v - 1 for v in n])]
    for i in range(12):
        k = 1 + i % 4
        dats = list(range(6))
        rng.shuffle(dats)
        lo, hi = ranges[i % len(ranges)]
        ins = [{"dat": a, "stencil": centre, "access": "R"} for a in dats[1:1 + k]]
        loops.append({"op": "WSUM", "start": lo, "end": hi, "params": [rng.uniform(-1, 1) for _ in ins],
                      "args": [{"dat": dats[0], "stencil": centre, "access": "W"}] + ins})
    ch = {"ndim": ndim, "ndat": 6, "n": n, "halo": h, "loops": loops}
    data = op_chain_data(ch, seed=77 + ndim)
    ref = run_op_chain_oracle(ch, data)
    for name, mode, tile in (("untiled", tc.TC_TILING_NONE, (0, 0, 0)),
                             ("skewed", tc.TC_TILING_SKEWED, (0, 7, 4)[:ndim] + (0,) * (3 - ndim))):
        say(f"centre-only weighted sums ndim={ndim} {name}")
        got, _ = run_gpu_op_chain(tc, ch, data, mode, tile)
        for g, r in zip(got, ref):
            assert rel_err(g, r) <= TOL
            assert np.array_equal(g, r)


@pytest.mark.parametrize("ndim,n,ndat,nloops,tiles", [
    (2, 67, 12, 40, [(0, 16, 0), (24, 7, 0), (67, 67, 0)]),
    (2, 300, 12, 40, [(0, 0, 0)]),
    (3, 23, 25, 20, [(0, 0, 5), (9, 6, 4)]),
    (3, 67, 25, 12, [(0, 0, 9)]),
])
def test_synthetic_chain_small(tc, ndim, n, ndat, nloops, tiles):
    from paper_1704_00693_amd.apps import ChainRunner
    ch = make_chain(ndim, n, ndat, nloops, seed=1 + ndim)
    data = chain_data(ch)
    ref = oracle.run_chain(ch, oracle.run_chain(ch, oracle.run_chain(ch, data)))
    results = {}
    fused = [(tc.TC_TILING_FUSED, t) for t in [(0, 0, 0), (9, 0, 0), (40, 64, 0), (0, 0, 3)]] if ndim == 2 else []
    for mode, tile in [(tc.TC_TILING_NONE, (0, 0, 0))] + [(tc.TC_TILING_SKEWED, t) for t in tiles] + fused:
        say(f"synthetic chain ndim={ndim} n={n} mode={mode} tile={tile}")
        with tc.Context() as c:
            c.tc_set_tiling(mode, tile)
            r = ChainRunner(c, ch, data)
            r.run()
            r.run()  # a second flush reuses the cached plan (and the ping-pong buffers)
            r.run()  # a third replays the captured graph (per-loop schedules)
            results[(mode, tile)] = [r.read(d) for d in range(ndat)]
            st = c.tc_get_stats()
            if mode == tc.TC_TILING_FUSED:
                say(f"  fused groups={st['last_groups']} blocks={st['last_tiles']} steps={st['last_launches']}")
                assert st["last_groups"] >= 1
    # the generic weighted-sum kernel instead of the register-window one, and
    # in 3D the register-window kernel's other workgroup shapes (rows of
    # wavefronts, planes per workgroup; ragged in y and z here)
    # In 3D the fused mode keeps every loop on its own kernel (no group is
    # modelled faster); with TC_STAGED=2 every run the staged analysis
    # accepts becomes a staged group
    import os
    variants = [("generic", {"TC_WSUM_MARCH": "0"})]
    if ndim == 3:
        variants += [("rows 4", {"TC_MARCH3_ROWS": "4"}), ("rows 8", {"TC_MARCH3_ROWS": "8"}),
                     ("rows 8, 8 planes", {"TC_MARCH3_ROWS": "8", "TC_MARCH3_TZ": "8"}),
                     ("rows 4, 12 planes", {"TC_MARCH3_ROWS": "4", "TC_MARCH3_TZ": "12"}),
                     ("staged groups", {"TC_STAGED": "2"})]
    for name, env in variants:
        say(f"synthetic chain ndim={ndim} n={n} {name}")
        os.environ.update(env)
        try:
            with tc.Context() as c:
                staged = "TC_STAGED" in env
                if staged:
                    c.tc_set_tiling(tc.TC_TILING_FUSED, (0, 0, 0))
                r = ChainRunner(c, ch, data)
                r.run()
                r.run()
                r.run()
                results[name] = [r.read(d) for d in range(ndat)]
                if staged:
                    st = c.tc_get_stats()
                    say(f"  staged groups={st['last_groups']} launches={st['last_launches']}")
                    assert st["last_groups"] >= 1
        finally:
            for k in env:
                del os.environ[k]
    base = results[(tc.TC_TILING_NONE, (0, 0, 0))]
    exact = 0
    for d in range(ndat):
        assert rel_err(base[d], ref[d]) <= TOL
        exact += int(np.array_equal(base[d], ref[d]))
    say(f"  datasets bit-identical to the oracle: {exact}/{ndat}")
    for k, v in results.items():
        for d in range(ndat):
            assert np.array_equal(v[d], base[d]), k


def test_chain_sum_reduction(tc):
    from paper_1704_00693_amd.apps import ChainRunner
    ch = make_chain(3, 19, 6, 7, seed=5, reduce_last=True)
    data = chain_data(ch)
    ref = oracle.run_chain(ch, data)
    g = oracle.Grid(3, ch.n, ch.halo)
    want = oracle.exact_sum(oracle.interior(g, ref[ch.last_written()]))
    for mode, tile in [(0, (0, 0, 0)), (1, (0, 0, 4)), (1, (5, 7, 3))]:
        say(f"chain with reduction mode={mode} tile={tile}")
        with tc.Context() as c:
            c.tc_set_tiling(mode, tile)
            r = ChainRunner(c, ch, data)
            got = r.run()
        assert abs(got - want) <= 4e-16 * abs(want) + 1e-300


def test_many_reductions_in_one_flush(tc):
    """21 reductions recorded in one chain (more than one combining launch
    holds): sums over random sub-ranges and one maximum, all fetched after
    a single flush, each equal to the exactly rounded sum (double-double
    partials) or the exact maximum of its range."""
    import math
    rng = np.random.default_rng(11)
    a = rng.uniform(-1.0, 1.0, size=(44, 53))
    with tc.Context() as c:
        b = c.tc_decl_block(2)
        d = c.tc_decl_dat(b, [51, 42], [1, 1], [1, 1], a)
        cen = c.tc_decl_stencil([(0, 0)])
        reds, want = [], []
        for k in range(20):
            x0, y0 = int(rng.integers(0, 30)), int(rng.integers(0, 25))
            x1, y1 = x0 + int(rng.integers(1, 21)), y0 + int(rng.integers(1, 17))
            r = c.tc_decl_reduction(tc.TC_RED_SUM, f"s{k}")
            c.tc_par_loop("SUM", b, [x0, x1, y0, y1], [(d, cen, "R"), ("red", r)])
            reds.append(r)
            want.append(math.fsum(a[1 + y0:1 + y1, 1 + x0:1 + x1].ravel().tolist()))
        mx = c.tc_decl_reduction(tc.TC_RED_MAX, "m")
        sx = c.tc_decl_stencil([(0, 0), (1, 0)])
        sy = c.tc_decl_stencil([(0, 0), (0, 1)])
        c.tc_par_loop("TEA_GERSH", b, [0, 50, 0, 41], [(d, sx, "R"), (d, sy, "R"), ("red", mx)])
        flushes = c.tc_get_stats()["flushes"]
        got = [c.tc_reduction_result(r) for r in reds]
        assert c.tc_get_stats()["flushes"] == flushes + 1  # one flush served every fetch
        gmax = c.tc_reduction_result(mx)
    for g, w in zip(got, want):
        assert abs(g - w) <= 4e-16 * max(abs(w), 1e-300) + 1e-300, (g, w)
    # the Gershgorin bound's per-point value, in the op's order: 2 s + 1 with
    # s = ((kx(x+1) + kx(x)) + ky(y+1)) + ky(y), one rounding for 2 s + 1
    kx0, kx1 = a[1:42, 1:51], a[1:42, 2:52]
    ky0, ky1 = a[1:42, 1:51], a[2:43, 1:51]
    assert gmax == float(np.max(2.0 * (((kx1 + kx0) + ky1) + ky0) + 1.0))


def test_reduction_accumulates_until_fetched(tc):
    with tc.Context() as c:
        b = c.tc_decl_block(2)
        a = np.zeros((12, 10))
        a[1:11, 1:9] = 1.5
        d = c.tc_decl_dat(b, [8, 10], [1, 1], [1, 1], a)
        cen = c.tc_decl_stencil([(0, 0)])
        red = c.tc_decl_reduction(tc.TC_RED_SUM)
        mx = c.tc_decl_reduction(tc.TC_RED_MAX)
        c.tc_par_loop("SUM", b, [0, 8, 0, 10], [(d, cen, "R"), ("red", red)])
        c.tc_flush()
        c.tc_par_loop("SUM", b, [0, 4, 0, 10], [(d, cen, "R"), ("red", red)])
        assert c.tc_reduction_result(red) == 1.5 * 120
        assert c.tc_reduction_result(red) == 0.0
        c.tc_par_loop("SUM", b, [0, 0, 0, 10], [(d, cen, "R"), ("red", red)])  # empty range
        assert c.tc_reduction_result(red) == 0.0


def test_full_size_2d_chain_sampled(tc):
    """The 4096^2, 12-dataset, 40-loop chain in the launch configuration the
    benchmark times (untiled and skewed with the automatic tile), checked on
    sampled windows (corners, edges, interior) against the oracle."""
    from paper_1704_00693_amd.apps import ChainRunner
    from synthgen import chain_2d
    ch = chain_2d()
    data = chain_data(ch)
    n = ch.n
    centres = [(0, 0), (n - 1, n - 1), (n // 2, 3), (1234, 2987), (4000, 2048)]
    refs = [window_oracle(ch, data, c, 100) for c in centres]
    outs = {}
    for mode in (tc.TC_TILING_NONE, tc.TC_TILING_SKEWED, tc.TC_TILING_FUSED):
        say(f"full-size 2D chain mode={mode}")
        with tc.Context() as c:
            c.tc_set_tiling(mode, (0, 0, 0))
            r = ChainRunner(c, ch, data)
            r.run()
            outs[mode] = [r.read(d) for d in range(ch.ndat)]
    for mode, out in outs.items():
        for (arrs, lo, glo, ghi) in refs:
            for d in range(ch.ndat):
                ys = slice(glo[1] + 2, ghi[1] + 2)
                xs = slice(glo[0] + 2, ghi[0] + 2)
                got = out[d][ys, xs]
                want = arrs[d][glo[1] - lo[1]:ghi[1] - lo[1], glo[0] - lo[0]:ghi[0] - lo[0]]
                assert got.size > 0
                assert rel_err(got, want) <= TOL
    for d in range(ch.ndat):
        assert np.array_equal(outs[0][d], outs[1][d])
        assert np.array_equal(outs[0][d], outs[2][d])


def test_autotuner_results_identical(tc, tmp_path, monkeypatch):
    """AUTO mode measures every candidate schedule on successive flushes
    (five each: two untimed, then three timed, the median kept), then keeps
    the fastest; each flush must give the untiled answer.  The choice is
    written to the TC_TUNE_CACHE file, and a new context that reads it starts
    with the chosen schedule."""
    from paper_1704_00693_amd.apps import ChainRunner
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TC_TUNE_CACHE", str(cache))
    ch = make_chain(2, 200, 8, 12, seed=9)
    data = chain_data(ch)
    ncand, per = 7, 5  # untiled, two skewed, four fused layouts for a 2D weighted-sum chain
    scheds, tuning = [], []
    with tc.Context() as c, tc.Context() as u:
        c.tc_set_tiling(tc.TC_TILING_AUTO, (0, 0, 0))
        r = ChainRunner(c, ch, data)
        ru = ChainRunner(u, ch, data)
        for k in range(ncand * per + 4):
            say(f"autotune flush {k}")
            r.run()
            ru.run()
            st = c.tc_get_stats()
            scheds.append((st["last_mode"], tuple(st["last_tile"]), st["last_cpl"]))
            tuning.append(st["tuning"])
            for d in range(ch.ndat):
                assert np.array_equal(r.read(d), ru.read(d))
    say(f"  schedules used: {scheds}")
    T = ncand * per
    assert len(set(m for m, _, _ in scheds[:T])) == 3  # untiled, skewed and fused were tried
    assert any(cpl == 2 for _, _, cpl in scheds[:T])  # two columns per lane among them
    assert len(set(scheds[:T])) == ncand
    for i in range(0, T, per):
        assert len(set(scheds[i:i + per])) == 1  # each candidate five flushes in a row
    assert all(tuning[:T - 1]) and not any(tuning[T - 1:])
    assert len(set(scheds[T - 1:])) == 1 or len(set(scheds[T:])) == 1  # then one was kept
    chosen = scheds[-1]
    lines = cache.read_text().split()
    assert len(lines) == 7 and (int(lines[1]), int(lines[5])) == (chosen[0], chosen[2])
    with tc.Context() as c2:
        c2.tc_set_tiling(tc.TC_TILING_AUTO, (0, 0, 0))
        r2 = ChainRunner(c2, ch, data)
        r2.run()
        st = c2.tc_get_stats()
        assert st["tuning"] == 0
        assert (st["last_mode"], tuple(st["last_tile"]), st["last_cpl"]) == chosen


def test_fused_weight_change(tc):
    """Fused kernels are generated with the weights of the first flush
    compiled in; a later flush of the same chain structure with other weights
    must switch to kernels that read them (same answers as untiled)."""
    import copy
    from paper_1704_00693_amd.apps import ChainRunner
    ch = make_chain(2, 150, 6, 10, seed=11)
    ch2 = copy.deepcopy(ch)
    for lp in ch2.loops:
        lp.weights = [-0.5 * w for w in lp.weights]
    data = chain_data(ch)
    ref = oracle.run_chain(ch2, oracle.run_chain(ch, data))
    outs = {}
    for mode in (tc.TC_TILING_NONE, tc.TC_TILING_FUSED):
        say(f"weight change mode={mode}")
        with tc.Context() as c:
            c.tc_set_tiling(mode, (0, 0, 0))
            r = ChainRunner(c, ch, data)
            r.run()
            r.chain = ch2
            r.run()
            outs[mode] = [r.read(d) for d in range(ch.ndat)]
            if mode == tc.TC_TILING_FUSED:
                assert c.tc_get_stats()["last_groups"] >= 1
    for d in range(ch.ndat):
        assert rel_err(outs[0][d], ref[d]) <= TOL
        assert np.array_equal(outs[0][d], outs[2][d])


@pytest.mark.parametrize("env", [{"TC_JIT_CPL": "2"}, {"TC_JIT_WPE": "0", "TC_JIT_UNROLL": "3", "TC_JIT_PREFETCH": "1"},
                                 {"TC_JIT_BAKE": "0"}])
def test_fused_generator_variants(tc, env):
    """Kernel-generation variants (two columns per lane, compiler-chosen
    occupancy with another unroll and prefetch distance, weights read from
    the kernel arguments) give the untiled bits."""
    import os
    from paper_1704_00693_amd.apps import ChainRunner
    ch = make_chain(2, 130, 10, 24, seed=17)
    data = chain_data(ch)
    with tc.Context() as c:
        r = ChainRunner(c, ch, data)
        r.run()
        ref = [r.read(d) for d in range(ch.ndat)]
    saved = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        with tc.Context() as c:
            c.tc_set_tiling(tc.TC_TILING_FUSED, (0, 0, 0))
            r = ChainRunner(c, ch, data)
            r.run()
            got = [r.read(d) for d in range(ch.ndat)]
            say(f"generator variant {env}: groups {c.tc_get_stats()['last_groups']}")
            assert c.tc_get_stats()["last_groups"] >= 1
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    for d in range(ch.ndat):
        assert np.array_equal(ref[d], got[d])


def test_full_size_3d_chain_sampled(tc):
    """The 3D workload at its full size (384^3 FP64, 25 datasets, 60 loops of
    7- and 13-point stars, a final SUM) untiled and skewed-tiled: a corner
    window and an edge window of every dataset against the window oracle,
    all datasets identical across modes, and the SUM equal to the exactly
    rounded sum of the read-back dataset (within the double-double bound)."""
    import math
    from paper_1704_00693_amd.apps import ChainRunner
    from synthgen import chain_3d
    ch = chain_3d()
    say("generating 3D inputs")
    data = chain_data(ch)
    n, h = ch.n, ch.halo
    wins = [(0, 0, 0), (n - 1, n // 2, 0)]
    say("window oracles")
    refs = [window_oracle(ch, data, c, 124) for c in wins]
    sums, outs = {}, {}
    for mode, tile in [(tc.TC_TILING_NONE, (0, 0, 0)), (tc.TC_TILING_SKEWED, (0, 0, 0))]:
        say(f"3D chain 384^3 mode={mode}")
        with tc.Context() as c:
            c.tc_set_tiling(mode, tile)
            r = ChainRunner(c, ch, data)
            sums[mode] = r.run()
            last = r.read(ch.last_written())
            kept = {}
            for d in range(ch.ndat):
                a = r.read(d)
                for k, (arrs, lo, glo, ghi) in enumerate(refs):
                    sl = tuple(slice(glo[i] + h, ghi[i] + h) for i in reversed(range(3)))
                    want = arrs[d][tuple(slice(glo[i] - lo[i], ghi[i] - lo[i]) for i in reversed(range(3)))]
                    got = a[sl]
                    assert got.size > 0
                    assert rel_err(got, want) <= TOL
                kept[d] = a[::7, ::5, ::3].copy()
            outs[mode] = kept
        inner = last[h:h + n, h:h + n, h:h + n]
        exact = math.fsum(inner.ravel().tolist())
        bound = 1e-15 * float(np.abs(inner).sum())
        say(f"  sum {sums[mode]!r} exact {exact!r}")
        assert abs(sums[mode] - exact) <= bound
        del last, inner
    assert sums[0] == sums[1]
    for d in range(ch.ndat):
        assert np.array_equal(outs[0][d], outs[1][d])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fused_offset_ranges(tc, seed):
    """Fused groups over a range that starts away from the origin (x start
    not on a 16-column line) of a non-square grid with wide halos: the
    interior grid sits inside the range with edge bands on all four sides.
    Fused results equal the untiled ones bit for bit, which match the
    oracle."""
    from randchains import star_pts
    rng = random.Random(900 + seed)
    n = [203, 171]
    ndat = 6
    st = [rng.randint(3, 20), rng.randint(1, 20)]
    en = [n[0] - rng.randint(0, 10), n[1] - rng.randint(0, 10)]
    loops = []
    for _ in range(rng.randint(10, 16)):
        dats = list(range(ndat))
        rng.shuffle(dats)
        ins = []
        for a in dats[1:1 + rng.randint(1, 3)]:
            if rng.random() < 0.6:
                sten = star_pts(2, rng.randint(1, 2))
            else:
                sten = [(0, 0)] + [tuple(rng.randint(-2, 2) for _ in range(2)) for _ in range(rng.randint(1, 4))]
            ins.append({"dat": a, "stencil": sten, "access": "R"})
        w = [rng.uniform(-0.3, 0.3) for a in ins for _ in a["stencil"]]
        loops.append({"op": "WSUM", "start": st, "end": en, "params": w,
                      "args": [{"dat": dats[0], "stencil": [(0, 0)], "access": "W"}] + ins})
    ch = {"ndim": 2, "ndat": ndat, "n": n, "halo": 4, "loops": loops}
    data = op_chain_data(ch, seed=seed)
    ref = run_op_chain_oracle(ch, data)
    base, _ = run_gpu_op_chain(tc, ch, data, tc.TC_TILING_NONE)
    for g, r in zip(base, ref):
        assert rel_err(g, r) <= TOL
    for tile in [(0, 0, 0), (24, 0, 0), (0, 96, 4)]:
        got, st_ = run_gpu_op_chain(tc, ch, data, tc.TC_TILING_FUSED, tile)
        say(f"offset range {st}..{en} loops={len(loops)} fused tile={tile}: groups {st_['last_groups']}")
        assert st_["last_groups"] >= 1
        for g, gf in zip(base, got):
            assert np.array_equal(g, gf)
