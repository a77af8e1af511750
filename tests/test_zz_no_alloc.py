"""The reduction entry point that allocates nothing (tc_reduction_result_static,
for callers that cannot allocate device memory) against tc_reduction_result.

Two contexts get the same seeded data and make the same sequence of calls;
one of them makes its last two calls through the static entry point, the
second over a smaller range than the first.  Reduction values and every
dataset must be bit-identical (the same kernels run; only where their
partial results live differs).  Requests the static scratch cannot hold,
and chains that still need kernels compiled or an autotuner choice, are
refused with a clear error and stay pending."""
import sys

import numpy as np
import pytest

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


N, H = 300, 2


def setup(tc, c):
    from synthgen import uniform_block
    blk = c.tc_decl_block(2)
    shape = (N + 2 * H, N + 2 * H)
    size = shape[0] * shape[1]
    dats = [c.tc_decl_dat(blk, [N, N], [H, H], [H, H], uniform_block(77, k * size, size, -1, 1).reshape(shape))
            for k in range(3)]
    st5 = c.tc_decl_stencil([(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)])
    st9 = c.tc_decl_stencil([(0, 0), (-1, 0), (1, 0), (-2, 0), (2, 0), (0, -1), (0, 1), (0, -2), (0, 2)])
    st1 = c.tc_decl_stencil([(0, 0)])
    reds = [c.tc_decl_reduction(tc.TC_RED_SUM, "dot"), c.tc_decl_reduction(tc.TC_RED_SUM, "sum"),
            c.tc_decl_reduction(tc.TC_RED_SUM, "sq")]
    return blk, dats, (st1, st5, st9), reds


def record(c, blk, dats, st, reds, m):
    st1, st5, st9 = st
    rng = [0, m, 0, m]
    w = [0.11 * (k + 1) * (-1) ** k for k in range(14)]
    c.tc_par_loop("WSUM", blk, rng, [(dats[2], st1, "W"), (dats[0], st5, "R"), (dats[1], st9, "R")], w)
    c.tc_par_loop("WSUM", blk, rng, [(dats[0], st1, "W"), (dats[2], st9, "R"), (dats[1], st5, "R")], w)
    c.tc_par_loop("AXPBY", blk, rng, [(dats[1], st1, "RW"), (dats[2], st1, "R")], [0.25, -0.5])
    c.tc_par_loop("DOT", blk, rng, [(dats[1], st1, "R"), (dats[2], st1, "R"), ("red", reds[0])])
    c.tc_par_loop("SUM", blk, rng, [(dats[0], st1, "R"), ("red", reds[1])])
    c.tc_par_loop("DOT", blk, rng, [(dats[0], st1, "R"), (dats[0], st1, "R"), ("red", reds[2])])


def fetch(c, reds, static):
    get = c.tc_reduction_result_static if static else c.tc_reduction_result
    return [get(r) for r in reds]


@pytest.mark.parametrize("mode,tile,warm", [
    ("none", (0, 0, 0), False),
    ("none", (0, 0, 0), True),
    ("skewed", (0, 64, 0), False),
    ("fused", (0, 0, 0), True),
])
def test_static_matches_regular(tc, mode, tile, warm):
    m = {"none": tc.TC_TILING_NONE, "skewed": tc.TC_TILING_SKEWED, "fused": tc.TC_TILING_FUSED}[mode]
    sizes = [N, N - 117]  # the second call covers a smaller range
    results = {}
    for static in (False, True):
        with tc.Context() as c:
            c.tc_set_tiling(m, tile)
            blk, dats, st, reds = setup(tc, c)
            got = []
            if warm:  # plans (and, fused, compiled kernels and second buffers) from regular calls
                for s in sizes:
                    record(c, blk, dats, st, reds, s)
                    got.append(fetch(c, reds, False))
            for s in sizes:
                say(f"static={static} mode={mode} warm={warm} range={s}")
                record(c, blk, dats, st, reds, s)
                got.append(fetch(c, reds, static))
            results[static] = (got, [c.tc_dat_read(d) for d in dats])
    (g0, d0), (g1, d1) = results[False], results[True]
    assert g0 == g1, (g0, g1)
    for a, b in zip(d0, d1):
        assert np.array_equal(a, b)
    assert all(np.isfinite(v) for row in g1 for v in row)


def test_static_refusals(tc):
    # the autotuner has not chosen a schedule: refused, chain kept
    with tc.Context() as c:
        c.tc_set_tiling(tc.TC_TILING_AUTO, (0, 0, 0))
        blk, dats, st, reds = setup(tc, c)
        record(c, blk, dats, st, reds, N)
        with pytest.raises(tc.TcError) as e:
            c.tc_reduction_result_static(reds[0])
        assert e.value.status == tc.TC_ERR_STATE and "autotuner" in str(e.value)
        assert c.tc_pending() == 6
    # a fused plan that was never built: refused, chain kept; after one
    # regular call the same structure goes through
    with tc.Context() as c:
        c.tc_set_tiling(tc.TC_TILING_FUSED, (0, 0, 0))
        blk, dats, st, reds = setup(tc, c)
        record(c, blk, dats, st, reds, N)
        with pytest.raises(tc.TcError) as e:
            c.tc_reduction_result_static(reds[0])
        assert e.value.status == tc.TC_ERR_STATE and "tc_flush" in str(e.value)
        assert c.tc_pending() == 6
        first = c.tc_reduction_result(reds[0])
        assert np.isfinite(first) and c.tc_pending() == 0
        record(c, blk, dats, st, reds, N)
        v = c.tc_reduction_result_static(reds[0])
        assert np.isfinite(v) and c.tc_pending() == 0


def test_static_scratch_limit(tc):
    """A sum over 17 million points needs 66407 workgroup partials (two
    doubles each) plus its result: more than the 131072 doubles of the
    static scratch, so the call is refused and the chain stays pending; the
    regular call then computes it."""
    n = 17_000_000
    with tc.Context() as c:
        blk = c.tc_decl_block(1)
        a = c.tc_decl_dat(blk, [n], [0], [0], np.full(n, 0.5))
        s1 = c.tc_decl_stencil([(0,)])
        r = c.tc_decl_reduction(tc.TC_RED_SUM, "s")
        c.tc_par_loop("SUM", blk, [0, n], [(a, s1, "R"), ("red", r)])
        with pytest.raises(tc.TcError) as e:
            c.tc_reduction_result_static(r)
        assert e.value.status == tc.TC_ERR_ARG and "scratch" in str(e.value)
        assert c.tc_pending() == 1
        assert c.tc_reduction_result(r) == 0.5 * n
