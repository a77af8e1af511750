"""Host-side tests of the library (no GPU): the shared library loads and
exports every function the header declares; recording, validation and error
reporting; the library's Algorithm 1 plans equal the oracle's plans exactly."""
import os
import random
import re

import numpy as np
import pytest

import paper_1704_00693_amd as tc
from oracle.skewed import skewed_plan
from randchains import random_op_chain, record_op_chain, to_oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "tilechain.h")).read()
    return sorted(set(re.findall(r"^(?:tc_status|const char \*)\s*(tc_\w+)\(", text, re.M)))


def test_exports_every_declared_symbol():
    L = tc.lib()
    names = header_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert sorted(tc.EXPORTS) == names


def test_library_binds_to_one_hip_runtime():
    """torch's wheel carries its own HIP runtime under the soname the library
    links: loading the library must leave exactly one HIP runtime in the
    process (the one torch uses), or the streams and memory a context borrows
    from torch would belong to another runtime.  Checked in a fresh process
    that loads the library before it imports torch itself."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1704_00693_amd as tc\n"
            "tc.lib()\n"
            "import torch\n"
            "paths = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(paths), *sorted(paths))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    fields = out.stdout.split()
    assert fields[0] == "1", out.stdout


def host_ctx():
    return tc.Context(host_only=True)


def test_status_strings():
    assert tc.tc_status_string(0) == "ok"
    assert tc.tc_status_string(-6) == "range outside halo"


def test_recording_is_delayed_and_validated():
    with host_ctx() as c:
        b = c.tc_decl_block(2)
        d0 = c.tc_decl_dat(b, [8, 8], [1, 1], [1, 1])
        d1 = c.tc_decl_dat(b, [8, 8], [1, 1], [1, 1])
        s1 = c.tc_decl_stencil([(0, 0), (1, 0), (-1, 0)])
        s2 = c.tc_decl_stencil([(0, 0), (2, 0)])
        cen = c.tc_decl_stencil([(0, 0)])
        c.tc_par_loop("WSUM", b, [0, 8, 0, 8], [(d1, cen, "W"), (d0, s1, "R")], [1, 2, 3])
        assert c.tc_pending() == 1
        # stencil leaves the halo
        with pytest.raises(tc.TcError) as e:
            c.tc_par_loop("WSUM", b, [0, 8, 0, 8], [(d1, cen, "W"), (d0, s2, "R")], [1, 2])
        assert e.value.status == tc.TC_ERR_RANGE
        # write through a non-centre stencil
        with pytest.raises(tc.TcError):
            c.tc_par_loop("WSUM", b, [0, 8, 0, 8], [(d1, s1, "W"), (d0, cen, "R")], [1])
        # wrong parameter count
        with pytest.raises(tc.TcError):
            c.tc_par_loop("WSUM", b, [0, 8, 0, 8], [(d1, cen, "W"), (d0, s1, "R")], [1, 2])
        # same dataset written and read at an offset
        with pytest.raises(tc.TcError):
            c.tc_par_loop("WSUM", b, [1, 7, 1, 7], [(d0, cen, "W"), (d0, s1, "R")], [1, 2, 3])
        # wrong access for the op
        with pytest.raises(tc.TcError):
            c.tc_par_loop("AXPBY", b, [0, 8, 0, 8], [(d1, cen, "W"), (d0, cen, "R")], [1, 2])
        # unknown op
        with pytest.raises(tc.TcError):
            c.tc_par_loop(77, b, [0, 8, 0, 8], [(d1, cen, "W")], [])
        assert c.tc_pending() == 1  # rejected calls left no trace
        # flushing a host-only context is refused
        with pytest.raises(tc.TcError) as e:
            c.tc_flush()
        assert e.value.status == tc.TC_ERR_STATE


def test_reflect_validation():
    with host_ctx() as c:
        b = c.tc_decl_block(2)
        d = c.tc_decl_dat(b, [8, 8], [2, 2], [2, 2])
        ok = c.tc_decl_stencil([(0, 0), (1, 0), (3, 0)])
        bad = c.tc_decl_stencil([(0, 0), (1, 0)])
        c.tc_par_loop("HALO_REFLECT", b, [-2, 0, 0, 8], [(d, ok, "RW")], [0, 0, 8])
        with pytest.raises(tc.TcError):
            c.tc_par_loop("HALO_REFLECT", b, [-2, 0, 0, 8], [(d, bad, "RW")], [0, 0, 8])
        with pytest.raises(tc.TcError):  # interior points are not ghosts
            c.tc_par_loop("HALO_REFLECT", b, [0, 2, 0, 8], [(d, ok, "RW")], [0, 0, 8])


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_plan_equals_oracle_plan(ndim):
    rng = random.Random(77 + ndim)
    for it in range(120):
        ch = random_op_chain(rng, ndim)
        tile = [rng.randint(1, 6) for _ in range(ndim)]
        with host_ctx() as c:
            record_op_chain(c, ch)
            num, start, end = c.tc_chain_plan(tile, len(ch["loops"]), ndim)
        ref = skewed_plan(to_oracle(ch), ndim, tile)
        assert num == ref.num_tiles
        assert start == ref.start and end == ref.end, (it, tile)


def test_paper_example_through_abi():
    """The paper's 1D example (Section 4.2) through the library's analyser."""
    with host_ctx() as c:
        b = c.tc_decl_block(1)
        d1 = c.tc_decl_dat(b, [8], [1], [1])
        d2 = c.tc_decl_dat(b, [8], [1], [1])
        cen = c.tc_decl_stencil([(0,)])
        s3 = c.tc_decl_stencil([(-1,), (0,), (1,)])
        c.tc_par_loop("COPY", b, [0, 8], [(d2, cen, "W"), (d1, cen, "R")])
        c.tc_par_loop("WSUM", b, [0, 8], [(d1, cen, "W"), (d2, s3, "R")], [1, 1, 1])
        num, start, end = c.tc_chain_plan([4], 2, 1)
    assert num == [2]
    assert [[start[0][t][0], end[0][t][0]] for t in range(2)] == [[0, 5], [5, 8]]
    assert [[start[0][t][1], end[0][t][1]] for t in range(2)] == [[0, 4], [4, 8]]


def test_fused_groups_generate_and_compile_host_only():
    """The fused mode's kernels are generated and compiled for gfx950 without
    a device (host-only context); groups are ordered, disjoint runs of at
    least two loops."""
    from paper_1704_00693_amd.apps import ChainRunner
    from synthgen import chain_2d
    ch = chain_2d(n=256)
    with tc.Context(host_only=True) as c:
        r = ChainRunner(c, ch, None)
        r.record()
        groups = c.tc_fused_groups()
        small = c.tc_fused_groups((16, 48, 3))
    for gs in (groups, small):
        assert gs
        last = 0
        for g0, g1 in gs:
            assert g0 >= last and g1 - g0 >= 2
            last = g1
    assert all(g1 - g0 <= 3 for g0, g1 in small)


@pytest.mark.parametrize("n", [9, 77, 333])
@pytest.mark.parametrize("hseg", [0, 20, 33])
def test_fused_layout_covers_range_once(n, hseg):
    """Interior wavefronts (segments of hseg rows) plus edge wavefronts
    (shorter segments around the interior rectangle) own every cell of each
    group's range exactly once; the library checks this before generating a
    group's kernels and refuses the plan otherwise."""
    from paper_1704_00693_amd.apps import ChainRunner
    from synthgen import chain_2d
    ch = chain_2d(n=n)
    with tc.Context(host_only=True) as c:
        r = ChainRunner(c, ch, None)
        r.record()
        assert c.tc_fused_groups((hseg, 0, 0))


@pytest.mark.parametrize("copy", [False, True])
def test_jacobi_plans_host_only(copy):
    """The Jacobi chain (halo-1 datasets, a one-cell Dirichlet layer) through
    the library's analysers: its Algorithm 1 plan equals the oracle's, with a
    skew of one row per later loop (each stencil loop reads its input one row
    out; each copy overwrites the array the stencil loop before it read one
    row out, a write-after-read dependency), and the fused mode puts every
    loop into a group whose kernels compile."""
    from oracle.skewed import Arg, Loop
    from paper_1704_00693_amd.apps import JacobiRunner
    from synthgen import JACOBI_POINTS, JACOBI_WEIGHTS
    n, iters = 300, 30
    pts = [tuple(p) for p in JACOBI_POINTS]
    loops = []
    for t in range(iters):
        if copy:
            loops.append(Loop([0, 0], [n, n], [Arg(1, [(0, 0)], "W"), Arg(0, pts, "R")]))
            loops.append(Loop([0, 0], [n, n], [Arg(0, [(0, 0)], "W"), Arg(1, [(0, 0)], "R")]))
        else:
            src, dst = (0, 1) if t % 2 == 0 else (1, 0)
            loops.append(Loop([0, 0], [n, n], [Arg(dst, [(0, 0)], "W"), Arg(src, pts, "R")]))
    tile = [n, 40]
    with tc.Context(host_only=True) as c:
        r = JacobiRunner(c, np.zeros((n + 2, n + 2)), JACOBI_POINTS, JACOBI_WEIGHTS, copy)
        r.record(iters)
        num, start, end = c.tc_chain_plan(tile, len(loops), 2)
        groups = c.tc_fused_groups()
    ref = skewed_plan(loops, 2, tile)
    assert num == ref.num_tiles
    assert start == ref.start and end == ref.end
    # the first tile's first loop ends one row per later loop above its last loop
    assert end[1][0][0] - end[1][0][len(loops) - 1] == len(loops) - 1
    assert groups[0][0] == 0 and groups[-1][1] == len(loops)
    assert all(a[1] == b[0] for a, b in zip(groups, groups[1:]))


@pytest.mark.parametrize("cpl,tile", [("1", (0, 0, 0)), ("2", (0, 0, 0)), ("2", (0, 240, 0))])
def test_jacobi_fused_layouts_host_only(monkeypatch, cpl, tile):
    """The fused layouts of the 8192^2 Jacobi chain, with one or two columns
    per lane (generator knob TC_JIT_CPL, read when a context starts): every
    loop in a group, groups in order, and each group's interior and edge
    wavefronts own its range exactly once (checked by the library before it
    generates and compiles the kernels)."""
    from paper_1704_00693_amd.apps import JacobiRunner
    from synthgen import JACOBI_POINTS, JACOBI_WEIGHTS
    monkeypatch.setenv("TC_JIT_CPL", cpl)
    n, iters = 8192, 48
    for copy in (False, True):
        with tc.Context(host_only=True) as c:
            r = JacobiRunner(c, np.zeros((n + 2, n + 2)), JACOBI_POINTS, JACOBI_WEIGHTS, copy)
            r.record(iters)
            groups = c.tc_fused_groups(tile)
        L = iters * (2 if copy else 1)
        assert groups[0][0] == 0 and groups[-1][1] == L
        assert all(a[1] == b[0] for a, b in zip(groups, groups[1:]))


def test_generator_error_returns_a_status(monkeypatch):
    """A failure inside the fused kernel generator reaches the caller as
    TC_ERR_STATE with its text (fault injection: every register window one
    row short), the process survives, and the context stays usable."""
    from paper_1704_00693_amd.apps import JacobiRunner
    from synthgen import JACOBI_POINTS, JACOBI_WEIGHTS
    monkeypatch.setenv("TC_JIT_TEST_SHORT_WINDOWS", "1")
    with tc.Context(host_only=True) as c:
        r = JacobiRunner(c, np.zeros((130, 130)), JACOBI_POINTS, JACOBI_WEIGHTS, False)
        r.record(6)
        with pytest.raises(tc.TcError) as e:
            c.tc_fused_groups()
        assert e.value.status == tc.TC_ERR_STATE
        assert "register window" in str(e.value)
        assert c.tc_pending() == 6
        num, start, end = c.tc_chain_plan([0, 16], 6, 2)
        assert num == [1, 8]


def test_fused_plan_reports_recomputed_extents():
    """A run of Jacobi steps (radius 1, one dataset pair) fused into one
    group: loop l of an L-loop group computes L - 1 - l extra columns and
    rows on every side of a wavefront's owned block (Section 4.4: each loop
    computes what the later loops of the group read from it)."""
    from paper_1704_00693_amd.apps import JacobiRunner
    from synthgen import JACOBI_POINTS, JACOBI_WEIGHTS
    L = 5
    with tc.Context(host_only=True) as c:
        r = JacobiRunner(c, np.zeros((258, 258)), JACOBI_POINTS, JACOBI_WEIGHTS, False)
        r.record(L)
        groups, per = c.tc_fused_plan((0, 0, L))
    assert groups == [(0, L)]
    for l, (computed, left, right, below, above, zlo, zhi) in enumerate(per):
        assert computed == 1
        assert (left, right, below, above) == (L - 1 - l,) * 4
        assert (zlo, zhi) == (0, 0)


def test_par_loops_records_like_par_loop():
    """tc_par_loops records the same loops as tc_par_loop one by one (same
    plans), stops at the first rejected loop keeping the ones before it, and
    its parameters can change between recordings."""
    from paper_1704_00693_amd.apps import HeatSolver, chebyshev_coefs
    n = 32
    theta, delta, al, be = chebyshev_coefs(1.0, 50.0, 4)
    plans = []
    for batched in (False, True):
        with tc.Context(host_only=True) as c:
            hs = HeatSolver(c, np.full((n, n), 0.5), np.full((n, n), 1.5))
            if batched:
                b = hs._batch(("p",), lambda: hs.precondition(theta, al, be, 4))
                assert c.tc_pending() == 0
                b.record()
            else:
                hs.precondition(theta, al, be, 4)
            assert c.tc_pending() == 1 + 4 * 4 + 4 + 3
            L = c.tc_pending()
            plans.append((c.tc_chain_plan((0, 8, 0), L, 2), c.tc_fused_plan()))
    assert plans[0] == plans[1]
    with tc.Context(host_only=True) as c:
        hs = HeatSolver(c, np.full((n, n), 0.5), np.full((n, n), 1.5))
        with c.capture() as loops:
            hs.precondition(theta, al, be, 2)
        bad = list(loops)
        op, blk, rng, args, params = bad[3]
        bad[3] = (op, blk, rng, args, params + (1.0,))  # one parameter too many
        b = tc.LoopBatch(c, bad)
        with pytest.raises(tc.TcError) as e:
            b.record()
        assert e.value.status == tc.TC_ERR_ARG
        assert c.tc_pending() == 3
        good = tc.LoopBatch(c, loops)
        p2 = [i for i, l in enumerate(loops) if l[0] == "TEA_P2"][0]
        good.params[good.first_param[p2]:good.first_param[p2] + 2] = (0.25, -0.5)
        good.record()
        assert c.tc_pending() == 3 + len(loops)


def test_euler_step_plan_fuses_stages_with_copies_and_primitives():
    """The fused mode's plan of one RK3 step of the 3D Euler workload (host
    only): each stage is one Runge-Kutta stage group; the first also takes
    the step's five copies Q0 = Q and its primitive-variable loop, the second
    its primitive-variable loop, and the third none (its primitives are
    datasets the chain leaves behind).  A copy over another range stays a
    loop of its own."""
    import math
    from paper_1704_00693_amd.apps import EulerRunner
    n = 24
    q = [np.zeros((n + 4,) * 3) for _ in range(5)]
    with tc.Context(host_only=True) as c:
        r = EulerRunner(c, q, n, 2 * math.pi / n)
        r.record_step(1e-3)
        assert c.tc_fused_groups() == [(0, 16), (16, 27), (28, 38)]
    with tc.Context(host_only=True) as c:
        r = EulerRunner(c, q, n, 2 * math.pi / n)
        # the same step with the last copy over the padded range
        record = c.tc_par_loop

        def widened(op, blk, rng, args, params=(), name=""):
            return record(op, blk, r.padded if name == "q0_4" else rng, args, params, name=name)

        c.tc_par_loop = widened
        r.record_step(1e-3)
        assert c.tc_fused_groups() == [(5, 16), (16, 27), (28, 38)]
