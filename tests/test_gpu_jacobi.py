"""GPU parity of the Jacobi heat-equation iteration (the paper's baseline
benchmark: five-point weighted stencil, one Dirichlet layer, copy and
non-copy variants) against the oracle, in every execution mode.

Small grids: the whole field against the oracle, element by element.  The
benchmark size (8192^2, 250 iterations, the modes the benchmark times):
sampled blocks against the window oracle (corners, edges and the middle),
and a sine mode over the whole field against its closed-form decay.
Tolerance 1e-12 relative (the FP64 bound of the workload); the execution
modes must agree with each other bit for bit."""
import math
import sys

import numpy as np
import pytest

from oracle.jacobi import jacobi
from synthgen import JACOBI_POINTS, JACOBI_WEIGHTS, jacobi_field, jacobi_mode
from windows import jacobi_window

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
    tcm.lib()
    return tcm


def rel_err(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def run_gpu(tc, u0, iters, copy, mode, tile=(0, 0, 0), chunks=1, cpl=1):
    """cpl: columns per lane of the fused kernels (generator knob
    TC_JIT_CPL, read when the context starts; restored afterwards)."""
    import os
    from paper_1704_00693_amd.apps import JacobiRunner
    old = os.environ.get("TC_JIT_CPL")
    os.environ["TC_JIT_CPL"] = str(cpl)
    try:
        c = tc.Context()
    finally:
        if old is None:
            del os.environ["TC_JIT_CPL"]
        else:
            os.environ["TC_JIT_CPL"] = old
    with c:
        c.tc_set_tiling(mode, tile)
        r = JacobiRunner(c, u0, JACOBI_POINTS, JACOBI_WEIGHTS, copy)
        left = iters
        for k in range(chunks):
            step = left // (chunks - k)
            r.run(step)
            left -= step
        out = r.result()
        st = c.tc_get_stats()
    return out, st


def modes(tc):
    return [("untiled", tc.TC_TILING_NONE, (0, 0, 0), 1),
            ("skewed", tc.TC_TILING_SKEWED, (0, 0, 0), 1),
            ("skewed 0x23", tc.TC_TILING_SKEWED, (0, 23, 0), 1),
            ("fused", tc.TC_TILING_FUSED, (0, 0, 0), 1),
            ("fused hseg 16", tc.TC_TILING_FUSED, (16, 0, 0), 1),
            ("fused 2 columns per lane", tc.TC_TILING_FUSED, (0, 0, 0), 2),
            ("fused 2 columns per lane, 240 registers", tc.TC_TILING_FUSED, (0, 240, 0), 2)]


@pytest.mark.parametrize("n,iters", [(203, 21), (130, 40), (64, 7)])
@pytest.mark.parametrize("copy", [False, True])
def test_jacobi_small_all_modes(tc, n, iters, copy):
    u0 = jacobi_field(n, seed=n)
    ref = jacobi(u0, iters, JACOBI_POINTS, JACOBI_WEIGHTS, copy)
    base = None
    for name, mode, tile, cpl in modes(tc):
        say(f"jacobi n={n} iters={iters} copy={copy} {name}")
        got, st = run_gpu(tc, u0, iters, copy, mode, tile, cpl=cpl)
        err = rel_err(got, ref)
        say(f"  error {err:.2e}, identical to the oracle: {np.array_equal(got, ref)}, "
            f"launches {st['last_launches']}, groups {st['last_groups']}")
        assert err <= TOL
        if mode == tc.TC_TILING_FUSED:
            assert st["last_groups"] >= 1
        if base is None:
            base = got
        else:
            assert np.array_equal(got, base), name


@pytest.mark.parametrize("copy", [False, True])
def test_jacobi_flushes_and_autotuner(tc, copy):
    """The iterations split over several flushes (the non-copy variant
    continues its alternation across them, and chunks of odd length give two
    chain structures) under the autotuner, which times its candidates on the
    first flushes and then keeps the fastest."""
    n, iters = 150, 61
    u0 = jacobi_field(n, seed=17)
    ref = jacobi(u0, iters, JACOBI_POINTS, JACOBI_WEIGHTS, copy)
    say(f"jacobi autotuned, copy={copy}: {iters} iterations in 20 flushes")
    got, st = run_gpu(tc, u0, iters, copy, tc.TC_TILING_AUTO, chunks=20)
    assert rel_err(got, ref) <= TOL
    assert st["flushes"] >= 20


@pytest.fixture(scope="module")
def field8192():
    return jacobi_field(8192, seed=5)


@pytest.mark.parametrize("copy", [False, True])
def test_jacobi_benchmark_size_sampled(tc, field8192, copy):
    """8192^2, 250 iterations, untiled and fused (both fused layouts the
    benchmark times): sampled 32 x 32 blocks against the window oracle, the
    Dirichlet layer unchanged, the modes identical."""
    n, iters, s = 8192, 250, 32
    u0 = field8192
    blocks = [(0, 0), (0, n - s), (n - s, 0), (n - s, n - s), (4093, 2050), (17, 6000), (7000, 300)]
    refs = [jacobi_window(u0, iters, JACOBI_POINTS, JACOBI_WEIGHTS, copy, y, x, s) for y, x in blocks]
    outs = []
    for name, mode, tile, cpl in (("fused", tc.TC_TILING_FUSED, (0, 0, 0), 1),
                                  ("fused 2 columns, 240 registers", tc.TC_TILING_FUSED, (0, 240, 0), 2),
                                  ("untiled", tc.TC_TILING_NONE, (0, 0, 0), 1)):
        say(f"jacobi 8192^2 x 250 copy={copy} {name}")
        got, st = run_gpu(tc, u0, iters, copy, mode, tile, cpl=cpl)
        say(f"  launches {st['last_launches']}, groups {st['last_groups']}")
        for (y, x), ref in zip(blocks, refs):
            blk = got[y + 1:y + 1 + s, x + 1:x + 1 + s]
            assert rel_err(blk, ref) <= TOL, (y, x)
        assert np.array_equal(got[0, :], u0[0, :]) and np.array_equal(got[-1, :], u0[-1, :])
        assert np.array_equal(got[:, 0], u0[:, 0]) and np.array_equal(got[:, -1], u0[:, -1])
        outs.append(got)
        del got
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("cpl,tile", [(1, (0, 0, 0)), (2, (0, 240, 0))])
@pytest.mark.parametrize("copy", [False, True])
def test_jacobi_benchmark_size_sine_mode(tc, copy, cpl, tile):
    """Every cell of the 8192^2 field after 250 fused iterations against the
    closed form: a discrete sine mode decays by its eigenvalue per iteration."""
    n, iters, k, l = 8192, 250, 64, 100
    u0 = jacobi_mode(n, k, l)
    lam = 0.2 * (1.0 + 2.0 * math.cos(math.pi * k / (n + 1)) + 2.0 * math.cos(math.pi * l / (n + 1)))
    say(f"jacobi 8192^2 sine mode ({k},{l}) copy={copy} fused, {cpl} column(s) per lane, tile {tile}")
    got, st = run_gpu(tc, u0, iters, copy, tc.TC_TILING_FUSED, tile, cpl=cpl)
    assert st["last_groups"] >= 1
    err = float(np.abs(got - lam ** iters * u0).max())
    say(f"  max error against the closed form {err:.2e}")
    assert err <= 16 * iters * np.finfo(float).eps
