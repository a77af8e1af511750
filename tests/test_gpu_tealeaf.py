"""GPU parity of the heat-conduction PPCG solve (the TeaLeaf-style workload):
every loop runs through the library (untiled, skewed-tiled, fused modes) and
is compared with the oracle's program-order FP64 solve.

Tolerance: 1e-12 relative (max-norm) on the solution; reductions are
double-double on the GPU and exactly rounded in the oracle, so the scalar
histories agree to a few ulps and the iterates stay within the bound over
50 outer iterations."""
import math
import sys

import numpy as np
import pytest

from oracle.tealeaf import ppcg_solve
from synthgen import heat_problem

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


def gpu_solve(tc, hp, outer, mode=0, tile=(0, 0, 0), tol=None):
    from paper_1704_00693_amd.apps import HeatSolver
    with tc.Context() as c:
        c.tc_set_tiling(mode, tile)
        s = HeatSolver(c, hp.density, hp.energy)
        info = s.solve(outer=outer, inner=10, tol=tol)
        x = s.field("u")
        st = c.tc_get_stats()
    return x, info, st


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("n,outer,ndim", [(32, 6, 2), (45, 3, 2), (12, 3, 3)])
def test_ppcg_small(tc, n, outer, ndim):
    hp = heat_problem(n, seed=5, ndim=ndim)
    ref = ppcg_solve(hp.density, hp.energy, outer=outer)
    say(f"ppcg n={n} ndim={ndim} outer={outer}")
    x, info, _ = gpu_solve(tc, hp, outer)
    assert abs(info["lmax"] - ref.lmax) <= 1e-15 * ref.lmax
    assert rel(x, ref.x) <= TOL
    for a, b in zip(info["rr"], ref.rr):
        assert abs(a - b) <= 1e-10 * abs(b)


def test_ppcg_tealeaf_256_all_modes(tc):
    """The 256^2 workload: 50 outer iterations of 10 Chebyshev steps, seed 0."""
    hp = heat_problem(256, seed=0)
    ref = ppcg_solve(hp.density, hp.energy, outer=50)
    xs = {}
    for mode, tile in [(0, (0, 0, 0)), (1, (0, 64, 0)), (2, (0, 0, 0))]:
        say(f"ppcg 256^2 mode={mode} tile={tile}")
        x, info, st = gpu_solve(tc, hp, 50, mode, tile)
        xs[mode] = x
        assert info["iterations"] == 50
        e = rel(x, ref.x)
        say(f"  relative error vs oracle {e:.3e}; rr {math.sqrt(info['rr'][-1]) / info['bnorm']:.3e}")
        assert e <= TOL
    assert np.array_equal(xs[0], xs[1])
    assert np.array_equal(xs[0], xs[2])


def test_ppcg_converges_to_tolerance(tc):
    hp = heat_problem(40, seed=2)
    ref = ppcg_solve(hp.density, hp.energy, tol=1e-10, max_iter=500)
    x, info, _ = gpu_solve(tc, hp, 0, tol=1e-10)
    assert info["iterations"] == ref.iterations
    assert rel(x, ref.x) <= TOL


def true_residual(hp, x):
    """||b - A x|| / ||b|| evaluated by the oracle's FP64 operator."""
    from oracle.tealeaf import HeatOracle
    o = HeatOracle(hp.density, hp.energy)
    lmax = o.setup()
    h, n = o.halo, o.n
    o.f["u"][tuple([slice(h, h + n)] * o.ndim)] = x
    b = o.inner("u0")
    return float(np.linalg.norm(b - o.apply_A("u")) / np.linalg.norm(b)), lmax


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("n,ndim,tol", [(40, 2, 1e-8), (96, 2, 1e-10), (16, 3, 1e-8)])
def test_mixed_precision_refinement(tc, n, ndim, tol, fused):
    """FP32 sweeps + FP64 reductions + FP64 refinement reach the FP64 residual
    tolerance; the error against the FP64 solution is bounded by the condition
    number (lmax / lmin, lmin = 1) times the two residuals."""
    from paper_1704_00693_amd.apps import MixedHeatSolver
    hp = heat_problem(n, seed=3, ndim=ndim)
    say(f"mixed n={n} ndim={ndim} tol={tol} fused={fused}")
    with tc.Context() as c:
        if fused:  # FP32 corrections through the fused groups (2D: Chebyshev groups)
            c.tc_set_tiling(tc.TC_TILING_FUSED, (0, 0, 0))
        s = MixedHeatSolver(c, hp.density, hp.energy)
        info = s.solve(tol=tol)
        x = s.field("u")
    say(f"  refinements {info['refinements']} inner {info['inner_iterations']} history {info['history']}")
    assert info["history"][-1] <= tol
    res, lmax = true_residual(hp, x)
    say(f"  oracle residual {res:.3e}")
    assert res <= tol * (1 + 1e-6) + 1e-14
    ref = ppcg_solve(hp.density, hp.energy, tol=1e-13, max_iter=3000)
    bound = lmax * (res + 1e-13) * 1.01
    err = float(np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x))
    say(f"  error vs FP64 solve {err:.3e} (bound {bound:.3e})")
    assert err <= bound
    assert info["refinements"] >= 2  # FP32 alone cannot reach the tolerance
