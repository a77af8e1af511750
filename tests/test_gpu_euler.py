"""GPU parity of the compressible-Euler RK3 chain (EULER_PRIM, EULER_RHS,
RK_STAGE loops through the chain API, untiled, skewed-tiled and fused: in 3D
each stage's five right-hand sides and five updates run as one z-marching
kernel) with the
oracle's step: small grids element by element (1e-12 relative; the same fma
sequences make it bit-exact in practice) and the 256^3 Taylor-Green workload
on two z-slabs against the window oracle, with the energy sum checked against
the exactly rounded sum of the read-back field."""
import math
import os
import sys

import numpy as np
import pytest

from oracle.euler import EulerOracle
from synthgen import taylor_green
from windows import euler_window

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


def rel(a, b):
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / (s if s > 0 else 1.0))


def state_2d(n, h):
    c = (np.arange(-2, n + 2, dtype=np.float64) + 0.5) * h
    y, x = np.meshgrid(c, c, indexing="ij")
    rho = 1.0 + 0.1 * np.sin(x) * np.cos(2 * y)
    u = 0.3 * np.cos(y)
    v = -0.2 * np.sin(x)
    p = 2.0 + 0.05 * np.cos(x + y)
    E = p / 0.4 + 0.5 * rho * (u * u + v * v)
    return [np.ascontiguousarray(a) for a in (rho, rho * u, rho * v, E)]


@pytest.mark.parametrize("ndim,n", [(3, 20), (3, 67), (2, 37)])
def test_rk3_step_small(tc, ndim, n):
    from paper_1704_00693_amd.apps import EulerRunner
    h = 2 * math.pi / n
    q = taylor_green(n) if ndim == 3 else state_2d(n, h)
    ref = EulerOracle(q, n, h)
    ref.step(1e-3)
    outs = {}
    runs = [(0, tc.TC_TILING_NONE, (0, 0, 0), {}),
            (1, tc.TC_TILING_SKEWED, (0, 0, 5) if ndim == 3 else (0, 7, 0), {}),
            (2, tc.TC_TILING_FUSED, (0, 0, 0), {})]
    if ndim == 3:
        # the fused stage kernel's other workgroup shapes (rows of
        # wavefronts, planes per workgroup; ragged in y and z here)
        runs += [(3, tc.TC_TILING_FUSED, (0, 0, 0), {"TC_MARCH3_ROWS": "8"}),
                 (4, tc.TC_TILING_FUSED, (0, 0, 0), {"TC_MARCH3_ROWS": "8", "TC_MARCH3_TZ": "12"}),
                 (5, tc.TC_TILING_FUSED, (0, 0, 0), {"TC_MARCH3_ROWS": "4", "TC_MARCH3_TZ": "8"})]
    for key, mode, tile, env in runs:
        say(f"euler ndim={ndim} n={n} mode={mode} {env}")
        os.environ.update(env)
        try:
            with tc.Context() as c:
                c.tc_set_tiling(mode, tile)
                r = EulerRunner(c, q, n, h)
                esum = r.step(1e-3)
                got = [c.tc_dat_read(d) for d in r.Q + r.R + r.vel + [r.p]]
                groups = c.tc_get_stats()["last_groups"]
        finally:
            for k in env:
                del os.environ[k]
        want = ref.q + ref.r + ref.vel + [ref.p]
        hh = 2
        for g, w in zip(got, want):
            sl = tuple([slice(hh, hh + n)] * ndim)
            assert rel(g[sl], w[sl]) <= TOL
        e = ref.interior(ref.q[ndim + 1])
        assert abs(esum - math.fsum(e.ravel().tolist())) <= 1e-15 * float(np.abs(e).sum())
        outs[key] = got
        if mode == tc.TC_TILING_FUSED and ndim == 3:
            # the three stages ran as fused Runge-Kutta stage kernels
            assert groups == 3
    for m in outs:
        for a, b in zip(outs[0], outs[m]):
            assert np.array_equal(a, b)


def test_rhs_march_kernel_equals_per_point_kernel(tc, monkeypatch):
    """The z-marching 3D right-hand-side kernel and the per-point loop kernel
    (selected with TC_WSUM_MARCH=0 at context creation) give the same bits on
    a ragged grid: two x blocks, a partial row block and three z blocks."""
    from paper_1704_00693_amd.apps import EulerRunner
    n = 67
    h = 2 * math.pi / n
    q = taylor_green(n)
    outs = []
    for march in ("1", "0"):
        monkeypatch.setenv("TC_WSUM_MARCH", march)
        say(f"euler rhs n={n} march={march}")
        with tc.Context() as c:
            r = EulerRunner(c, q, n, h)
            r.step(1e-3)
            outs.append([c.tc_dat_read(d) for d in r.Q + r.R])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_rk3_taylor_green_256_sampled(tc):
    from paper_1704_00693_amd.apps import EulerRunner
    n = 256
    h = 2 * math.pi / n
    say("taylor-green 256^3 inputs")
    q = taylor_green(n)
    slabs = [(0, 3), (126, 130), (253, 256)]
    refs = [euler_window(q, n, h, a, b, 1e-3) for a, b in slabs]
    res = {}
    for mode, tile in [(tc.TC_TILING_NONE, (0, 0, 0)), (tc.TC_TILING_SKEWED, (0, 0, 0)),
                       (tc.TC_TILING_FUSED, (0, 0, 0))]:
        say(f"taylor-green 256^3 mode={mode}")
        with tc.Context() as c:
            c.tc_set_tiling(mode, tile)
            r = EulerRunner(c, q, n, h)
            esum = r.step(1e-3)
            qs = [c.tc_dat_read(d) for d in r.Q]
            rs = [c.tc_dat_read(d) for d in r.R]
        hh = 2
        for (a, b), (wq, wr) in zip(slabs, refs):
            for comp in range(5):
                g = qs[comp][a + hh:b + hh, hh:hh + n, hh:hh + n]
                assert rel(g, wq[comp][:, hh:hh + n, hh:hh + n]) <= TOL
                g = rs[comp][a + hh:b + hh, hh:hh + n, hh:hh + n]
                assert rel(g, wr[comp][:, hh:hh + n, hh:hh + n]) <= TOL
        e = qs[4][hh:hh + n, hh:hh + n, hh:hh + n]
        exact = math.fsum(e.ravel().tolist())
        say(f"  energy sum {esum!r} exact {exact!r}")
        assert abs(esum - exact) <= 1e-15 * float(np.abs(e).sum())
        res[mode] = (esum, [a[::5, ::3, ::7].copy() for a in qs])
    for m in (1, 2):
        assert res[0][0] == res[m][0]
        for a, b in zip(res[0][1], res[m][1]):
            assert np.array_equal(a, b)


def test_rk3_two_steps_fused(tc):
    """Two steps in one chain (the first step's last-stage R is overwritten
    by the second step before any read, so the fused stage skips writing it):
    the fused mode gives the untiled bits for Q, R and the primitives."""
    from paper_1704_00693_amd.apps import EulerRunner
    n = 37
    h = 2 * math.pi / n
    q = taylor_green(n)
    outs = []
    for mode in (tc.TC_TILING_NONE, tc.TC_TILING_FUSED):
        say(f"euler two steps n={n} mode={mode}")
        with tc.Context() as c:
            c.tc_set_tiling(mode, (0, 0, 0))
            r = EulerRunner(c, q, n, h)
            r.record_step(1e-3)
            r.step(1e-3)
            if mode == tc.TC_TILING_FUSED:
                assert c.tc_get_stats()["last_groups"] >= 6
            outs.append([c.tc_dat_read(d) for d in r.Q + r.R + r.vel + [r.p]])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
