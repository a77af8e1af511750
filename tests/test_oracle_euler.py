"""Pins of the Euler / SSP-RK3 oracle against closed forms: a uniform state is
a fixed point (differences first); single-mode pressure and density waves
give -dF/dx to fourth order along each axis; the Runge-Kutta stages reproduce
the third-order Taylor polynomial of exp(lambda dt) for a linear right-hand
side."""
import math

import numpy as np
import pytest

from oracle.euler import EulerOracle

GAMMA = 1.4


def coords(n, h, halo=2):
    c = (np.arange(-halo, n + halo, dtype=np.float64) + 0.5) * h
    return np.meshgrid(c, c, c, indexing="ij")  # z, y, x


def state(rho, vel, p):
    e = p / (GAMMA - 1.0) + 0.5 * rho * sum(v * v for v in vel)
    return [rho] + [rho * v for v in vel] + [e]


@pytest.mark.parametrize("ndim", [2, 3])
def test_uniform_state_is_fixed(ndim):
    n, halo = 12, 2
    shape = [n + 2 * halo] * ndim
    vel = [np.full(shape, 0.3), np.full(shape, -0.2), np.full(shape, 0.1)][:ndim]
    q = state(np.full(shape, 1.2), vel, np.full(shape, 2.5))
    o = EulerOracle(q, n, 2 * math.pi / n)
    o.prim()
    o.rhs()
    for r in o.r:
        assert np.all(o.interior(r) == 0.0)
    before = [a.copy() for a in o.q]
    o.step(1e-3)
    # the stage weights 1/3 and 2/3 are not exact in binary: a few ulps
    for a, b in zip(before, o.q):
        assert np.all(np.abs(b - a) <= 4 * np.finfo(float).eps * np.abs(a))


def _max_err(n, axis, kind):
    """Max error of the oracle's right-hand side against the analytic
    -dF/dx_axis for a single-mode wave along `axis`."""
    h = 2 * math.pi / n
    z, y, x = coords(n, h)
    s = [x, y, z][axis]
    eps, U, p0 = 1e-3, 0.4, 3.0
    ones = np.ones_like(x)
    vel = [np.zeros_like(x) for _ in range(3)]
    if kind == "pressure":  # rho = 1, u = 0, p = p0 + eps sin(s): R_{axis+1} = -eps cos(s)
        q = state(ones, vel, p0 + eps * np.sin(s))
        comp, exact = axis + 1, -eps * np.cos(s)
    elif kind == "density":  # u_axis = U, p const, rho = 1 + eps sin(s): R_0 = -U eps cos(s)
        vel[axis] = U * ones
        q = state(1.0 + eps * np.sin(s), vel, p0 * ones)
        comp, exact = 0, -U * eps * np.cos(s)
    else:  # energy: u_axis = U, rho = 1, p = p0 + eps sin(s): R_4 = -U gamma/(gamma-1) eps cos(s)
        vel[axis] = U * ones
        q = state(ones, vel, p0 + eps * np.sin(s))
        comp, exact = 4, -U * GAMMA / (GAMMA - 1.0) * eps * np.cos(s)
    o = EulerOracle(q, n, h)
    o.prim()
    o.rhs()
    return float(np.abs(o.interior(o.r[comp]) - o.interior(exact)).max())


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("kind", ["pressure", "density", "energy"])
def test_fourth_order_derivatives(axis, kind):
    e1 = _max_err(16, axis, kind)
    e2 = _max_err(32, axis, kind)
    order = math.log2(e1 / e2)
    assert 3.7 < order < 4.3, (e1, e2, order)
    assert e2 < 1e-7


def test_rk3_linear_rhs_is_third_order_taylor():
    n, halo, lam, dt = 6, 2, -0.7, 0.05
    shape = [n + 2 * halo] * 3
    rng = np.random.default_rng(3)
    q = [rng.uniform(0.5, 1.5, shape) for _ in range(5)]
    o = EulerOracle(q, n, 1.0)
    start = [o.interior(a).copy() for a in o.q]

    def linear(orc):
        for c in range(5):
            orc.r[c][...] = lam * orc.q[c]

    o.step(dt, rhs=linear)
    zz = lam * dt
    amp = 1 + zz + zz * zz / 2 + zz ** 3 / 6
    for a, b in zip(start, o.q):
        got = o.interior(b)
        assert np.allclose(got, a * amp, rtol=1e-14, atol=0)


@pytest.mark.parametrize("zlo,zhi", [(0, 3), (10, 14), (21, 24)])
def test_euler_window_equals_full_step(zlo, zhi):
    """The z-slab window oracle used for full-size checks gives exactly the
    full oracle's values on its planes."""
    import sys
    sys.path.insert(0, "tests")
    from synthgen import taylor_green
    from windows import euler_window
    n = 24
    h = 2 * math.pi / n
    q = taylor_green(n)
    full = EulerOracle(q, n, h)
    full.step(1e-3)
    wq, wr = euler_window(q, n, h, zlo, zhi, 1e-3)
    hh = 2
    for c in range(5):
        a = full.q[c][zlo + hh:zhi + hh, hh:hh + n, hh:hh + n]
        b = wq[c][:, hh:hh + n, hh:hh + n]
        assert np.array_equal(a, b)
        assert np.array_equal(full.r[c][zlo + hh:zhi + hh, hh:hh + n, hh:hh + n], wr[c][:, hh:hh + n, hh:hh + n])
