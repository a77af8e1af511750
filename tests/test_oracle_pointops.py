"""Pins of the oracle's single-point update loops (AXPBY and the CG / Chebyshev
updates of the heat solve) and of the face coefficients of the heat operator
on a layered medium.

* The update loops are pinned element by element against their definitions
  evaluated in exact rational arithmetic and rounded once per operation
  (Python's ``fractions``), and against plain numpy within an fma-rounding
  bound.  The two scalars and the two fields differ, so a swapped operand
  or scalar changes the result; points outside the loop range must keep
  their values.
* The face coefficients are pinned by a physical property that fixes the
  harmonic mean: in a medium whose density varies along one axis only, the
  steady 1D profile whose increments are the series resistances of the two
  half-cells on either side of a face, (rho_left + rho_right) / 2 per face,
  carries the same flux through every face.  Then A u = u on every cell
  whose faces are both interior.  Any other mean of the conductivity 1/rho
  (the arithmetic mean, say) breaks the flux balance at the layer
  interfaces.
"""
import ctypes
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.tealeaf import HeatOracle


def _r(v):
    """Round an exact rational to the nearest double."""
    return float(Fraction(v))


def _exact_fma(a, b, c):
    return _r(Fraction(a) * Fraction(b) + Fraction(c))


def _fields(seed, n=9, h=2):
    rng = np.random.default_rng(seed)
    shape = (n + 2 * h, n + 2 * h)
    return [rng.uniform(-2.0, 2.0, shape) for _ in range(4)], oracle.Grid(2, n, h)


LO, HI = [1, 2], [8, 7]  # a range strictly inside the interior: the rest must stay unchanged


def _inside(h):
    ys = range(LO[1] + h, HI[1] + h)
    xs = range(LO[0] + h, HI[0] + h)
    mask = np.zeros((9 + 2 * h, 9 + 2 * h), dtype=bool)
    mask[LO[1] + h:HI[1] + h, LO[0] + h:HI[0] + h] = True
    return ys, xs, mask


def test_axpby_matches_its_definition():
    """y = fma(a, x, b*y) over the range, with a != b and x != y."""
    (y0, x0, _, _), grid = _fields(1)
    a, b = 0.7310585786300049, -1.3862943611198906
    y = y0.copy()
    l, h = grid.box(LO, HI)
    oracle.lib().orc_axpby(l, h, grid.view(y), grid.view(x0), ctypes.c_double(a), ctypes.c_double(b))
    ys, xs, mask = _inside(2)
    for j in ys:
        for i in xs:
            assert y[j, i] == _exact_fma(a, x0[j, i], b * y0[j, i])
    assert np.array_equal(y[~mask], y0[~mask])
    # independent numpy form: within one rounding of each of the two terms
    ref = a * x0 + b * y0
    bound = 2 * np.finfo(float).eps * (np.abs(a * x0) + np.abs(b * y0))
    assert np.all(np.abs(y - ref)[mask] <= bound[mask])
    # the swapped forms are far away: the test tells them apart
    for wrong in (b * x0 + a * y0, a * y0 + b * x0):
        assert np.abs(y - wrong)[mask].max() > 1e-3


def test_cg_update_and_cg_p_match_their_definitions():
    """x = fma(alpha, p, x); r = fma(-alpha, w, r); then p = fma(beta, p, z)."""
    (x0, r0, p0, w0), grid = _fields(2)
    alpha, beta = 0.4142135623730951, 1.7320508075688772
    x, r, p = x0.copy(), r0.copy(), p0.copy()
    L = oracle.lib()
    l, h = grid.box(LO, HI)
    L.orc_tea_cg_update(l, h, grid.view(x), grid.view(r), grid.view(p), grid.view(w0), ctypes.c_double(alpha))
    z = w0 * 0.5 + 0.25
    L.orc_tea_cg_p(l, h, grid.view(p), grid.view(z), ctypes.c_double(beta))
    ys, xs, mask = _inside(2)
    for j in ys:
        for i in xs:
            assert x[j, i] == _exact_fma(alpha, p0[j, i], x0[j, i])
            assert r[j, i] == _exact_fma(-alpha, w0[j, i], r0[j, i])
            assert p[j, i] == _exact_fma(beta, p0[j, i], z[j, i])
    for got, old in ((x, x0), (r, r0), (p, p0)):
        assert np.array_equal(got[~mask], old[~mask])


def test_precon_init_and_p2_match_their_definitions():
    """rt = r, sd = r / theta, z = 0; then sd = fma(alpha, sd, beta*rt)."""
    (r0, rt0, sd0, z0), grid = _fields(3)
    theta, alpha, beta = 3.25, 0.6180339887498949, -0.2360679774997897
    rt, sd, z = rt0.copy(), sd0.copy(), z0.copy()
    L = oracle.lib()
    l, h = grid.box(LO, HI)
    L.orc_tea_precon_init(l, h, grid.view(r0), grid.view(rt), grid.view(sd), grid.view(z), ctypes.c_double(theta))
    ys, xs, mask = _inside(2)
    for j in ys:
        for i in xs:
            assert rt[j, i] == r0[j, i]
            assert sd[j, i] == _r(Fraction(r0[j, i]) / Fraction(theta))
            assert z[j, i] == 0.0
    sd1 = sd.copy()
    rt[mask] = rt[mask] * 1.5 - 0.125  # make rt differ from sd * theta
    L.orc_tea_p2(l, h, grid.view(sd), grid.view(rt), ctypes.c_double(alpha), ctypes.c_double(beta))
    for j in ys:
        for i in xs:
            assert sd[j, i] == _exact_fma(alpha, sd1[j, i], beta * rt[j, i])
    for got, old in ((sd, sd0), (z, z0)):
        assert np.array_equal(got[~mask], old[~mask])


def _layered(n, axis, D, cuts, values):
    """Density constant across the other axes, piecewise constant along
    ``axis`` (layer k from cuts[k] to cuts[k + 1])."""
    prof = np.empty(n)
    for k, v in enumerate(values):
        prof[cuts[k]:cuts[k + 1]] = v
    shape = [1] * D
    shape[D - 1 - axis] = n  # arrays are (z, y, x): axis 0 (x) is the last index
    return np.broadcast_to(prof.reshape(shape), [n] * D).copy(), prof


@pytest.mark.parametrize("D,n,axis", [(2, 16, 0), (2, 16, 1), (3, 10, 0), (3, 10, 2)])
def test_face_coefficients_balance_flux_in_a_layered_medium(D, n, axis):
    cuts = [0, n // 4, n // 2 + 1, n]
    rho, prof = _layered(n, axis, D, cuts, [0.2, 0.9, 0.45])
    H = HeatOracle(rho, np.ones([n] * D))
    H.setup()
    # cell-centre profile: each face adds the resistance of its two half-cells
    c = 0.01
    u = np.empty(n)
    u[0] = 0.3
    for i in range(1, n):
        u[i] = u[i - 1] + c * (prof[i - 1] + prof[i]) / 2.0
    shape = [1] * D
    shape[D - 1 - axis] = n
    field = np.broadcast_to(u.reshape(shape), [n] * D).copy()
    h = H.halo
    H.f["p"][tuple([slice(h, h + n)] * D)] = field
    Au = H.apply_A("p")
    # cells 1 .. n-2 along the axis: both faces interior, flux in = flux out
    sel = [slice(None)] * D
    sel[D - 1 - axis] = slice(1, n - 1)
    err = np.abs(Au - field)[tuple(sel)].max()
    scale = np.abs(Au).max()
    assert err <= 1e-13 * scale, err
    # the face next to a wall carries no flux (reflective ghosts), so the
    # profile is not a fixed point there: the check is not vacuous
    sel[D - 1 - axis] = 0
    assert np.abs(Au - field)[tuple(sel)].min() > 1e-3


def test_arithmetic_mean_would_break_the_balance():
    """The same profile under the arithmetic mean of 1/rho: the residual at
    a layer interface is of the order of the flux itself.  (Computed here from
    the definition; it shows that the previous test separates the two means.)"""
    n, rx = 16, 0.004 * 16 * 16
    prof = np.array([0.2] * 4 + [0.9] * 5 + [0.45] * 7)
    u = np.empty(n)
    u[0] = 0.3
    for i in range(1, n):
        u[i] = u[i - 1] + 0.01 * (prof[i - 1] + prof[i]) / 2.0
    flux_h = [rx * 2.0 / (prof[i - 1] + prof[i]) * (u[i] - u[i - 1]) for i in range(1, n)]
    flux_a = [rx * (1 / prof[i - 1] + 1 / prof[i]) / 2.0 * (u[i] - u[i - 1]) for i in range(1, n)]
    assert max(flux_h) - min(flux_h) < 1e-14
    assert max(flux_a) - min(flux_a) > 1e-3


@pytest.mark.parametrize("D,n", [(2, 12), (3, 6)])
def test_gershgorin_bound_closed_form_at_constant_density(D, n):
    """At constant density every face coefficient is rx / rho (reflective
    ghosts included), so the row bound max(1 + 2 * sum of the cell's 2 D face
    coefficients) is 1 + 4 D rx / rho; the dense spectrum's largest
    eigenvalue lies below it."""
    rho0 = 0.35
    H = HeatOracle(np.full([n] * D, rho0), np.ones([n] * D))
    got = H.setup()
    want = 1.0 + 4.0 * D * H.rx / rho0
    assert abs(got - want) <= 8 * np.finfo(float).eps * want
    # one denser cell raises the bound at its neighbours: the maximum is taken
    rho = np.full([n] * D, rho0)
    rho[(1,) * D] = 0.1
    H2 = HeatOracle(rho, np.ones([n] * D))
    assert H2.setup() > got * (1 + 1e-6)
