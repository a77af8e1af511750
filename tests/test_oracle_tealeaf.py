"""Pins of the oracle's heat-conduction operator, Chebyshev preconditioner and
PPCG solve: closed-form eigenpairs, the Chebyshev error polynomial, dense
linear algebra on tiny grids, a manufactured solution."""
import math

import numpy as np
import pytest

from oracle.tealeaf import HeatOracle, chebyshev_coefs, ppcg_solve
from synthgen import heat_problem


def cell_centres(n):
    return (np.arange(n) + 0.5) / n


def dense_A(H):
    n, D = H.n, H.ndim
    N = n ** D
    A = np.zeros((N, N))
    h = H.halo
    inner = tuple([slice(h, h + n)] * D)
    for k in range(N):
        H.f["p"][...] = 0.0
        e = np.zeros(N)
        e[k] = 1.0
        H.f["p"][inner] = e.reshape([n] * D)
        A[:, k] = H.apply_A("p").ravel()
    return A


def mode(n, ks, D):
    c = cell_centres(n)
    grids = np.meshgrid(*([c] * D), indexing="ij")  # (z, y, x) order for 3D, (y, x) for 2D
    v = np.ones([n] * D)
    for g, k in zip(grids, ks):
        v = v * np.cos(math.pi * k * g)
    return v


@pytest.mark.parametrize("D,n", [(2, 16), (3, 8)])
def test_constant_density_eigenmodes(D, n):
    rho0 = 0.4
    H = HeatOracle(np.full([n] * D, rho0), np.ones([n] * D))
    H.setup()
    K = H.rx / rho0
    for ks in [(0,) * D, (1,) + (0,) * (D - 1), (3, 5) + (2,) * (D - 2), (n - 1,) * D]:
        v = mode(n, ks, D)
        h = H.halo
        H.f["p"][tuple([slice(h, h + n)] * D)] = v
        Av = H.apply_A("p")
        lam = 1.0 + 4.0 * K * sum(math.sin(math.pi * k / (2 * n)) ** 2 for k in ks)
        assert np.abs(Av - lam * v).max() <= 1e-13 * lam * np.abs(v).max()


def test_spectrum_bounds_dense():
    hp = heat_problem(8, seed=0)
    H = HeatOracle(hp.density, hp.energy)
    lmax_bound = H.setup()
    A = dense_A(H)
    assert np.abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[0] - 1.0) <= 1e-12
    assert ev[-1] <= lmax_bound


def cheb_T(m, x):
    if abs(x) <= 1:
        return math.cos(m * math.acos(x))
    return math.cosh(m * math.acosh(x)) * (1 if x > 0 or m % 2 == 0 else -1)


@pytest.mark.parametrize("steps", [1, 4, 10])
def test_chebyshev_polynomial_closed_form(steps):
    n, rho0 = 16, 0.25
    H = HeatOracle(np.full((n, n), rho0), np.ones((n, n)))
    H.setup()
    K = H.rx / rho0
    lmax = 1.0 + 8.0 * K          # the exact spectrum lies in [1, 1 + 8K)
    cheb = chebyshev_coefs(1.0, lmax, steps)
    sigma = cheb.theta / cheb.delta
    for ks in [(0, 0), (2, 1), (7, 9), (15, 15)]:
        v = mode(n, ks, 2)
        lam = 1.0 + 4.0 * K * sum(math.sin(math.pi * k / (2 * n)) ** 2 for k in ks)
        H.f["r"][2:2 + n, 2:2 + n] = v
        H.precondition(cheb, steps)
        z = H.inner("z")
        p = (1.0 - cheb_T(steps, (cheb.theta - lam) / cheb.delta) / cheb_T(steps, sigma)) / lam
        assert np.abs(z - p * v).max() <= 1e-12 * abs(p) * np.abs(v).max() + 1e-15


@pytest.mark.parametrize("D,n", [(2, 8), (2, 12), (3, 5)])
def test_ppcg_matches_dense_solve(D, n):
    hp = heat_problem(n, seed=3, ndim=D)
    res = ppcg_solve(hp.density, hp.energy, tol=1e-14, max_iter=200)
    H = HeatOracle(hp.density, hp.energy)
    H.setup()
    A = dense_A(H)
    b = (hp.density * hp.energy).ravel()
    xs = np.linalg.solve(A, b)
    assert np.abs(res.x.ravel() - xs).max() <= 1e-12 * np.abs(xs).max()
    assert res.true_rel_resid <= 1e-13


def test_manufactured_solution():
    n = 24
    c = cell_centres(n)
    y, x = np.meshgrid(c, c, indexing="ij")
    ustar = np.cos(math.pi * x) * np.cos(math.pi * y) + 2.0
    hp = heat_problem(n, seed=9)
    H = HeatOracle(hp.density, np.ones((n, n)))
    H.setup()
    H.f["p"][2:2 + n, 2:2 + n] = ustar
    b = H.apply_A("p")
    energy = b / hp.density
    res = ppcg_solve(hp.density, energy, tol=1e-13, max_iter=500)
    assert np.abs(res.x - ustar).max() <= 1e-9 * np.abs(ustar).max()


def test_fixed_iteration_history_is_monotone_in_energy_norm():
    """CG minimises the A-norm of the error over growing Krylov spaces, so the
    error's A-norm never increases from one outer iteration to the next."""
    n = 10
    hp = heat_problem(n, seed=4)
    H = HeatOracle(hp.density, hp.energy)
    H.setup()
    A = dense_A(H)
    b = (hp.density * hp.energy).ravel()
    xs = np.linalg.solve(A, b)
    errs = []
    for k in range(1, 8):
        r = ppcg_solve(hp.density, hp.energy, outer=k)
        e = r.x.ravel() - xs
        errs.append(float(e @ A @ e))
    for a, b2 in zip(errs, errs[1:]):
        assert b2 <= a * (1 + 1e-9) + 1e-28
