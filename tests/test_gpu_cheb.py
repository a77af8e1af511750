"""GPU parity of the fused Chebyshev-step groups (runs of the heat-conduction
preconditioner's steps, one launch each) against the untiled execution and
the oracle.

* PPCG solves of ragged sizes (37^2, 130^2: partial 64 x 16 tiles on the
  top and right) with 1, 2, 3, 4, 7, 9 and 12 inner steps, which give groups
  of one to nine steps, with and without the last TEA_P2: every dataset (halos
  included, so the ghost cells of sd the groups store) and every scalar of
  the solve equal the untiled run's bits, and the solution matches the
  oracle's FP64 solve.
* FP32 datasets (the precision the mixed solver's corrections use), and
  1000^2 for two iterations (many tiles), fused against untiled.
* Grids of 4^2, 5^2 and 9^2, smaller than one tile and its border.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("u", "r", "p", "w", "z", "rt", "sd", "kx", "ky")


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


def solve(tc, hp, mode, outer, inner, dtype):
    from paper_1704_00693_amd.apps import HeatSolver
    with tc.Context() as c:
        c.tc_set_tiling(mode, (0, 0, 0))
        s = HeatSolver(c, hp.density, hp.energy, dtype=dtype)
        info = s.solve(outer=outer, inner=inner)
        fields = {k: c.tc_dat_read(s.f[k]) for k in FIELDS}
    return info, fields


@pytest.mark.parametrize("steps", ["", "7", "9"])
@pytest.mark.parametrize("n", [37, 130])
@pytest.mark.parametrize("inner", [1, 2, 3, 4, 7, 9, 12])
def test_chebyshev_groups_match_untiled(tc, n, inner, steps, monkeypatch):
    # groups as the split search picks them (at most five steps), or of
    # seven or nine steps (the kernel's wider borders)
    if steps:
        monkeypatch.setenv("TC_CHEB_STEPS", steps)
    from oracle.tealeaf import ppcg_solve
    from synthgen import heat_problem
    hp = heat_problem(n, seed=11)
    outer = 3
    say(f"chebyshev groups n={n} inner={inner} steps={steps or 'searched'}")
    base, fb = solve(tc, hp, tc.TC_TILING_NONE, outer, inner, tc.TC_F64)
    got, fg = solve(tc, hp, tc.TC_TILING_FUSED, outer, inner, tc.TC_F64)
    for k in FIELDS:
        assert np.array_equal(fg[k], fb[k]), k
    assert got["rr"] == base["rr"] and got["rz"] == base["rz"] and got["pw"] == base["pw"]
    ref = ppcg_solve(hp.density, hp.energy, outer=outer, inner=inner)
    h = 2
    x = fg["u"][h:h + n, h:h + n]
    assert float(np.abs(x - ref.x).max() / np.abs(ref.x).max()) <= 1e-12


@pytest.mark.parametrize("n", [4, 5, 9])
@pytest.mark.parametrize("inner", [3, 10])
def test_chebyshev_groups_on_tiny_grids(tc, n, inner):
    """Grids as small as the groups take (n = 4 = twice the ghost depth: a
    cell mirrors ghosts on one side only), far smaller than a tile and its
    border: the same bits as untiled, and the oracle's solution."""
    from oracle.tealeaf import ppcg_solve
    from synthgen import heat_problem
    hp = heat_problem(n, seed=13)
    outer = 3
    say(f"chebyshev groups tiny n={n} inner={inner}")
    base, fb = solve(tc, hp, tc.TC_TILING_NONE, outer, inner, tc.TC_F64)
    got, fg = solve(tc, hp, tc.TC_TILING_FUSED, outer, inner, tc.TC_F64)
    for k in FIELDS:
        assert np.array_equal(fg[k], fb[k]), k
    assert got["rr"] == base["rr"] and got["rz"] == base["rz"]
    ref = ppcg_solve(hp.density, hp.energy, outer=outer, inner=inner)
    x = fg["u"][2:2 + n, 2:2 + n]
    assert float(np.abs(x - ref.x).max() / np.abs(ref.x).max()) <= 1e-12


def test_chebyshev_groups_in_the_plan(tc):
    from paper_1704_00693_amd.apps import HeatSolver, chebyshev_coefs
    from synthgen import heat_problem
    hp = heat_problem(130, seed=2)
    with tc.Context() as c:
        c.tc_set_tiling(tc.TC_TILING_FUSED, (0, 0, 0))
        s = HeatSolver(c, hp.density, hp.energy)
        s.setup()
        theta, delta, al, be = chebyshev_coefs(1.0, 50.0, 10)
        s.loop("TEA_PRECON_INIT", [s.F("r", "R"), s.F("rt", "W"), s.F("sd", "W"), s.F("z", "W")], [theta])
        s.precondition(theta, al, be, 10)
        groups, per = c.tc_fused_plan()
        assert groups and all(per[l][0] == 4 for g0, g1 in groups for l in range(g0, g1))
        c.tc_flush()
        assert c.tc_get_stats()["last_groups"] == len(groups)


@pytest.mark.parametrize("n,outer,inner", [(61, 3, 10), (1000, 2, 10)])
def test_chebyshev_groups_fp32_and_large(tc, n, outer, inner):
    from synthgen import heat_problem
    hp = heat_problem(n, seed=4)
    for dtype in ((tc.TC_F32, tc.TC_F64) if n < 100 else (tc.TC_F64,)):
        say(f"chebyshev groups n={n} dtype={dtype}")
        base, fb = solve(tc, hp, tc.TC_TILING_NONE, outer, inner, dtype)
        got, fg = solve(tc, hp, tc.TC_TILING_FUSED, outer, inner, dtype)
        for k in FIELDS:
            assert np.array_equal(fg[k], fb[k]), (dtype, k)
        assert got["rr"] == base["rr"]
