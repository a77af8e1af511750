"""GPU tests of the batched and served heat-conduction solves (tc_batch_*).

Every instance is checked against the oracle's FP64 PPCG solve of the same
problem (inputs drawn from the same SplitMix64 stream on the host):
FP64 batches must take the same number of iterations and agree to 1e-12
relative; mixed-precision batches must reach the FP64 true residual and stay
within cond(A) * residual of the FP64 solution.  A solve must give the same
bits alone and inside a mix of other solves admitted at other times."""
import math
import sys

import numpy as np
import pytest

from oracle.tealeaf import HeatOracle, ppcg_solve
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


def true_residual(hp, x):
    o = HeatOracle(hp.density, hp.energy)
    lmax = o.setup()
    h, n = o.halo, o.n
    o.f["u"][tuple([slice(h, h + n)] * o.ndim)] = x
    b = o.inner("u0")
    return float(np.linalg.norm(b - o.apply_A("u")) / np.linalg.norm(b)), lmax


CASES = [(2, 20, 11), (2, 33, 12), (2, 70, 13), (2, 129, 14), (3, 12, 15), (3, 17, 16)]


def test_batch_fp64_matches_oracle(tc):
    tol = 1e-10
    with tc.Context() as c, tc.Batch(c, mixed=False, max_instances=8) as b:
        tickets = [b.tc_batch_submit(nd, n, seed, tol=tol, keep_x=True) for nd, n, seed in CASES]
        say(f"fp64 batch of {len(CASES)} solves")
        b.tc_batch_wait()
        for (nd, n, seed), t in zip(CASES, tickets):
            r = b.tc_batch_poll(t)
            x = b.tc_batch_read_x(t)
            hp = heat_problem(n, seed=seed, ndim=nd)
            ref = ppcg_solve(hp.density, hp.energy, tol=tol, max_iter=5000)
            err = float(np.abs(x - ref.x).max() / np.abs(ref.x).max())
            say(f"  ndim={nd} n={n}: iterations {r['iterations']} (oracle {ref.iterations}), error {err:.2e}, "
                f"true residual {r['rel_residual']:.2e}")
            assert r["state"] == tc.TC_SOLVE_DONE
            assert r["iterations"] == ref.iterations
            assert abs(r["lmax"] - ref.lmax) <= 1e-15 * ref.lmax
            assert err <= TOL
            res, _ = true_residual(hp, x)
            assert abs(res - r["rel_residual"]) <= 1e-6 * res + 1e-15


def test_batch_fp64_equals_per_loop_solver(tc):
    """The batched solve and the per-loop solver (TEA_* loops through the
    chain API) compute the same arithmetic; for n > 16 their reductions use
    the same tile order, so the solutions are bit-identical."""
    from paper_1704_00693_amd.apps import HeatSolver
    nd, n, seed = 2, 96, 21
    hp = heat_problem(n, seed=seed, ndim=nd)
    with tc.Context() as c:
        s = HeatSolver(c, hp.density, hp.energy)
        info = s.solve(outer=0, inner=10, tol=1e-9)
        x_loop = s.field("u")
    with tc.Context() as c, tc.Batch(c) as b:
        t = b.tc_batch_submit(nd, n, seed, tol=1e-9, keep_x=True)
        b.tc_batch_wait()
        r = b.tc_batch_poll(t)
        x = b.tc_batch_read_x(t)
    assert r["iterations"] == info["iterations"]
    assert np.array_equal(x, x_loop)


@pytest.mark.parametrize("tol", [1e-8, 1e-10])
def test_batch_mixed_reaches_fp64_residual(tc, tol):
    with tc.Context() as c, tc.Batch(c, mixed=True, max_instances=8) as b:
        tickets = [b.tc_batch_submit(nd, n, seed, tol=tol, keep_x=True) for nd, n, seed in CASES]
        b.tc_batch_wait()
        for (nd, n, seed), t in zip(CASES, tickets):
            r = b.tc_batch_poll(t)
            x = b.tc_batch_read_x(t)
            hp = heat_problem(n, seed=seed, ndim=nd)
            res, lmax = true_residual(hp, x)
            ref = ppcg_solve(hp.density, hp.energy, tol=1e-13, max_iter=5000)
            err = float(np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x))
            say(f"  mixed ndim={nd} n={n}: corrections {r['outer']} iterations {r['iterations']} "
                f"residual {res:.2e} error {err:.2e}")
            assert r["state"] == tc.TC_SOLVE_DONE and r["converged"] == 1
            assert res <= tol * (1 + 1e-6)
            assert abs(res - r["rel_residual"]) <= 1e-6 * res + 1e-15
            assert err <= lmax * (res + 1e-13) * 1.01


@pytest.mark.parametrize("mixed", [False, True])
def test_same_result_alone_and_in_a_mix(tc, mixed):
    """Continuous batching: a solve admitted alone and the same solve admitted
    while others are running (and others arriving after it) give the same
    bits."""
    probe = (2, 77, 31)
    with tc.Context() as c, tc.Batch(c, mixed=mixed, max_instances=4, replays_per_step=2) as b:
        t = b.tc_batch_submit(*probe, tol=1e-9, keep_x=True)
        b.tc_batch_wait()
        alone = b.tc_batch_read_x(t)
        r_alone = b.tc_batch_poll(t)
    with tc.Context() as c, tc.Batch(c, mixed=mixed, max_instances=4, replays_per_step=2) as b:
        others = [b.tc_batch_submit(2, 150, 41, tol=1e-9), b.tc_batch_submit(3, 20, 42, tol=1e-9)]
        b.tc_batch_step()
        b.tc_batch_step()
        t = b.tc_batch_submit(*probe, tol=1e-9, keep_x=True)
        b.tc_batch_step()
        late = [b.tc_batch_submit(2, 40, 43, tol=1e-9), b.tc_batch_submit(2, 64, 44, tol=1e-9),
                b.tc_batch_submit(3, 9, 45, tol=1e-9)]
        b.tc_batch_wait()
        mixed_x = b.tc_batch_read_x(t)
        r_mix = b.tc_batch_poll(t)
        for o in others + late:
            assert b.tc_batch_poll(o)["state"] == tc.TC_SOLVE_DONE
    assert r_mix["iterations"] == r_alone["iterations"]
    assert np.array_equal(alone, mixed_x)


def test_admission_by_footprint_and_rejection(tc):
    """With an HBM budget that holds two 64^2 solves at once, eight of them
    still all finish (admitted as earlier ones retire); a solve larger than
    the budget is rejected."""
    with tc.Context() as c:
        per = 12 * ((66 * 66 * 8 + 255) // 256 * 256)  # FP64 fields of one 64^2 solve
        with tc.Batch(c, max_instances=8, hbm_budget=2 * per + 100) as b:
            ts = [b.tc_batch_submit(2, 64, 100 + i, tol=1e-8) for i in range(8)]
            big = b.tc_batch_submit(2, 512, 7, tol=1e-8)
            peak = 0
            left = 1
            while left:
                left = b.tc_batch_step()
                running = sum(b.tc_batch_poll(t)["state"] == tc.TC_SOLVE_RUNNING for t in ts)
                peak = max(peak, running)
            b.tc_batch_step()
            assert peak <= 2
            for t in ts:
                r = b.tc_batch_poll(t)
                assert r["state"] == tc.TC_SOLVE_DONE and r["converged"] == 1
            assert b.tc_batch_poll(big)["state"] == tc.TC_SOLVE_REJECTED


def test_serving_trace_small(tc):
    """A short Poisson trace (mixed 2D/3D sizes) served in real time: every
    request completes, latencies are measured from arrival, and sampled
    requests give the same bits as the same solve run alone."""
    from paper_1704_00693_amd.apps import serve
    from synthgen import Request, SplitMix64
    rng = SplitMix64(77)
    reqs, t = [], 0.0
    for i in range(24):
        t += -math.log(1.0 - rng.unit()) / 40.0
        nd = 2 if rng.randint(2) == 0 else 3
        n = int(round(math.exp(rng.uniform(math.log(16), math.log(96 if nd == 2 else 24)))))
        reqs.append(Request(t, nd, n, rng.next()))
    sample = [0, 5, 11, 23]
    for mixed in (False, True):
        with tc.Context() as c:
            out = serve(c, reqs, mixed=mixed, tol=1e-9, max_instances=8, keep_x=sample)
        lat = [v for v in out["latency"] if v is not None]
        say(f"served mixed={mixed}: {len(lat)}/{len(reqs)} in {out['wall_s']:.2f} s, "
            f"p50 {np.percentile(lat, 50) * 1e3:.1f} ms p99 {np.percentile(lat, 99) * 1e3:.1f} ms")
        assert len(lat) == len(reqs) and min(lat) > 0
        for i in sample:
            q = reqs[i]
            with tc.Context() as c, tc.Batch(c, mixed=mixed) as b:
                tk = b.tc_batch_submit(q.ndim, q.n, q.seed, tol=1e-9, keep_x=True)
                b.tc_batch_wait()
                alone = b.tc_batch_read_x(tk)
            assert np.array_equal(alone, out["x"][i])


@pytest.mark.parametrize("mixed", [False, True])
def test_fused_chebyshev_shapes_bit_identical(tc, monkeypatch, mixed):
    """The 2D Chebyshev steps run several at a time on tiles with a
    recomputed border (TC_BATCH_FUSED=steps,tile height; 0: one launch per
    step): every shape gives the bits of the per-step kernels."""
    cases = [(2, 20, 51), (2, 70, 52), (2, 129, 53), (3, 12, 54)]
    results = {}
    for shape in ("0", "3,16", "3,32", "5,16", "5,32", "9,16"):
        monkeypatch.setenv("TC_BATCH_FUSED", shape)
        say(f"batch mixed={mixed} fused={shape}")
        with tc.Context() as c, tc.Batch(c, mixed=mixed, max_instances=4) as b:
            ts = [b.tc_batch_submit(nd, n, seed, tol=1e-9, keep_x=True) for nd, n, seed in cases]
            b.tc_batch_wait()
            results[shape] = [(b.tc_batch_poll(t)["iterations"], b.tc_batch_read_x(t)) for t in ts]
    base = results["0"]
    for shape, res in results.items():
        for (it0, x0), (it, x) in zip(base, res):
            assert it == it0, shape
            assert np.array_equal(x, x0), shape


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("cheb_steps", [10, 5, 2])
def test_fused_chebyshev_3d_bit_identical(tc, monkeypatch, mixed, cheb_steps):
    """The 3D Chebyshev steps run three (or one) at a time, marching up
    z-segments of 32 planes on 64 x 8 tiles with a recomputed border: 12^3
    (one tile, one segment), 40^3 (two segments, the second partial) and
    70^3 (two x tiles and three segments, all partial), next to a 2D solve.
    Every solve takes the iterations and gives the bits of the per-step
    kernels (TC_BATCH_FUSED=0), also with only the 2D steps fused
    (TC_BATCH_FUSED3=0).  10 steps per preconditioner give launches of
    3 + 3 + 3 steps, 5 give 3 + 1 and 2 give 1."""
    cases = [(3, 12, 71), (3, 40, 72), (2, 50, 73), (3, 70, 74)]
    results = {}
    for name, env in (("per step", {"TC_BATCH_FUSED": "0"}), ("2D fused", {"TC_BATCH_FUSED3": "0"}),
                      ("2D and 3D fused", {})):
        for k in ("TC_BATCH_FUSED", "TC_BATCH_FUSED3"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        say(f"batch 3D mixed={mixed} cheb_steps={cheb_steps} {name}")
        with tc.Context() as c, tc.Batch(c, mixed=mixed, max_instances=4, cheb_steps=cheb_steps) as b:
            ts = [b.tc_batch_submit(nd, n, seed, tol=1e-9, keep_x=True) for nd, n, seed in cases]
            b.tc_batch_wait()
            results[name] = [(b.tc_batch_poll(t)["iterations"], b.tc_batch_poll(t)["converged"],
                              b.tc_batch_read_x(t)) for t in ts]
    base = results["per step"]
    for name, res in results.items():
        for (nd, n, _), (it0, cv0, x0), (it, cv, x) in zip(cases, base, res):
            assert cv == cv0 and (mixed or cv0 == 1), (name, nd, n)
            assert it == it0, (name, nd, n)
            assert np.array_equal(x, x0), (name, nd, n)


@pytest.mark.parametrize("mixed", [False, True])
def test_batch_full_size_instances(tc, mixed):
    """Instances at the top of the batched workload's size range (1023^2,
    the largest 2D size drawn) next to smaller 2D and 3D ones: every solve
    converges and its true relative residual, recomputed by the oracle's
    operator from the returned x, is within the tolerance and equal to the
    one the engine reports."""
    tol = 1e-8
    cases = [(2, 1023, 61), (2, 700, 62), (2, 97, 63), (3, 64, 64)]
    with tc.Context() as c, tc.Batch(c, mixed=mixed, max_instances=4) as b:
        ts = [b.tc_batch_submit(nd, n, seed, tol=tol, keep_x=True) for nd, n, seed in cases]
        b.tc_batch_wait()
        for (nd, n, seed), t in zip(cases, ts):
            r = b.tc_batch_poll(t)
            x = b.tc_batch_read_x(t)
            hp = heat_problem(n, seed=seed, ndim=nd)
            res, _ = true_residual(hp, x)
            say(f"  mixed={mixed} ndim={nd} n={n}: iterations {r['iterations']} residual {res:.3e}")
            assert r["state"] == tc.TC_SOLVE_DONE and r["converged"] == 1
            assert res <= tol * (1 + 1e-6)
            assert abs(res - r["rel_residual"]) <= 1e-6 * res + 1e-15
