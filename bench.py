"""Benchmark: run-time tiled execution of a synthetic 2D loop chain on one MI355X.

Workload (one step = one flush of the whole chain over the grid, inputs
resident in HBM): 4096^2 FP64 cells, 12 datasets with halo 2, a chain of 40
weighted-sum loops each reading 2-4 datasets through 5-point or 9-point
stencils (seeded, synthgen.chain_2d).

Every execution mode runs the same chain; the JSON line reports the best
tiled mode as `value` (cell-updates/s) next to the untiled run, the effective
bandwidth under the per-loop byte model, a roofline entry for the dominant
kernel (timed with HIP events inside the run) and the oracle timed on the
host's cores on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--modes none,skewed,fused]

Each mode is warmed for W flushes and at least WARM_SECONDS of wall time
before its K timed flushes (the GPU's clocks ramp up under sustained load).

Measured HBM traffic comes from rocprofv3 counter runs of this script (one
run per counter and mode, ingested with --ingest-counters on the host),
scaled by what the same counters read for a plain copy kernel of known size
(--modes copy).
"""
import argparse
import csv
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tiled vs untiled cell-updates/s & HBM GB/s; batched solves/s + p99 latency"
HBM_PEAK_GBS = 8000.0
MODE_NAMES = {"none": 0, "skewed": 1, "fused": 2}
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1704_00693_amd", "csrc")
    for f in sorted(os.listdir(src)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(open(os.path.join(src, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_entry(mode_name: str):
    """Counter-derived HBM traffic of a mode from the committed summary, or
    None if absent or taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    try:
        t = json.load(open(TRAFFIC_JSON))
    except ValueError:
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    return t.get("modes", {}).get(mode_name)


WARM_SECONDS = 0.5  # the GPU's clocks ramp up under sustained load: warm every mode at least this long


def time_mode(ctx, runner, mode, tile, steps, warmup, cells_per_step, warm_seconds=WARM_SECONDS):
    import torch
    ctx.tc_set_tiling(mode, tile)
    # the first flush builds the plan (and compiles fused kernels); the warm
    # period, in which the clocks ramp up, starts after it
    runner.record()
    ctx.tc_flush()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 1
    while k < warmup or time.perf_counter() - t0 < warm_seconds:
        runner.record()
        ctx.tc_flush()
        k += 1
        if k % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        runner.record()
        ctx.tc_flush()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.tc_get_stats()
    # one more flush with per-launch HIP-event timing (separate from the timed loop)
    ctx.tc_set_profiling(True)
    runner.record()
    ctx.tc_flush()
    prof = ctx.tc_get_stats()
    ctx.tc_set_profiling(False)
    return {
        "ms_per_step": dt / steps * 1e3,
        "cell_updates_per_s": cells_per_step * steps / dt,
        "effective_GBps": st["modelled_bytes"] * steps / dt / 1e9,
        "launches_per_step": st["last_launches"],
        "tiles": st["last_tiles"],
        "groups": st["last_groups"],
        "max_skew": st["max_skew"],
        "plan_seconds": st["plan_seconds"],
        "jit_compile_seconds": st["jit_compile_seconds"],
        "modelled_bytes": st["modelled_bytes"],
        "fused_bytes": st["fused_bytes"],
        "kernel_seconds": prof["prof_kernel_seconds"],
        "kernel_launches": prof["prof_launches"],
        "fused_kernel_seconds": prof["prof_fused_seconds"],
    }


def copy_probe(tc, n: int, steps: int, warmup: int, reference: bool = True):
    """A plain copy of one n^2 FP64 dataset into another (the library's COPY
    loop): the counter calibration kernel and the achievable-bandwidth probe."""
    import torch
    with tc.Context(0) as c:
        blk = c.tc_decl_block(2, "copy")
        a = c.tc_decl_dat(blk, [n, n], [2, 2], [2, 2], None, tc.TC_F64, "a")
        b = c.tc_decl_dat(blk, [n, n], [2, 2], [2, 2], None, tc.TC_F64, "b")
        s0 = c.tc_decl_stencil([(0, 0)])

        def rec():
            c.tc_par_loop("COPY", blk, [0, n, 0, n], [(b, s0, "W"), (a, s0, "R")], [], name="copy")

        for _ in range(warmup):
            rec()
            c.tc_flush()
        torch.cuda.synchronize()
        c.tc_set_profiling(True)
        tot = 0.0
        for _ in range(steps):
            rec()
            c.tc_flush()
            tot += c.tc_get_stats()["prof_kernel_seconds"]
        c.tc_set_profiling(False)
    alg = 2 * n * n * 8
    return {"alg_bytes_per_launch": alg, "launches": steps + warmup, "avg_launch_us": tot / steps * 1e6,
            "GBps": alg * steps / tot / 1e9, "reference_copy_GBps": reference_copy_GBps() if reference else None}


def reference_copy_GBps(nbytes: int = 1 << 31, reps: int = 20) -> float:
    """Device-to-device copy of a 2 GiB buffer by the runtime's own copy
    kernel (torch's ``copy_``), warmed for 0.5 s: the bandwidth a copy reaches
    on this part, as a reference for the library's kernels."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.5:
        b.copy_(a)
        torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


# Algorithmic bytes of one FP64 PPCG iteration per cell, loop by loop (8 B
# per R or W access, 16 B per RW): matvec (p, Kx, Ky read, w written) 32,
# x and r update (x, r RW, p, w read) 48, preconditioner set-up (r read; rt,
# sd, z written) 32, ten Chebyshev steps (P1: Kx, Ky, sd read, rt, z RW, 56
# B; P2: sd RW, rt read, 24 B; nine P2) 776, the two dot products 24 and
# the p update 24.
BATCH_BYTES_PER_CELL_ITERATION = 32 + 48 + 32 + 10 * 56 + 9 * 24 + 24 + 24


def batch_bench(tc, count: int, seed: int = 3, tol: float = 1e-8,
                modes=("fp64", "mixed", "fp64_sequential")):
    """Batched heat-conduction solves: `count` instances of log-uniform size
    64^2..1024^2 (synthgen.batch_sizes), all submitted at once, to `tol`
    relative residual; FP64 sweeps, FP32 sweeps with FP64 reductions and
    refinement, and FP64 solves one at a time (the sequential baseline)."""
    import numpy as np
    from synthgen import batch_sizes
    unknown = set(modes) - {"fp64", "mixed", "fp64_sequential"}
    if unknown:
        raise SystemExit(f"unknown batched-solve modes {sorted(unknown)}: use fp64, mixed, fp64_sequential")
    sizes = batch_sizes(count, seed)
    cells = sum((n + 2) ** 2 for n, _ in sizes)
    out = {"instances": count, "sizes": "n log-uniform in [64, 1024), 2D", "tol": tol}
    for mode in modes:
        seq = mode == "fp64_sequential"
        with tc.Context(0) as c, tc.Batch(c, mixed=(mode == "mixed"), max_instances=1 if seq else count,
                                         max_cells=max(n * n for n, _ in sizes) if seq else cells,
                                         hbm_budget=200 << 30, replays_per_step=8 if seq else 4) as b:
            t0 = time.perf_counter()
            tickets = [b.tc_batch_submit(2, n, s, tol=tol) for n, s in sizes]
            b.tc_batch_wait()
            dt = time.perf_counter() - t0
            rs = [b.tc_batch_poll(t) for t in tickets]
        lat = np.array([r["seconds"] for r in rs])
        cell_iters = float(sum(n * n * r["iterations"] for (n, _), r in zip(sizes, rs)))
        out[mode] = {"solves_per_s": count / dt, "makespan_s": dt, "p50_latency_s": float(np.percentile(lat, 50)),
                     "p99_latency_s": float(np.percentile(lat, 99)),
                     "iterations": int(sum(r["iterations"] for r in rs)),
                     "converged": int(sum(r["converged"] for r in rs)),
                     "max_rel_residual": float(max(r["rel_residual"] for r in rs)),
                     "cell_iterations": cell_iters}
        if mode != "mixed":
            # the paper's effective bandwidth: the per-loop byte model of one
            # FP64 PPCG iteration per cell (BATCH_BYTES_PER_CELL_ITERATION)
            # over the makespan; fused Chebyshev launches and cache-resident
            # small instances move fewer bytes than the model counts, so it
            # can exceed the HBM peak (a model figure, not a roofline fraction)
            eff = cell_iters * BATCH_BYTES_PER_CELL_ITERATION / dt / 1e9
            out[mode]["effective_bandwidth"] = {"GBps": eff, "of_hbm_peak": eff / HBM_PEAK_GBS,
                                                "bytes_per_cell_iteration": BATCH_BYTES_PER_CELL_ITERATION,
                                                "model": "per-loop bytes of one PPCG iteration, makespan time"}
        log(f"batch {mode}: {out[mode]['solves_per_s']:.1f} solves/s, makespan {dt:.2f} s, "
            f"converged {out[mode]['converged']}/{count}")
    if "fp64_sequential" in out:
        for mode, key in (("mixed", "mixed_over_sequential_fp64"), ("fp64", "fp64_batched_over_sequential")):
            if mode in out:
                out[key] = out[mode]["solves_per_s"] / out["fp64_sequential"]["solves_per_s"]
    return out


def serve_bench(tc, rate: float, seconds: float, drain: float, seed: int = 4, tol: float = 1e-8):
    """Serving: Poisson arrivals at `rate` solves/s for `seconds` seconds, each
    a 2D (128^2..2048^2) or 3D (64^3..256^3) solve (synthgen.serving_requests),
    replayed in real time against a batch engine (continuous batching,
    admission by HBM footprint); unfinished work is drained for at most
    `drain` seconds.  Latency = completion - arrival of completed solves."""
    import numpy as np
    from paper_1704_00693_amd.apps import serve
    from synthgen import serving_requests
    reqs = serving_requests(rate, seconds, seed)
    out = {"rate_per_s": rate, "window_s": seconds, "requests": len(reqs), "tol": tol}
    for mode in ("fp64", "mixed"):
        with tc.Context(0) as c:
            r = serve(c, reqs, mixed=(mode == "mixed"), tol=tol, max_instances=512, hbm_budget=160 << 30,
                      max_cells=1 << 29, horizon=seconds, drain=drain)
        lat = np.array([v for v in r["latency"] if v is not None])
        done = len(lat)
        out[mode] = {"completed": done, "submitted": r["submitted"], "wall_s": r["wall_s"],
                     "solves_per_s": done / r["wall_s"],
                     "p50_latency_s": float(np.percentile(lat, 50)) if done else None,
                     "p99_latency_s": float(np.percentile(lat, 99)) if done else None}
        log(f"serve {mode}: {done}/{len(reqs)} completed in {r['wall_s']:.1f} s, "
            f"p50 {out[mode]['p50_latency_s']} s, p99 {out[mode]['p99_latency_s']} s")
    return out


def _timed(fn, steps, warm=0.5):
    import torch
    t0 = time.perf_counter()
    k = 0
    while k < 2 or time.perf_counter() - t0 < warm:
        fn()
        k += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _tune(ctx, fn, limit=80):
    """Flush until the autotuner has measured its candidates for the chain
    structures fn records (tc_stats.tuning drops to 0), at most `limit` times."""
    for _ in range(limit):
        fn()
        if not ctx.tc_get_stats()["tuning"]:
            return True
    return False


def other_workloads(tc, which, steps, jacobi_sizes=(8192,), jacobi_skew_rows=(), jacobi_two_columns=True,
                    tealeaf_sizes=(256,), jacobi_select=None, jacobi_variants=("non_copy", "copy"),
                    chain3d_staged=False):
    """The other configurations, each in the execution modes that apply:
    heat-conduction PPCG 256^2 (50 iterations of 10 Chebyshev steps), the
    256^3 Taylor-Green RK3 step, the 8192^2 Jacobi iteration (250 iterations,
    copy and non-copy) and (optionally) the 384^3 synthetic chain."""
    out = {}
    modes = [("none", tc.TC_TILING_NONE, (0, 0, 0)), ("skewed", tc.TC_TILING_SKEWED, (0, 0, 0))]
    if "tealeaf" in which:
        from paper_1704_00693_amd.apps import HeatSolver
        from synthgen import heat_problem
        for n in tealeaf_sizes:
            hp = heat_problem(n, seed=0)
            res = {}
            for name, m, tile in modes + [("fused", tc.TC_TILING_FUSED, (0, 0, 0))]:
                with tc.Context(0) as c:
                    c.tc_set_tiling(m, tile)
                    s = HeatSolver(c, hp.density, hp.energy)
                    dt = _timed(lambda: s.solve(outer=50, inner=10), max(1, steps // 10))
                    st = c.tc_get_stats()
                res[name] = {"seconds_per_solve": dt, "loops_recorded": st["loops_recorded"],
                             "cell_updates_per_s": 50 * 63 * n * n / dt}
            out[f"tealeaf_{n}"] = {"workload": f"heat conduction {n}^2 FP64, PPCG 50 x 10 Chebyshev steps, seed 0",
                                   "modes": res,
                                   "fused_speedup_vs_untiled": res["none"]["seconds_per_solve"] /
                                   res["fused"]["seconds_per_solve"],
                                   "context_paper_speedup": {"2000^2": 3.56, "700^2": 1.07}}
            log(f"tealeaf {n}^2: {res}")
            del hp
    if "euler" in which:
        from paper_1704_00693_amd.apps import EulerRunner
        from synthgen import taylor_green
        n = 256
        q = taylor_green(n)
        res = {}
        for name, m, tile in modes + [("fused", tc.TC_TILING_FUSED, (0, 0, 0))]:
            with tc.Context(0) as c:
                c.tc_set_tiling(m, tile)
                r = EulerRunner(c, q, n, 2 * math.pi / n)
                dt = _timed(lambda: r.step(1e-3), steps)
                st = c.tc_get_stats()
            res[name] = {"ms_per_step": dt * 1e3, "cell_updates_per_s": st["cell_updates"] / dt,
                         "effective_GBps": st["modelled_bytes"] / dt / 1e9, "launches": st["last_launches"],
                         "groups": st["last_groups"]}
        out["euler_rk3_256"] = {"workload": "Taylor-Green vortex 256^3 FP64, one SSP-RK3 step of 4th-order central "
                                            "differences (40 loops + energy sum)", "modes": res}
        log(f"euler 256^3: {res}")
    if "jacobi" in which:
        from paper_1704_00693_amd.apps import JacobiRunner
        from synthgen import JACOBI_POINTS, JACOBI_WEIGHTS, jacobi_field
        iters = 250
        for n in jacobi_sizes:
            u0 = jacobi_field(n, seed=5)
            res = {}
            for variant, copy in (("non_copy", False), ("copy", True)):
                if variant not in jacobi_variants:
                    continue
                per = {}
                extra = [(f"skewed_rows{t}", tc.TC_TILING_SKEWED, (0, t, 0)) for t in jacobi_skew_rows]
                if jacobi_two_columns:
                    # fused kernels with two columns per lane and a 240-register budget
                    # (generator knob TC_JIT_CPL, read when a context starts), and the
                    # autotuner, which has this layout among its candidates
                    extra.append(("fused_2col_regs240", tc.TC_TILING_FUSED, (0, 240, 0)))
                    extra.append(("auto", tc.TC_TILING_AUTO, (0, 0, 0)))
                for name, m, tile in modes + [("fused", tc.TC_TILING_FUSED, (0, 0, 0))] + extra:
                    if jacobi_select and name not in jacobi_select:
                        continue
                    saved = os.environ.get("TC_JIT_CPL")
                    if name == "fused_2col_regs240":
                        os.environ["TC_JIT_CPL"] = "2"
                    try:
                        with tc.Context(0) as c:
                            c.tc_set_tiling(m, tile)
                            r = JacobiRunner(c, u0, JACOBI_POINTS, JACOBI_WEIGHTS, copy)
                            settled = True
                            if m == tc.TC_TILING_AUTO:
                                settled = _tune(c, lambda: r.run(iters))
                            dt = _timed(lambda: r.run(iters), steps)
                            st = c.tc_get_stats()
                    finally:
                        if saved is None:
                            os.environ.pop("TC_JIT_CPL", None)
                        else:
                            os.environ["TC_JIT_CPL"] = saved
                    per[name] = {"seconds_per_run": dt, "cell_iterations_per_s": iters * n * n / dt,
                                 "ps_per_point_iteration": dt / (iters * n * n) * 1e12,
                                 "effective_GBps": st["modelled_bytes"] / dt / 1e9, "launches": st["last_launches"],
                                 "groups": st["last_groups"]}
                    if m == tc.TC_TILING_AUTO:
                        per[name].update({"tuned": settled, "chosen_mode": st["last_mode"],
                                          "chosen_tile": st["last_tile"], "chosen_columns_per_lane": st["last_cpl"]})
                fused_names = [k for k in per if k.startswith("fused")]
                if fused_names and "none" in per:
                    best_fused = min(fused_names, key=lambda k: per[k]["seconds_per_run"])
                    per["fused_best_layout"] = best_fused
                    per["fused_speedup_vs_untiled"] = (per["none"]["seconds_per_run"] /
                                                       per[best_fused]["seconds_per_run"])
                res[variant] = per
                log(f"jacobi {n}^2 {variant}: {per}")
            out[f"jacobi_{n}"] = {
                "workload": f"Jacobi heat equation {n}^2 FP64 with a one-cell Dirichlet layer, 250 iterations of "
                            "the 5-point stencil (all weights 0.2), copy and non-copy variants, uniform [0,1) field, "
                            "seed 5",
                "footprint_MB": 2 * (n + 2) ** 2 * 8 / 1e6,
                "modes": res}
            if n == 8192:
                out[f"jacobi_{n}"]["context_paper_cpu_seconds_untiled_tiled"] = {"copy": [16.06, 5.11],
                                                                                  "non_copy": [8.58, 3.69]}
            del u0
    if "chain3d" in which:
        from paper_1704_00693_amd.apps import ChainRunner
        from synthgen import chain_3d, chain_data
        ch = chain_3d()
        data = chain_data(ch)
        res = {}
        # fused: the split search keeps a loop on its own kernel unless a
        # group is modelled faster; fused_staged_all: every run the staged
        # analysis accepts becomes a staged group (TC_STAGED=2), to time them
        runs = [(None, modes + [("fused", tc.TC_TILING_FUSED, (0, 0, 0))])]
        if chain3d_staged:
            runs.append(("2", [("fused_staged_all", tc.TC_TILING_FUSED, (0, 0, 0))]))
        for env, ms in runs:
            old = os.environ.get("TC_STAGED")
            if env is not None:
                os.environ["TC_STAGED"] = env
            try:
                with tc.Context(0) as c:
                    r = ChainRunner(c, ch, data)
                    for name, m, tile in ms:
                        c.tc_set_tiling(m, tile)
                        dt = _timed(lambda: r.run(), steps)
                        st = c.tc_get_stats()
                        res[name] = {"ms_per_step": dt * 1e3, "cell_updates_per_s": st["cell_updates"] / dt,
                                     "effective_GBps": st["modelled_bytes"] / dt / 1e9,
                                     "launches": st["last_launches"], "groups": st["last_groups"]}
            finally:
                if env is not None:
                    if old is None:
                        del os.environ["TC_STAGED"]
                    else:
                        os.environ["TC_STAGED"] = old
        del data
        out["chain_384_3d"] = {"workload": "3D synthetic chain 384^3 FP64, 25 datasets, 60 loops of 7/13-point "
                                           "stars + final sum, seed 2", "modes": res}
        log(f"chain 384^3: {res}")
    return out


_CPU_WORKER = """
import sys, time
sys.path.insert(0, {root!r})
import oracle
from synthgen import make_chain, chain_data
ch = make_chain(2, {n}, {ndat}, {nloops}, {seed})
data = chain_data(ch)
print("ready", flush=True)
sys.stdin.readline()
t0 = time.perf_counter()
oracle.run_chain(ch, data)
print(ch.cell_updates(), time.perf_counter() - t0, flush=True)
"""


def cpu_baseline(ch_full, n_sample: int, procs: int = 0):
    """The oracle (single-threaded C, FP64) on the same chain over an
    n_sample^2 grid (a bounded sample of the workload), run as one process
    per host core at once (at most 16, the host share of one GPU); the
    throughput is the sum of the processes' cell-updates over the wall time
    of the slowest.  The processes only import the oracle; none touches the
    GPU."""
    import subprocess
    if procs <= 0:
        procs = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))
    code = _CPU_WORKER.format(root=ROOT, n=n_sample, ndat=ch_full.ndat, nloops=len(ch_full.loops), seed=ch_full.seed)
    ps = [subprocess.Popen([sys.executable, "-c", code], stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)
          for _ in range(procs)]
    for p in ps:
        assert p.stdout.readline().strip() == "ready"
    t0 = time.perf_counter()
    for p in ps:  # inputs are generated: start the timed runs together
        p.stdin.write("go\n")
        p.stdin.flush()
    cells = 0
    for p in ps:
        c, _ = p.stdout.readline().split()
        cells += int(c)
        p.wait()
    wall = time.perf_counter() - t0
    return {"value": cells / wall, "unit": "cell-updates/s", "cores": procs, "kind": "oracle",
            "sample": f"same 40-loop chain on a {n_sample}^2 grid, {procs} single-threaded oracle processes at once "
                      f"({cells} cell-updates in {wall:.1f} s wall)",
            "cpu": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# counter ingestion (host only): rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs
# ---------------------------------------------------------------------------
def _family(name: str) -> str:
    if "tcj_g" in name:
        return "fused"
    if "OpCopy" in name:
        return "copy"
    if "wsum" in name or "OpWsum" in name:
        return "wsum"
    return "other"


MODE_FAMILY = {"copy": "copy", "fused": "fused", "none": "wsum", "skewed": "wsum"}


def ingest_counters(spec):
    """spec: MODE:COUNTER:DIR:FLUSHES entries (FLUSHES = flushes of that mode
    in the profiled run).  Writes profiles/traffic.json: per mode, the HBM
    bytes per flush and per dispatch of its chain kernels, scaled so that the
    copy kernel reads and writes exactly its algorithmic bytes."""
    raw = {}
    for item in spec:
        mode, counter, d, flushes = item.split(":")
        tot, disp = 0.0, 0
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter or _family(r["Kernel_Name"]) != MODE_FAMILY[mode]:
                    continue
                tot += float(r["Counter_Value"]) * 1024.0  # counters are in KiB
                disp += 1
        raw.setdefault(mode, {})[counter] = {"bytes": tot, "dispatches": disp, "flushes": int(flushes)}
    cal = raw["copy"]
    half = json.load(open(os.path.join(ROOT, "profiles", "copy_probe.json")))["alg_bytes_per_launch"] / 2
    f_fetch = half / (cal["FETCH_SIZE"]["bytes"] / cal["FETCH_SIZE"]["dispatches"])
    f_write = half / (cal["WRITE_SIZE"]["bytes"] / cal["WRITE_SIZE"]["dispatches"])
    out = {"source_sha": kernel_source_sha(),
           "calibration": {"copy_bytes_read_per_launch": half, "copy_bytes_written_per_launch": half,
                           "factor_fetch": f_fetch, "factor_write": f_write},
           "modes": {}}
    for mode, ent in raw.items():
        if mode == "copy":
            continue
        fe, wr = ent["FETCH_SIZE"], ent["WRITE_SIZE"]
        rd = fe["bytes"] * f_fetch / fe["flushes"]
        wt = wr["bytes"] * f_write / wr["flushes"]
        disp = fe["dispatches"] / fe["flushes"]
        out["modes"][mode] = {"hbm_bytes_per_flush": rd + wt, "read_bytes_per_flush": rd,
                              "write_bytes_per_flush": wt, "dispatches_per_flush": disp,
                              "hbm_bytes_per_launch": (rd + wt) / disp}
    with open(TRAFFIC_JSON, "w") as fp:
        json.dump(out, fp, indent=1)
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--modes", default="none,skewed,fused",
                    help="comma list of none, skewed, fused; 'copy' alone runs the copy probe")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--warm-seconds", type=float, default=WARM_SECONDS,
                    help="least wall time each chain mode is warmed before timing (counter runs use 0)")
    ap.add_argument("--cpu-sample", type=int, default=2048, help="grid edge of the oracle's timed sample (0: skip)")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle processes run at once for the CPU baseline (0: one per host core, at most 16)")
    ap.add_argument("--fused-tile", default="0,0,0",
                    help="fused mode tile: rows per wavefront segment, window-register budget, most loops per group "
                         "(0: automatic)")
    ap.add_argument("--batch-count", type=int, default=512,
                    help="batched heat-conduction solves to run after the chain (0: skip)")
    ap.add_argument("--other", default="tealeaf,euler,jacobi,chain3d",
                    help="other workloads to time: comma list of tealeaf, euler, jacobi, chain3d ('' to skip)")
    ap.add_argument("--jacobi-n", default="8192",
                    help="grid edges of the Jacobi workload, comma list (a cache-capacity sweep)")
    ap.add_argument("--tealeaf-n", default="256",
                    help="grid edges of the heat-conduction PPCG workload, comma list (a problem-size sweep)")
    ap.add_argument("--jacobi-skew-rows", default="",
                    help="extra skewed Jacobi runs with these tile heights in rows, comma list (a tile-height study)")
    ap.add_argument("--jacobi-one-layout", action="store_true",
                    help="time the fused Jacobi in its default layout only (no two-column layout, no autotuner)")
    ap.add_argument("--jacobi-select", default="",
                    help="Jacobi modes to time, comma list of none, skewed, fused, fused_2col_regs240, auto "
                         "(default: all)")
    ap.add_argument("--chain3d-staged", action="store_true",
                    help="also time the 3D chain with every run the staged analysis accepts as a staged group")
    ap.add_argument("--jacobi-variants", default="non_copy,copy", help="Jacobi variants to time: non_copy, copy")
    ap.add_argument("--batch-modes", default="fp64,mixed,fp64_sequential",
                    help="batched-solve modes to time: fp64, mixed, fp64_sequential")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="serving trace window in seconds (0: skip); arrivals at --serve-rate")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-drain", type=float, default=15.0)
    ap.add_argument("--ingest-counters", nargs="*", default=None,
                    help="host only: MODE:COUNTER:DIR:FLUSHES entries from rocprofv3 --pmc runs")
    args = ap.parse_args()
    if args.ingest_counters is not None:
        ingest_counters(args.ingest_counters)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(several GPUs would split the grid into slabs with one deep-halo exchange per chain; "
              "that path is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1704_00693_amd as tc
    from paper_1704_00693_amd.apps import ChainRunner
    from synthgen import chain_2d, chain_data

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.modes == "copy":
        print(json.dumps(copy_probe(tc, args.n, args.steps, args.warmup)))
        return
    copy = copy_probe(tc, args.n, 10, 2, reference=args.warm_seconds > 0)
    log(f"copy probe: {copy['GBps']:.0f} GB/s (runtime's copy of 2 GiB: {copy['reference_copy_GBps']} GB/s)")
    ch = chain_2d(n=args.n)
    log(f"generating inputs: {ch.ndat} x {ch.n + 4}^2 FP64")
    data = chain_data(ch)
    cells = ch.cell_updates()
    results = {}
    with tc.Context(0) as ctx:
        runner = ChainRunner(ctx, ch, data)
        del data
        torch.cuda.synchronize()
        for name in args.modes.split(","):
            mode = MODE_NAMES[name]
            log(f"mode {name}: warmup {args.warmup}, steps {args.steps}")
            try:
                tile = tuple(int(v) for v in args.fused_tile.split(",")) if name == "fused" else (0, 0, 0)
                results[name] = time_mode(ctx, runner, mode, tile, args.steps, args.warmup, cells, args.warm_seconds)
            except tc.TcError as e:
                if e.status != tc.TC_ERR_UNSUPPORTED:
                    raise
                log(f"mode {name} unsupported: {e}")
                continue
            log(f"  {results[name]['ms_per_step']:.3f} ms/step, "
                f"{results[name]['cell_updates_per_s'] / 1e9:.2f} Gcell/s, "
                f"{results[name]['effective_GBps']:.0f} GB/s effective")
    tiled = {k: v for k, v in results.items() if k != "none"}
    best_name = max(tiled, key=lambda k: tiled[k]["cell_updates_per_s"]) if tiled else "none"
    best = results[best_name]
    if best_name == "fused" and best["groups"] > 0:
        # dominant kernels: the generated fused-group kernels (one interior and
        # one edge launch per group); algorithmic bytes = chain-start datasets
        # read + datasets written, once over the group's range
        launches = best["groups"]
        secs = best["fused_kernel_seconds"]
        alg = best["fused_bytes"] / launches
        kname = "tcj_g*_in + tcj_g*_edge (generated fused-group kernels), per group"
    else:
        launches = max(best["kernel_launches"], 1)
        secs = best["kernel_seconds"]
        alg = best["modelled_bytes"] / launches
        kname = "wsum_march_kernel (per-loop weighted sum)"
    avg = secs / launches
    achieved = alg / avg / 1e9 if avg > 0 else 0.0
    tr = traffic_entry(best_name)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": None if tr is None else tr["hbm_bytes_per_flush"] / launches,
                "kernel": kname, "avg_launch_us": avg * 1e6, "algorithmic_bytes_per_launch": alg}
    others = (other_workloads(tc, args.other.split(","), 10, [int(v) for v in args.jacobi_n.split(",")],
                              [int(v) for v in args.jacobi_skew_rows.split(",") if v], not args.jacobi_one_layout,
                              [int(v) for v in args.tealeaf_n.split(",")],
                              [v for v in args.jacobi_select.split(",") if v] or None,
                              tuple(v for v in args.jacobi_variants.split(",") if v), args.chain3d_staged)
              if args.other else None)
    batched = (batch_bench(tc, args.batch_count, modes=[m for m in args.batch_modes.split(",") if m])
               if args.batch_count > 0 else None)
    served = serve_bench(tc, args.serve_rate, args.serve_seconds, args.serve_drain) if args.serve_seconds > 0 else None
    cpu = cpu_baseline(ch, args.cpu_sample, args.cpu_procs) if args.cpu_sample > 0 else None
    untiled = results.get("none")
    tr_none = traffic_entry("none")
    line = {
        "metric": METRIC,
        "value": best["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D synthetic loop chain {ch.n}^2 FP64, 12 datasets (halo 2), 40 weighted-sum "
                               f"loops with 5/9-point stencils, seed {ch.seed}",
                   "tiling": best_name},
        "effective_GBps": best["effective_GBps"],
        "untiled": None if untiled is None else {
            "cell_updates_per_s": untiled["cell_updates_per_s"], "ms_per_step": untiled["ms_per_step"],
            "effective_GBps": untiled["effective_GBps"],
            "hbm_bytes_per_flush": None if tr_none is None else tr_none["hbm_bytes_per_flush"]},
        "speedup_vs_untiled": None if untiled is None else best["cell_updates_per_s"] / untiled["cell_updates_per_s"],
        "hbm_bytes_per_flush": None if tr is None else tr["hbm_bytes_per_flush"],
        "hbm_byte_ratio_untiled_over_tiled": (None if tr is None or tr_none is None
                                              else tr_none["hbm_bytes_per_flush"] / tr["hbm_bytes_per_flush"]),
        "copy_probe_GBps": copy["GBps"],
        "reference_copy_GBps": copy["reference_copy_GBps"],
        "modes": results,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "other_workloads": others,
        "batched_solves": batched,
        "serving": served,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
