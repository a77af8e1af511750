"""Python binding of the tilechain C ABI (``include/tilechain.h``).

Argument marshalling only: every loop runs in the HIP kernels of
``libtilechain.so``.  The functions keep the C names (``tc_init``,
``tc_par_loop``, ...).  Device memory comes from PyTorch's caching allocator
through the allocator callbacks of ``tc_init`` and work runs on PyTorch's
current HIP stream, so the library interleaves with torch work.

The shared library must have been built (``python -m paper_1704_00693_amd.build``
or ``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtilechain.so")

# ---- enums (mirror include/tilechain.h) -----------------------------------
TC_OK, TC_ERR_ARG, TC_ERR_STATE, TC_ERR_DEVICE, TC_ERR_NOMEM, TC_ERR_UNSUPPORTED, TC_ERR_RANGE = 0, -1, -2, -3, -4, -5, -6
TC_F64, TC_F32 = 0, 1
TC_READ, TC_WRITE, TC_RW, TC_INC = 0, 1, 2, 3
TC_ARG_DAT, TC_ARG_RED = 0, 1
TC_RED_SUM, TC_RED_MIN, TC_RED_MAX = 0, 1, 2
TC_TILING_NONE, TC_TILING_SKEWED, TC_TILING_FUSED, TC_TILING_AUTO = 0, 1, 2, 3
TC_INIT_HOST_ONLY = 1
TC_INIT_BORROW_STREAM = 2
OPS = {
    "WSUM": 0, "COPY": 1, "AXPBY": 2, "DOT": 3, "SUM": 4, "HALO_REFLECT": 5,
    "TEA_INIT": 10, "TEA_K": 11, "TEA_RESID": 12, "TEA_MATVEC_DOT": 13, "TEA_P1": 14, "TEA_P2": 15,
    "TEA_PRECON_INIT": 16, "TEA_CG_UPDATE": 17, "TEA_CG_P": 18, "TEA_GERSH": 19,
    "EULER_PRIM": 20, "EULER_RHS": 21, "RK_STAGE": 22,
}
ACCESS = {"R": TC_READ, "W": TC_WRITE, "RW": TC_RW, "INC": TC_INC}
EXPORTS = ["tc_init", "tc_finalize", "tc_decl_block", "tc_decl_dat", "tc_decl_stencil", "tc_decl_reduction",
           "tc_par_loop", "tc_par_loops", "tc_reduction_result", "tc_reduction_result_static", "tc_flush", "tc_dat_read", "tc_dat_write", "tc_dat_device_view",
           "tc_set_tiling", "tc_set_profiling", "tc_get_stats", "tc_chain_plan", "tc_staged_tiles", "tc_pending", "tc_status_string",
           "tc_last_error", "tc_batch_create", "tc_batch_submit", "tc_batch_step", "tc_batch_poll", "tc_batch_wait",
           "tc_batch_read_x", "tc_batch_destroy"]
TC_SOLVE_PENDING, TC_SOLVE_RUNNING, TC_SOLVE_DONE, TC_SOLVE_REJECTED = 0, 1, 2, -1


class TcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class InitOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("flags", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_user", ctypes.c_void_p)]


class Arg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("handle", ctypes.c_int32), ("stencil", ctypes.c_int32),
                ("access", ctypes.c_int32)]


class LoopSpec(ctypes.Structure):
    """tc_loop: one loop of a tc_par_loops call."""
    _fields_ = [("op", ctypes.c_int32), ("block", ctypes.c_int32), ("range", ctypes.c_int32 * 6),
                ("first_arg", ctypes.c_int32), ("nargs", ctypes.c_int32), ("first_param", ctypes.c_int32),
                ("nparams", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("loops_recorded", ctypes.c_int64), ("flushes", ctypes.c_int64), ("plan_hits", ctypes.c_int64),
                ("plan_misses", ctypes.c_int64), ("plan_seconds", ctypes.c_double),
                ("max_skew", ctypes.c_int32 * 3), ("last_tiles", ctypes.c_int32), ("last_groups", ctypes.c_int32),
                ("last_launches", ctypes.c_int32), ("last_mode", ctypes.c_int32),
                ("modelled_bytes", ctypes.c_int64), ("cell_updates", ctypes.c_int64),
                ("last_flush_seconds", ctypes.c_double), ("prof_kernel_seconds", ctypes.c_double),
                ("prof_launches", ctypes.c_int64), ("fused_bytes", ctypes.c_int64),
                ("prof_fused_seconds", ctypes.c_double), ("jit_compile_seconds", ctypes.c_double),
                ("last_tile", ctypes.c_int32 * 3), ("last_cpl", ctypes.c_int32), ("tuning", ctypes.c_int32),
                ("pad", ctypes.c_int32)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name in ("max_skew", "last_tile") else v
        return out


class BatchOpts(ctypes.Structure):
    _fields_ = [("mixed", ctypes.c_int32), ("max_instances", ctypes.c_int32), ("max_cells", ctypes.c_int64),
                ("hbm_budget", ctypes.c_int64), ("cheb_steps", ctypes.c_int32), ("replays_per_step", ctypes.c_int32),
                ("inner_tol", ctypes.c_double)]


class SolveDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32), ("seed", ctypes.c_uint64), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("max_outer", ctypes.c_int32), ("dt", ctypes.c_double),
                ("keep_x", ctypes.c_int32), ("pad", ctypes.c_int32)]


class SolveResult(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("iterations", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("bnorm", ctypes.c_double),
                ("lmax", ctypes.c_double), ("seconds", ctypes.c_double), ("queue_seconds", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load libtilechain.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1704_00693_amd.build`")
    # torch's wheel carries its own HIP runtime under the same soname: loaded
    # first, it is the one the library binds to, so the streams and memory a
    # context borrows from torch belong to the library's runtime too (loaded
    # after the library, a second HIP and HSA runtime would come up beside it)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    i32p = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "tc_init": [ctypes.POINTER(InitOpts), ctypes.POINTER(P)],
        "tc_finalize": [P],
        "tc_decl_block": [P, ctypes.c_int, ctypes.c_char_p, i32p],
        "tc_decl_dat": [P, i32, i32, i32p, i32p, i32p, P, ctypes.c_char_p, i32p],
        "tc_decl_stencil": [P, ctypes.c_int, ctypes.c_int, i32p, ctypes.c_char_p, i32p],
        "tc_decl_reduction": [P, i32, ctypes.c_char_p, i32p],
        "tc_par_loop": [P, ctypes.c_char_p, i32, i32, i32p, ctypes.POINTER(Arg), ctypes.c_int,
                        ctypes.POINTER(ctypes.c_double), ctypes.c_int],
        "tc_par_loops": [P, i32, ctypes.POINTER(LoopSpec), ctypes.POINTER(Arg), ctypes.POINTER(ctypes.c_double),
                         i32p],
        "tc_reduction_result": [P, i32, ctypes.POINTER(ctypes.c_double)],
        "tc_reduction_result_static": [P, i32, ctypes.POINTER(ctypes.c_double)],
        "tc_staged_tiles": [P, i32p, i32, i32p, i32p, i64],
        "tc_flush": [P],
        "tc_dat_read": [P, i32, P],
        "tc_dat_write": [P, i32, P],
        "tc_dat_device_view": [P, i32, ctypes.POINTER(P), ctypes.POINTER(i64)],
        "tc_set_tiling": [P, i32, i32p],
        "tc_get_stats": [P, ctypes.POINTER(Stats)],
        "tc_set_profiling": [P, ctypes.c_int],
        "tc_chain_plan": [P, i32, i32p, i32p, i32p, i64],
        "tc_pending": [P, i32p],
        "tc_status_string": [i32],
        "tc_last_error": [P],
        "tc_batch_create": [P, ctypes.POINTER(BatchOpts), ctypes.POINTER(P)],
        "tc_batch_submit": [P, ctypes.POINTER(SolveDesc), ctypes.POINTER(i64)],
        "tc_batch_step": [P, i32p],
        "tc_batch_poll": [P, i64, ctypes.POINTER(SolveResult)],
        "tc_batch_wait": [P],
        "tc_batch_read_x": [P, i64, ctypes.POINTER(ctypes.c_double), i64],
        "tc_batch_destroy": [P],
    }
    for name, argtypes in sig.items():
        f = getattr(L, name)
        f.argtypes = argtypes
        f.restype = ctypes.c_char_p if name in ("tc_status_string", "tc_last_error") else ctypes.c_int32
    _lib = L
    return L


def _i32(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_int32 * max(len(vals), 1))(*vals)


class Context:
    """One tilechain context (``tc_ctx*``) plus the Python objects that must
    outlive it (allocator callbacks and the tensors they handed out)."""

    def __init__(self, device: int = 0, host_only: bool = False, torch_memory: bool = True,
                 stream: Optional[int] = None):
        L = lib()
        self._tensors: Dict[int, object] = {}
        self._loop_arrays: Dict[tuple, tuple] = {}
        self._capture: Optional[list] = None
        self._no_params = (ctypes.c_double * 1)()
        opts = InitOpts()
        opts.device = device
        opts.flags = TC_INIT_HOST_ONLY if host_only else 0
        self._alloc_cb = ALLOC_FN(0)
        self._free_cb = FREE_FN(0)
        if not host_only:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("tilechain needs a HIP device (torch.cuda.is_available() is False)")
            torch.cuda.set_device(device)
            if stream is None:
                stream = torch.cuda.current_stream(device).cuda_stream
            opts.stream = stream
            opts.flags |= TC_INIT_BORROW_STREAM
            if torch_memory:
                dev = torch.device("cuda", device)

                def _alloc(nbytes, _user):
                    try:
                        t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
                    except RuntimeError:
                        return None
                    p = t.data_ptr()
                    self._tensors[p] = t
                    return p

                def _free(ptr, _user):
                    self._tensors.pop(ptr, None)

                self._alloc_cb = ALLOC_FN(_alloc)
                self._free_cb = FREE_FN(_free)
                opts.alloc = self._alloc_cb
                opts.free = self._free_cb
        self.ptr = ctypes.c_void_p()
        st = L.tc_init(ctypes.byref(opts), ctypes.byref(self.ptr))
        if st != TC_OK:
            raise TcError(st, "tc_init failed")
        self.host_only = host_only
        self.dat_shapes: Dict[int, tuple] = {}
        self.dat_dtypes: Dict[int, int] = {}

    # error helper
    def _ck(self, st: int, what: str):
        if st != TC_OK:
            msg = lib().tc_last_error(self.ptr).decode()
            raise TcError(st, f"{what}: {msg}")

    def close(self):
        if self.ptr:
            st = lib().tc_finalize(self.ptr)
            self.ptr = ctypes.c_void_p()
            self._tensors.clear()
            if st != TC_OK:
                raise TcError(st, "tc_finalize failed")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- declarations ----------------------------------------------------
    def tc_decl_block(self, ndim: int, name: str = "") -> int:
        out = ctypes.c_int32()
        self._ck(lib().tc_decl_block(self.ptr, ndim, name.encode(), ctypes.byref(out)), "tc_decl_block")
        return out.value

    def tc_decl_dat(self, blk: int, size: Sequence[int], halo_neg: Sequence[int], halo_pos: Sequence[int],
                    init: Optional[np.ndarray] = None, dtype: int = TC_F64, name: str = "") -> int:
        out = ctypes.c_int32()
        ptr = None
        keep = None
        npdt = np.float64 if dtype == TC_F64 else np.float32
        shape = tuple(int(s) + int(a) + int(b) for s, a, b in zip(size, halo_neg, halo_pos))[::-1]
        if init is not None:
            keep = np.ascontiguousarray(init, dtype=npdt)
            if keep.shape != shape:
                raise ValueError(f"init has shape {keep.shape}, expected padded shape {shape}")
            ptr = keep.ctypes.data
        self._ck(lib().tc_decl_dat(self.ptr, blk, dtype, _i32(size), _i32(halo_neg), _i32(halo_pos), ptr,
                                   name.encode(), ctypes.byref(out)), "tc_decl_dat")
        self.dat_shapes[out.value] = shape
        self.dat_dtypes[out.value] = dtype
        return out.value

    def tc_decl_stencil(self, points: Sequence[Sequence[int]], name: str = "") -> int:
        pts = [tuple(p) for p in points]
        ndim = len(pts[0])
        flat = [c for p in pts for c in p]
        out = ctypes.c_int32()
        self._ck(lib().tc_decl_stencil(self.ptr, ndim, len(pts), _i32(flat), name.encode(), ctypes.byref(out)),
                 "tc_decl_stencil")
        return out.value

    def tc_decl_reduction(self, op: int = TC_RED_SUM, name: str = "") -> int:
        out = ctypes.c_int32()
        self._ck(lib().tc_decl_reduction(self.ptr, op, name.encode(), ctypes.byref(out)), "tc_decl_reduction")
        return out.value

    # ---- loops -------------------------------------------------------------
    def tc_par_loop(self, op, blk: int, rng: Sequence[int], args, params: Sequence[float] = (), name: str = ""):
        """args: tuples (dat, stencil, access) for datasets, ("red", handle)
        for reductions; access as "R"/"W"/"RW"/"INC" or the TC_ constant."""
        if self._capture is not None:  # building a LoopBatch: keep the loop instead
            self._capture.append((op, blk, tuple(rng), tuple(args), tuple(float(p) for p in params)))
            return
        # the marshalled op, range and argument arrays of a loop shape are
        # kept (applications record the same shapes every iteration)
        key = (op, blk, tuple(rng), tuple(args), name)
        m = self._loop_arrays.get(key)
        if m is None:
            opc = OPS[op] if isinstance(op, str) else int(op)
            arr = (Arg * max(len(args), 1))()
            for i, a in enumerate(args):
                if a[0] == "red":
                    arr[i] = Arg(TC_ARG_RED, int(a[1]), 0, 0)
                else:
                    acc = ACCESS[a[2]] if isinstance(a[2], str) else int(a[2])
                    arr[i] = Arg(TC_ARG_DAT, int(a[0]), int(a[1]), acc)
            if len(self._loop_arrays) > 4096:
                self._loop_arrays.clear()
            m = self._loop_arrays[key] = (opc, arr, len(args), _i32(rng), name.encode())
        opc, arr, nargs, rarr, bname = m
        n = len(params)
        prm = (ctypes.c_double * n)(*params) if n else self._no_params
        st = lib().tc_par_loop(self.ptr, bname, opc, blk, rarr, arr, nargs, prm, n)
        if st != TC_OK:
            self._ck(st, f"tc_par_loop({name})")

    def capture(self):
        """Context manager: tc_par_loop calls inside it are collected (not
        recorded) into the list it yields, for a LoopBatch."""
        ctx = self

        class _Cap:
            def __enter__(self_):
                ctx._capture = []
                return ctx._capture

            def __exit__(self_, *exc):
                ctx._capture = None
                return False

        return _Cap()

    def tc_flush(self):
        self._ck(lib().tc_flush(self.ptr), "tc_flush")

    def tc_reduction_result(self, red: int) -> float:
        out = ctypes.c_double()
        self._ck(lib().tc_reduction_result(self.ptr, red, ctypes.byref(out)), "tc_reduction_result")
        return out.value

    def tc_reduction_result_static(self, red: int) -> float:
        """tc_reduction_result that allocates no device memory (static scratch)."""
        out = ctypes.c_double()
        self._ck(lib().tc_reduction_result_static(self.ptr, red, ctypes.byref(out)), "tc_reduction_result_static")
        return out.value

    def tc_dat_read(self, dat: int) -> np.ndarray:
        npdt = np.float64 if self.dat_dtypes[dat] == TC_F64 else np.float32
        out = np.empty(self.dat_shapes[dat], dtype=npdt)
        self._ck(lib().tc_dat_read(self.ptr, dat, out.ctypes.data), "tc_dat_read")
        return out

    def tc_dat_write(self, dat: int, values: np.ndarray):
        npdt = np.float64 if self.dat_dtypes[dat] == TC_F64 else np.float32
        a = np.ascontiguousarray(values, dtype=npdt)
        if a.shape != self.dat_shapes[dat]:
            raise ValueError("shape mismatch")
        self._ck(lib().tc_dat_write(self.ptr, dat, a.ctypes.data), "tc_dat_write")

    def tc_dat_device_view(self, dat: int):
        p = ctypes.c_void_p()
        st = (ctypes.c_int64 * 3)()
        self._ck(lib().tc_dat_device_view(self.ptr, dat, ctypes.byref(p), st), "tc_dat_device_view")
        return p.value, list(st)

    def tc_set_tiling(self, mode: int, tile: Sequence[int] = (0, 0, 0)):
        t = list(tile) + [0] * (3 - len(tile))
        self._ck(lib().tc_set_tiling(self.ptr, mode, _i32(t)), "tc_set_tiling")

    def tc_set_profiling(self, on: bool):
        self._ck(lib().tc_set_profiling(self.ptr, 1 if on else 0), "tc_set_profiling")

    def tc_get_stats(self) -> dict:
        s = Stats()
        self._ck(lib().tc_get_stats(self.ptr, ctypes.byref(s)), "tc_get_stats")
        return s.as_dict()

    def tc_pending(self) -> int:
        n = ctypes.c_int32()
        self._ck(lib().tc_pending(self.ptr, ctypes.byref(n)), "tc_pending")
        return n.value

    def tc_chain_plan(self, tile: Sequence[int], nloops: int, ndim: int):
        """Skewed plan of the pending chain: (num_tiles, start[d][t][l], end[d][t][l])."""
        t = list(tile) + [0] * (3 - len(tile))
        nt = (ctypes.c_int32 * 3)()
        st = lib().tc_chain_plan(self.ptr, TC_TILING_SKEWED, _i32(t), nt, None, 0)
        maxt = max(nt)
        cap = ndim * maxt * nloops * 2
        buf = (ctypes.c_int32 * max(cap, 1))()
        self._ck(lib().tc_chain_plan(self.ptr, TC_TILING_SKEWED, _i32(t), nt, buf, cap), "tc_chain_plan")
        a = np.frombuffer(buf, dtype=np.int32, count=cap).reshape(ndim, maxt, nloops, 2)
        num = list(nt)[:ndim]
        start = [[list(a[d, tt, :, 0]) for tt in range(num[d])] for d in range(ndim)]
        end = [[list(a[d, tt, :, 1]) for tt in range(num[d])] for d in range(ndim)]
        return num, start, end


    def tc_fused_groups(self, tile: Sequence[int] = (0, 0, 0)):
        """Fusion groups the fused mode would form for the pending chain, as
        (first, last + 1) loop indices; their kernels are generated and
        compiled (also on host-only contexts), nothing runs."""
        return self.tc_fused_plan(tile)[0]

    def tc_fused_plan(self, tile: Sequence[int] = (0, 0, 0)):
        """Fused-mode analysis of the pending chain: the groups as (first,
        last + 1) loop indices and, per chain loop, (computed, x below, x
        above, y below, y above, z below, z above): computed is 1 / 2 / 0 / -1
        (computed in a register-window group, in a staged group, in a group
        but dead, on its own), the others the points the loop computes beyond
        an owned block."""
        t = list(tile) + [0] * (3 - len(tile))
        nt = (ctypes.c_int32 * 3)()
        lib().tc_chain_plan(self.ptr, TC_TILING_FUSED, _i32(t), nt, None, 0)
        G, L = nt[0], nt[1]
        cap = max(2 * G + 7 * L, 1)
        buf = (ctypes.c_int32 * cap)()
        self._ck(lib().tc_chain_plan(self.ptr, TC_TILING_FUSED, _i32(t), nt, buf, cap), "tc_chain_plan")
        groups = [(int(buf[2 * g]), int(buf[2 * g + 1])) for g in range(G)]
        per = [tuple(int(buf[2 * G + 7 * l + k]) for k in range(7)) for l in range(L)]
        return groups, per

    def tc_staged_tiles(self, group: int, tile: Sequence[int] = (0, 0, 0)):
        """Staged tiles of fusion group ``group`` of the pending chain: (g0, g1,
        owned extents, [(owned lo, owned hi, [computed (lo, hi) or None per
        loop]) per tile]); no tiles for a register-window group."""
        t = list(tile) + [0] * (3 - len(tile))
        info = (ctypes.c_int32 * 6)()
        self._ck(lib().tc_staged_tiles(self.ptr, _i32(t), group, info, None, 0), "tc_staged_tiles")
        g0, g1, T = int(info[0]), int(info[1]), int(info[2])
        ext = tuple(int(info[3 + d]) for d in range(3))
        if T == 0:
            return g0, g1, ext, []
        L = g1 - g0
        per = 6 + 6 * L
        buf = (ctypes.c_int32 * (per * T))()
        self._ck(lib().tc_staged_tiles(self.ptr, _i32(t), group, info, buf, per * T), "tc_staged_tiles")
        tiles = []
        for k in range(T):
            r = buf[per * k: per * (k + 1)]
            own = (list(r[0:3]), list(r[3:6]))
            boxes = []
            for l in range(L):
                lo, hi = list(r[6 + 6 * l: 9 + 6 * l]), list(r[9 + 6 * l: 12 + 6 * l])
                boxes.append(None if any(h <= o for o, h in zip(lo, hi)) else (lo, hi))
            tiles.append((own, boxes))
        return g0, g1, ext, tiles


class LoopBatch:
    """A fixed list of loops recorded with one tc_par_loops call.  Built from
    (op, block, range, args, params) entries (as Context.capture collects
    them); ``params`` is a writable view of all loops' parameters, so a
    caller can change scalars between recordings."""

    def __init__(self, ctx: "Context", loops):
        self.ctx = ctx
        n = len(loops)
        nargs = sum(len(l[3]) for l in loops)
        nprm = sum(len(l[4]) for l in loops)
        self.specs = (LoopSpec * max(n, 1))()
        self.args = (Arg * max(nargs, 1))()
        self.cparams = (ctypes.c_double * max(nprm, 1))()
        self.first_param = []
        ka = kp = 0
        for i, (op, blk, rng, args, params) in enumerate(loops):
            sp = self.specs[i]
            sp.op = OPS[op] if isinstance(op, str) else int(op)
            sp.block = int(blk)
            for k, v in enumerate(rng):
                sp.range[k] = int(v)
            sp.first_arg, sp.nargs = ka, len(args)
            for a in args:
                if a[0] == "red":
                    self.args[ka] = Arg(TC_ARG_RED, int(a[1]), 0, 0)
                else:
                    acc = ACCESS[a[2]] if isinstance(a[2], str) else int(a[2])
                    self.args[ka] = Arg(TC_ARG_DAT, int(a[0]), int(a[1]), acc)
                ka += 1
            sp.first_param, sp.nparams = kp, len(params)
            self.first_param.append(kp)
            for v in params:
                self.cparams[kp] = float(v)
                kp += 1
        self.n = n
        self.params = np.ctypeslib.as_array(self.cparams)

    def record(self):
        done = ctypes.c_int32()
        self.ctx._ck(lib().tc_par_loops(self.ctx.ptr, self.n, self.specs, self.args, self.cparams,
                                        ctypes.byref(done)), "tc_par_loops")


class Batch:
    """A batch engine (``tc_batch*``) on a context: batched and served
    heat-conduction solves."""

    def __init__(self, ctx: Context, mixed: bool = False, max_instances: int = 64, max_cells: int = 1 << 22,
                 hbm_budget: int = 8 << 30, cheb_steps: int = 10, replays_per_step: int = 4, inner_tol: float = 1e-4):
        self.ctx = ctx
        o = BatchOpts(int(mixed), int(max_instances), int(max_cells), int(hbm_budget), int(cheb_steps),
                      int(replays_per_step), float(inner_tol))
        self.ptr = ctypes.c_void_p()
        ctx._ck(lib().tc_batch_create(ctx.ptr, ctypes.byref(o), ctypes.byref(self.ptr)), "tc_batch_create")
        self.sizes: Dict[int, tuple] = {}

    def tc_batch_submit(self, ndim: int, n: int, seed: int, tol: float = 1e-8, max_iter: int = 10000,
                        max_outer: int = 50, dt: float = 0.004, keep_x: bool = False) -> int:
        d = SolveDesc(int(ndim), int(n), int(seed) & ((1 << 64) - 1), float(tol), int(max_iter), int(max_outer),
                      float(dt), int(keep_x), 0)
        t = ctypes.c_int64()
        self.ctx._ck(lib().tc_batch_submit(self.ptr, ctypes.byref(d), ctypes.byref(t)), "tc_batch_submit")
        self.sizes[t.value] = (ndim, n)
        return t.value

    def tc_batch_step(self) -> int:
        left = ctypes.c_int32()
        self.ctx._ck(lib().tc_batch_step(self.ptr, ctypes.byref(left)), "tc_batch_step")
        return left.value

    def tc_batch_poll(self, ticket: int) -> dict:
        r = SolveResult()
        self.ctx._ck(lib().tc_batch_poll(self.ptr, int(ticket), ctypes.byref(r)), "tc_batch_poll")
        return r.as_dict()

    def tc_batch_wait(self):
        self.ctx._ck(lib().tc_batch_wait(self.ptr), "tc_batch_wait")

    def tc_batch_read_x(self, ticket: int) -> np.ndarray:
        ndim, n = self.sizes[ticket]
        out = np.empty([n] * ndim, dtype=np.float64)
        self.ctx._ck(lib().tc_batch_read_x(self.ptr, int(ticket), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            out.size), "tc_batch_read_x")
        return out

    def close(self):
        if self.ptr:
            lib().tc_batch_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def tc_status_string(status: int) -> str:
    return lib().tc_status_string(status).decode()
