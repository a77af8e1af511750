/*
 * tilechain -- run-time tiling of chains of stencil loops on AMD Instinct
 * MI355X (gfx950).
 *
 * C ABI of the library.  It follows the problem statement of Reguly, Mudalige
 * and Giles, "Loop Tiling in Large-Scale Stencil Codes at Run-time with OPS":
 *
 *   - Section 3: a computation is a sequence of parallel loops over an
 *     iteration range of a block; each loop applies a point kernel and names
 *     its datasets, each with a stencil and an access mode (read, write,
 *     read-write, increment).  Point order within a loop is irrelevant.
 *   - Section 4.1: loops are not executed when they are issued; they are
 *     recorded, and the recorded chain runs when the user needs data back
 *     (a reduction result, or a dataset).
 *   - Section 4.2: at that point the chain is analysed and executed tile by
 *     tile (skewed tiling, Algorithms 1 and 2); the plan is cached and reused
 *     when the same sequence of loops recurs.
 *   - Section 4.4: overlapped tiling (tiles recompute the points they need
 *     from their neighbours and run concurrently, read dependencies only).
 *
 * Conventions
 *   - Every call returns tc_status: TC_OK (0) or a negative error code.  No
 *     call aborts or throws across the ABI.  tc_last_error() gives the text
 *     of the last error of a context.
 *   - After a device (HIP) failure the context is poisoned: every later call
 *     on it returns TC_ERR_DEVICE until tc_finalize().
 *   - Handles (blocks, datasets, stencils, reductions) are small integers
 *     owned by their context; they stay valid until tc_finalize().
 *   - Coordinates are logical: dataset point (x, y, z) with 0 <= x < size[0]
 *     is an interior point, negative or >= size coordinates are halo points.
 *     x is the fastest-varying dimension.  Ranges are half-open [lo, hi).
 *   - A context is used from one host thread at a time.
 */
#ifndef TILECHAIN_H
#define TILECHAIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tc_status;
enum {
    TC_OK = 0,
    TC_ERR_ARG = -1,         /* invalid argument (bad handle, size, range, access) */
    TC_ERR_STATE = -2,       /* call not allowed in this state (e.g. host-only context) */
    TC_ERR_DEVICE = -3,      /* a HIP call failed; the context is poisoned */
    TC_ERR_NOMEM = -4,       /* device or host allocation failed */
    TC_ERR_UNSUPPORTED = -5, /* valid request the library does not implement */
    TC_ERR_RANGE = -6        /* iteration range plus stencil leaves the allocated halo */
};

typedef struct tc_ctx tc_ctx;
typedef int32_t tc_block;
typedef int32_t tc_dat;
typedef int32_t tc_stencil;
typedef int32_t tc_red;

/* Every enum below also holds TC_ENUM_MIN_ and TC_ENUM_MAX_, which name no
 * value: they give the type the whole int32 range, so a caller may pass any
 * int32 (calls reject values outside the listed ones with TC_ERR_ARG). */
#define TC_ENUM_MIN_ (-0x7fffffff - 1)
#define TC_ENUM_MAX_ 0x7fffffff

typedef enum { TC_F64 = 0, TC_F32 = 1, TC_DTYPE_MIN_ = TC_ENUM_MIN_, TC_DTYPE_MAX_ = TC_ENUM_MAX_ } tc_dtype;
typedef enum { TC_READ = 0, TC_WRITE = 1, TC_RW = 2, TC_INC = 3, TC_ACCESS_MIN_ = TC_ENUM_MIN_, TC_ACCESS_MAX_ = TC_ENUM_MAX_ } tc_access;
typedef enum { TC_ARG_DAT = 0, TC_ARG_RED = 1, TC_ARGKIND_MIN_ = TC_ENUM_MIN_, TC_ARGKIND_MAX_ = TC_ENUM_MAX_ } tc_argkind;
typedef enum { TC_RED_SUM = 0, TC_RED_MIN = 1, TC_RED_MAX = 2, TC_REDOP_MIN_ = TC_ENUM_MIN_, TC_REDOP_MAX_ = TC_ENUM_MAX_ } tc_redop;

/* Tiling of a flushed chain.
 *   NONE       : every loop runs over its whole range, one kernel per loop.
 *   SKEWED     : Algorithm 1 plan; tiles run in order, each (tile, loop) is a
 *                whole-GPU sweep of the tile's range (Algorithm 2).
 *   FUSED      : overlapped tiles (Section 4.4 applied per workgroup); each
 *                workgroup streams its tile through the chain with the
 *                working set in LDS; one kernel per fusion group.
 *   AUTO       : the autotuner measures the candidates once per chain
 *                structure and keeps the fastest. */
typedef enum {
    TC_TILING_NONE = 0,
    TC_TILING_SKEWED = 1,
    TC_TILING_FUSED = 2,
    TC_TILING_AUTO = 3,
    TC_TILING_MIN_ = TC_ENUM_MIN_,
    TC_TILING_MAX_ = TC_ENUM_MAX_
} tc_tiling;

/* Point operations (closed vocabulary).  Argument lists are positional; the
 * accesses and stencils given at tc_par_loop must match the signature.
 * Arithmetic is FP64 for F64 datasets and FP32 for F32 datasets; reductions
 * always accumulate in FP64 (double-double for sums).
 *
 *  TC_OP_WSUM        args: out(W), in_1..in_k(R, any stencil)   params: one weight per (input, stencil point)
 *                    out = sum over inputs, stencil points (listed order) of w * in[x+q], as acc = fma(w, v, acc) from 0
 *  TC_OP_COPY        args: out(W), in(R centre)                  out = in (also converts F64 <-> F32)
 *  TC_OP_AXPBY       args: y(RW), x(R centre)          params a,b y = fma(a, x, b*y)
 *  TC_OP_DOT         args: a(R), b(R), red(SUM)                  red += a*b
 *  TC_OP_SUM         args: a(R), red(SUM)                        red += a
 *  TC_OP_HALO_REFLECT args: v(RW, stencil covering the source offsets)  params axis, side, n
 *                    ghost c (outside [0,n) along axis) takes v at -1-c (side 0) or 2n-1-c (side 1)
 *  Heat conduction (2D/3D, K_d = face coefficient on the cell's low face along d):
 *  TC_OP_TEA_INIT    args: rho(R), e(R), u0(W), u(W)             u0 = u = e*rho
 *  TC_OP_TEA_K       args: rho(R: centre, -x, -y[, -z]), Kx(W), Ky(W)[, Kz(W)]   params r
 *                    K_d = (2r) / (rho(c - e_d) + rho(c))
 *  TC_OP_TEA_RESID   args: Kx, Ky[, Kz](R: centre, +e_d), x(R star), b(R), r(W)   r = b - A x
 *  TC_OP_TEA_MATVEC_DOT args: K..(R), p(R star), w(W), red(SUM)  w = A p; red += p*w
 *  TC_OP_TEA_P1      args: K..(R), sd(R star), rt(RW), z(RW)      rt = rt - A sd; z = z + sd
 *  TC_OP_TEA_P2      args: sd(RW), rt(R)              params alpha, beta   sd = fma(alpha, sd, beta*rt)
 *  TC_OP_TEA_PRECON_INIT args: r(R), rt(W), sd(W), z(W) params theta   rt = r; sd = r/theta; z = 0
 *  TC_OP_TEA_CG_UPDATE args: x(RW), r(RW), p(R), w(R) params alpha   x = fma(alpha,p,x); r = fma(-alpha,w,r)
 *  TC_OP_TEA_CG_P    args: p(RW), z(R)                params beta    p = fma(beta, p, z)
 *  TC_OP_TEA_GERSH   args: K..(R: centre, +e_d), red(MAX)         red = max(red, fma(2, sum of face K, 1))
 *
 * Compressible Euler (stand-in for the OpenSBLI Taylor-Green runs of Section 5
 * and Section 6.4; D = block dimension, Q = (rho, rho u_1..rho u_D, E)):
 *  TC_OP_EULER_PRIM  args: Q_0..Q_{D+1}(R), u_1..u_D(W), p(W)   params gm1 = gamma - 1
 *                    ri = 1/rho; u_d = (rho u_d) ri; k = (rho u_D) u_D, then
 *                    k = fma(rho u_d, u_d, k) for d = D-1..1; p = gm1 * fma(-0.5, k, E)
 *  TC_OP_EULER_RHS   args: R(W), Q_c(R: +-2 along every axis), u_1..u_D(R: same), p(R: same)
 *                    params c (component), s = 1/(12h).  Flux along axis d at a point:
 *                    f = Q_c u_d; f = f + p if c == d; f = fma(p, u_d, f) if c == D+1.
 *                    Per axis (in order) g_d = 8 (f(+1) - f(-1)) - (f(+2) - f(-2)),
 *                    acc = g_1 (+ g_2 (+ g_3)); R = -acc * s
 *  TC_OP_RK_STAGE    args: Q0(R), Q(RW), R(R)   params a, b, dt   t = fma(dt, R, Q); Q = fma(a, Q0, b t)
 *  where (A v) = diag*v - K_E v_E - K_W v_W - K_N v_N - K_S v_S [- K_T v_T - K_B v_B],
 *  diag = 1 + K_E + K_W + K_N + K_S [+ K_T + K_B] summed left to right, the
 *  off-diagonal terms applied with fma in the order E, W, N, S[, T, B].
 */
typedef enum {
    TC_OP_WSUM = 0,
    TC_OP_COPY = 1,
    TC_OP_AXPBY = 2,
    TC_OP_DOT = 3,
    TC_OP_SUM = 4,
    TC_OP_HALO_REFLECT = 5,
    TC_OP_TEA_INIT = 10,
    TC_OP_TEA_K = 11,
    TC_OP_TEA_RESID = 12,
    TC_OP_TEA_MATVEC_DOT = 13,
    TC_OP_TEA_P1 = 14,
    TC_OP_TEA_P2 = 15,
    TC_OP_TEA_PRECON_INIT = 16,
    TC_OP_TEA_CG_UPDATE = 17,
    TC_OP_TEA_CG_P = 18,
    TC_OP_TEA_GERSH = 19,
    TC_OP_EULER_PRIM = 20,
    TC_OP_EULER_RHS = 21,
    TC_OP_RK_STAGE = 22,
    TC_OP_MIN_ = TC_ENUM_MIN_,
    TC_OP_MAX_ = TC_ENUM_MAX_
} tc_op;

/* One loop argument: a dataset through a stencil with an access mode, or a
 * reduction handle (kind TC_ARG_RED; stencil and access are ignored). */
typedef struct {
    int32_t kind;    /* tc_argkind */
    int32_t handle;  /* tc_dat or tc_red */
    int32_t stencil; /* tc_stencil (datasets) */
    int32_t access;  /* tc_access (datasets) */
} tc_arg;

/* Device memory callbacks.  alloc returns device memory of at least `bytes`
 * bytes (256-byte aligned) or NULL; free releases it.  NULL callbacks mean
 * hipMalloc / hipFree. */
typedef void *(*tc_alloc_fn)(size_t bytes, void *user);
typedef void (*tc_free_fn)(void *ptr, void *user);

enum {
    TC_INIT_HOST_ONLY = 1,    /* record and analyse only; no device, flush fails */
    TC_INIT_BORROW_STREAM = 2 /* run on opts.stream even when it is NULL (the null stream) */
};

typedef struct {
    int32_t device;   /* HIP device ordinal */
    int32_t flags;    /* TC_INIT_* */
    void *stream;     /* hipStream_t to run on (borrowed); NULL without TC_INIT_BORROW_STREAM:
                         the library creates its own stream */
    tc_alloc_fn alloc;
    tc_free_fn free;
    void *alloc_user;
} tc_init_opts;

/* Create a context.  opts may be NULL (device 0, own stream, hipMalloc). */
tc_status tc_init(const tc_init_opts *opts, tc_ctx **out);

/* Flush the pending chain, release all device memory the library owns, free
 * the context.  Safe on a poisoned context.  ctx may be NULL. */
tc_status tc_finalize(tc_ctx *ctx);

/* Declare a structured block of dimension 1..3 (Section 3: blocks). */
tc_status tc_decl_block(tc_ctx *ctx, int ndim, const char *name, tc_block *out);

/* Declare a dataset on a block (Section 3: datasets, Section 3: ownership of
 * data is handed to the library).  size[d] interior points, halo_neg[d] /
 * halo_pos[d] halo depths per side (0..16).  host_init: NULL (zero fill) or
 * the initial values of the whole padded array INCLUDING halos, packed with x
 * fastest: dims (size[d] + halo_neg[d] + halo_pos[d]).  The buffer is copied
 * before the call returns and is not retained.  Device storage is allocated
 * here (plus, lazily, a second buffer used by fused execution). */
tc_status tc_decl_dat(tc_ctx *ctx, tc_block blk, tc_dtype dtype, const int32_t *size,
                      const int32_t *halo_neg, const int32_t *halo_pos, const void *host_init,
                      const char *name, tc_dat *out);

/* Declare a stencil: npoints offsets of ndim ints each (x first). */
tc_status tc_decl_stencil(tc_ctx *ctx, int ndim, int npoints, const int32_t *offsets,
                          const char *name, tc_stencil *out);

/* Declare a global reduction (Section 4.1: fetching its result flushes). */
tc_status tc_decl_reduction(tc_ctx *ctx, tc_redop op, const char *name, tc_red *out);

/* Record a parallel loop (Section 3; delayed, Section 4.1).  range has 2*ndim
 * ints: lo[0], hi[0], lo[1], hi[1], ...  The call validates, deep-copies the
 * arguments and parameters and returns; nothing runs.  On error the chain is
 * unchanged.  Rejected: block or dimension mismatch; range plus stencil
 * outside a dataset's allocated halo (TC_ERR_RANGE); a write with a stencil
 * other than the centre; a dataset read at an offset and written in the same
 * loop (except TC_OP_HALO_REFLECT, whose reads and writes are disjoint);
 * arguments or parameter count not matching the op's signature. */
tc_status tc_par_loop(tc_ctx *ctx, const char *name, tc_op op, tc_block blk, const int32_t *range,
                      const tc_arg *args, int nargs, const double *params, int nparams);

/* Record n loops in one call: the same as n calls of tc_par_loop in order
 * (each validated and copied; nothing runs).  Loop i takes its arguments
 * from args[loops[i].first_arg ..] and its parameters from
 * params[loops[i].first_param ..]; loops get empty names.  Stops at the first
 * loop rejected and returns its status: the loops before it stay recorded and
 * *recorded (may be NULL) gives their number.  For callers that record the
 * same loops every iteration (one call per chain instead of one per loop). */
typedef struct {
    int32_t op;      /* tc_op */
    int32_t block;
    int32_t range[6];  /* as tc_par_loop: lo[0], hi[0], lo[1], hi[1], ... (first 2*ndim used) */
    int32_t first_arg, nargs;
    int32_t first_param, nparams;
} tc_loop;
tc_status tc_par_loops(tc_ctx *ctx, int32_t n, const tc_loop *loops, const tc_arg *args, const double *params,
                       int32_t *recorded);

/* Flush the chain (Section 4.1), then return the reduction's value (as
 * double) and reset it to its identity.  A reduction accumulates over every
 * loop that used it since its previous fetch. */
tc_status tc_reduction_result(tc_ctx *ctx, tc_red red, double *out);

/* Execute the pending chain now. */
tc_status tc_flush(tc_ctx *ctx);

/* tc_reduction_result for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same flush and result as tc_reduction_result, but the call
 * allocates nothing: its reduction partials and finalised results live in a
 * static device array of the library (1 MiB, 131072 doubles per device, held
 * until the process ends), no graph is captured or replayed, no kernel is
 * compiled or loaded and profiling is off for the call.
 *   - The chain's reductions may need at most 131072 doubles: two per
 *     workgroup of every reduction loop plus two per reduction handle;
 *     otherwise TC_ERR_ARG (nothing runs, the chain stays pending).
 *   - A chain structure whose schedule needs a compiled fused plan, an
 *     undecided autotuner choice or a not yet allocated second buffer must
 *     first be flushed once with tc_flush or tc_reduction_result; otherwise
 *     TC_ERR_STATE (nothing runs, the chain stays pending).
 *   - Every call on one device shares that device's array and leaves the last
 *     call's values in it: calls that overlap on one device (from any context
 *     or thread) race. */
tc_status tc_reduction_result_static(tc_ctx *ctx, tc_red red, double *out);

/* Flush, then copy a dataset to / from host memory.  The host layout is the
 * padded array with halos, packed, x fastest (as in tc_decl_dat). */
tc_status tc_dat_read(tc_ctx *ctx, tc_dat dat, void *host);
tc_status tc_dat_write(tc_ctx *ctx, tc_dat dat, const void *host);

/* Flush, then return the device address of logical point (0,0,0) of the
 * dataset's current buffer and its element strides (x stride is 1).  Valid
 * until the next flush. */
tc_status tc_dat_device_view(tc_ctx *ctx, tc_dat dat, void **origin, int64_t strides[3]);

/* Choose how the following flushes are tiled (Section 4.3: manual tile sizes
 * or automatic choice).  tile[d] <= 0 means "choose automatically" for that
 * dimension (skewed: the whole extent along x, a cache-sized height along the
 * slowest dimension).  For TC_TILING_FUSED (Section 4.4, overlapped tiles
 * fused per wavefront): tile[0] is the number of rows one wavefront streams
 * (its segment), tile[1] the budget of register-window words per lane that
 * bounds a fusion group, tile[2] the most loops in one group; 0 chooses
 * automatically.  Fused groups are generated and compiled (hipRTC) when a
 * chain structure is first planned. */
tc_status tc_set_tiling(tc_ctx *ctx, tc_tiling mode, const int32_t *tile);

typedef struct {
    int64_t loops_recorded;
    int64_t flushes;
    int64_t plan_hits;
    int64_t plan_misses;
    double plan_seconds;        /* total host time spent building plans */
    int32_t max_skew[3];        /* largest tile-boundary skew of the last plan (Section 6 skew report) */
    int32_t last_tiles;         /* tiles (skewed) or workgroups (fused) of the last flush */
    int32_t last_groups;        /* fusion groups of the last flush */
    int32_t last_launches;      /* kernel launches of the last flush */
    int32_t last_mode;          /* tc_tiling actually used by the last flush */
    int64_t modelled_bytes;     /* bytes of the last flush under the per-loop model:
                                   range points x element size x (1 for R or W, 2 for RW/INC) */
    int64_t cell_updates;       /* sum of loop range sizes of the last flush */
    double last_flush_seconds;  /* host wall time of the last flush, including the final sync */
    /* kernel timing of the last flush (only with tc_set_profiling on): sum of
       the device durations of its kernels, measured with HIP events recorded
       on the library's stream around every launch, and the number of launches
       timed; the main kernels only (reduction finalisation excluded) */
    double prof_kernel_seconds;
    int64_t prof_launches;
    /* fused groups of the last flush: their algorithmic HBM bytes (every
       dataset whose chain-start value a group reads, plus every dataset it
       writes, once over the group's range) and, with profiling on, the
       device time of their kernels */
    int64_t fused_bytes;
    double prof_fused_seconds;
    double jit_compile_seconds; /* total host time spent compiling fused kernels */
    int32_t last_tile[3];       /* tile used by the last flush (the autotuner's pick under AUTO) */
    int32_t last_cpl;           /* columns per lane of the last flush's fused kernels (1 or 2) */
    int32_t tuning;             /* 1 if the last flush was one of the autotuner's measurement
                                   flushes (its chain structure has no choice yet), else 0 */
    int32_t pad;
} tc_stats;

tc_status tc_get_stats(tc_ctx *ctx, tc_stats *out);

/* Turn per-launch kernel timing on (1) or off (0).  Timing records two HIP
 * events around every kernel launch and synchronises at the end of each
 * flush, so it is for measurement runs, not production. */
tc_status tc_set_profiling(tc_ctx *ctx, int on);

/* Analyse the pending chain without running it (works on host-only
 * contexts); the chain stays pending.  cap is the number of int32 slots of
 * ranges.  Returns TC_ERR_ARG if cap is too small (num_tiles is still
 * written, so a first call with ranges = NULL sizes the buffer).
 *
 * TC_TILING_SKEWED (Algorithm 1): num_tiles[d] tiles per dimension and, for
 * every tile index t_d of every dimension d and every loop l, the pair
 * (start, end) at ranges[((d * max_tiles + t_d) * nloops + l) * 2 + {0,1}],
 * max_tiles the largest num_tiles[d].
 *
 * TC_TILING_FUSED (Section 4.4, overlapped tiles fused per group):
 * num_tiles[0] = G fusion groups, num_tiles[1] = L loops in the chain,
 * num_tiles[2] = 0; needs 2 G + 7 L slots.  ranges[2 g], ranges[2 g + 1] are
 * the first and one-past-last chain loop of group g.  Then seven ints per
 * chain loop l at ranges[2 G + 7 l + k]: k = 0 is 1 if a register-window
 * group computes the loop, 2 if a staged group does (LDS-staged tiles, any
 * op and range), 3 if a fused 3D Runge-Kutta stage does (the five
 * EULER_RHS loops and the five RK_STAGE loops of a stage in one z-marching
 * kernel; no recomputed overlap), 0 if the loop is in a group but never computed (its result
 * is neither read later in the group nor the final value of its dataset),
 * -1 if it runs on its own; k = 1..6 are the points below and above the
 * owned block along x, y and z that the loop computes (the recomputed
 * overlap; register-window groups: a wavefront's owned block, z entries 0;
 * staged groups: the most interior tile's owned box; 0 unless computed).
 * Register-window kernels are generated and compiled (hipRTC) by this call;
 * generation errors are returned as TC_ERR_STATE. */
tc_status tc_chain_plan(tc_ctx *ctx, tc_tiling mode, const int32_t *tile, int32_t *num_tiles,
                        int32_t *ranges, int64_t cap);

/* Staged tiles of one fusion group of the pending chain, as TC_TILING_FUSED
 * with `tile` would plan them (Section 4.4: every tile's owned box and the
 * box each loop of the group computes for it; works on host-only contexts;
 * the chain stays pending).  info (6 ints): first and one-past-last chain
 * loop of the group, the number of tiles T (0 if the group is a
 * register-window group, which has no tiles), and the owned box extents.
 * boxes (may be NULL to query info only): per tile, 6 + 6 L ints (L loops of
 * the group): the owned box lo[3], hi[3], then per loop its computed box
 * lo[3], hi[3] (empty when some hi <= lo); TC_ERR_ARG if cap is below
 * T (6 + 6 L) or group is not a group index. */
tc_status tc_staged_tiles(tc_ctx *ctx, const int32_t *tile, int32_t group, int32_t *info, int32_t *boxes, int64_t cap);

/* Number of loops currently recorded and not yet executed. */
tc_status tc_pending(tc_ctx *ctx, int32_t *nloops);

/* ---------------------------------------------------------------------------
 * Batched and served heat-conduction solves.
 *
 * Not in the paper: many independent implicit heat-conduction solves (the
 * TeaLeaf-style PPCG workload of Section 5 and Section 6.4, with the
 * operator, reflective boundaries, Gershgorin bound and Chebyshev
 * preconditioner of the library's TEA_* loops) advanced together on one
 * GPU.  Every solver phase is one kernel launch over all resident instances
 * (the Chebyshev steps run several per launch, with the same per-cell
 * arithmetic: for 2D instances on tiles with a recomputed border, for 3D
 * instances in a march up z-segments of their planes); the phases of one
 * iteration are captured once in a HIP graph and replayed.  The HBM
 * footprint of a solve is 10 + ndim field arrays of (n + 2)^ndim values
 * (FP64; mixed: 3 + ndim FP64 and 9 + ndim FP32 arrays), each rounded up to
 * 256 bytes.
 * Each instance keeps its state machine, scalars and convergence test on the
 * device; the host admits new solves into free slots by HBM footprint
 * (continuous batching), retires finished ones and rebuilds the tile list
 * between replays.
 *
 * Instance inputs are generated on the device from the seed: density
 * uniform [0.1, 1) for every interior cell (draw k + 1 of the SplitMix64
 * stream with state `seed`, cell k in row-major order, x fastest), then
 * energy uniform [1, 2) (draws cells + k + 1); dx = 1/n, rx = dt * n * n.
 * --------------------------------------------------------------------------- */
typedef struct tc_batch tc_batch;

typedef struct {
    int32_t mixed;            /* 0: FP64 sweeps; 1: FP32 sweeps with FP64 reductions inside FP64
                                 iterative refinement (x, b and the true residual in FP64) */
    int32_t max_instances;    /* resident solves at once (slots), >= 1 */
    int64_t max_cells;        /* cells of all resident solves at once (sizes the tile list) */
    int64_t hbm_budget;       /* bytes of instance fields resident at once; admission stops above it */
    int32_t cheb_steps;       /* Chebyshev steps per preconditioner application (0: 10) */
    int32_t replays_per_step; /* iterations replayed per tc_batch_step (0: 4) */
    double inner_tol;         /* mixed: relative drop of the FP32 residual per correction (0: 1e-4) */
} tc_batch_opts;

typedef struct {
    int32_t ndim;      /* 2 or 3 */
    int32_t n;         /* cells per axis, >= 2 */
    uint64_t seed;     /* instance input stream */
    double tol;        /* stop at ||r|| <= tol ||b|| (FP64 mode: recursive residual, then the true
                          residual is reported; mixed: true residual) */
    int32_t max_iter;  /* PPCG iteration cap (mixed: per correction) */
    int32_t max_outer; /* mixed: refinement steps cap */
    double dt;         /* time step (dx = 1/n) */
    int32_t keep_x;    /* keep the solution for tc_batch_read_x */
    int32_t pad;
} tc_solve_desc;

enum { TC_SOLVE_PENDING = 0, TC_SOLVE_RUNNING = 1, TC_SOLVE_DONE = 2, TC_SOLVE_REJECTED = -1 };

typedef struct {
    int32_t state;        /* TC_SOLVE_* */
    int32_t iterations;   /* PPCG iterations (mixed: summed over corrections) */
    int32_t outer;        /* mixed: refinement steps */
    int32_t converged;    /* true residual <= tol ||b|| */
    double rel_residual;  /* FP64 true residual ||b - A x|| / ||b|| */
    double bnorm;         /* ||b|| */
    double lmax;          /* Gershgorin bound used by the preconditioner */
    double seconds;       /* submission to completion (host clock) */
    double queue_seconds; /* submission to admission */
} tc_solve_result;

/* Create a batch engine on a context (its stream and allocator).  Device
 * arrays for max_instances slots and max_cells cells are allocated here. */
tc_status tc_batch_create(tc_ctx *ctx, const tc_batch_opts *opts, tc_batch **out);
/* Queue one solve; returns its ticket.  TC_ERR_ARG for a bad description. */
tc_status tc_batch_submit(tc_batch *b, const tc_solve_desc *desc, int64_t *ticket);
/* One scheduling round: wait for the previous replays, retire finished
 * solves, admit queued ones that fit, replay replays_per_step iterations.
 * *unfinished = solves queued or resident afterwards.  A solve that can never
 * fit (footprint above the budget or cells above max_cells) is rejected. */
tc_status tc_batch_step(tc_batch *b, int32_t *unfinished);
/* Result of a ticket (state TC_SOLVE_PENDING / RUNNING while unfinished). */
tc_status tc_batch_poll(tc_batch *b, int64_t ticket, tc_solve_result *out);
/* Step until every submitted solve has finished. */
tc_status tc_batch_wait(tc_batch *b);
/* Copy a finished solve's kept solution (n^ndim doubles, x fastest) to host
 * memory; cap is the number of doubles available.  TC_ERR_STATE if the solve
 * did not keep x or has not finished. */
tc_status tc_batch_read_x(tc_batch *b, int64_t ticket, double *host, int64_t cap);
/* Release the engine (resident solves are dropped). */
tc_status tc_batch_destroy(tc_batch *b);

const char *tc_status_string(tc_status s);
const char *tc_last_error(tc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* TILECHAIN_H */
