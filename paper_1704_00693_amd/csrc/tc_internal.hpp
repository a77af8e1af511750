// Internal types of the tilechain library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "tilechain.h"

namespace tc {

constexpr int kMaxArgs = 12;     // dataset + reduction arguments of one loop
constexpr int kMaxPts = 96;      // stencil points over all dataset arguments of one loop
constexpr int kMaxParams = 64;   // scalar parameters of one loop
constexpr int kMaxHalo = 16;
constexpr int kXAlign = 16;      // x origin and row pitch aligned to 16 elements

struct Block {
    int ndim;
    std::string name;
};

struct Stencil {
    int ndim;
    std::vector<int> pts;  // npoints * 3 (x, y, z), unused dims 0
    int lo[3], hi[3];      // min / max offset per dimension
    std::string name;
    int npoints() const { return (int)pts.size() / 3; }
    bool centre_only() const {
        for (int v : pts)
            if (v != 0) return false;
        return npoints() >= 1;
    }
};

struct Dataset {
    int block;
    tc_dtype dtype;
    int ndim;
    int size[3];
    int hneg[3], hpos[3];
    // padded device layout: x origin at column xorg of a row of `pitch`
    // elements; rows of ny_alloc per plane
    int64_t pitch, ny_alloc, nz_alloc, xorg;
    int64_t bytes;
    void *buf[2] = {nullptr, nullptr};
    void *raw[2] = {nullptr, nullptr};  // allocations (buf = raw + stagger)
    int64_t stagger = 0;                // byte offset of buf in raw
    int cur = 0;               // buffer holding the current values
    bool twin_synced = false;  // buf[1-cur] equals buf[cur] outside the written hull
    // hull of every point written by any loop so far (logical coords)
    int wlo[3], whi[3];
    bool ever_written = false;
    std::string name;

    size_t esize() const { return dtype == TC_F64 ? 8 : 4; }
    int64_t origin_offset() const {  // element offset of logical (0,0,0) in a buffer
        return (int64_t)hneg[2] * ny_alloc * pitch + (int64_t)hneg[1] * pitch + xorg;
    }
    int64_t sy() const { return pitch; }
    int64_t sz() const { return pitch * ny_alloc; }
    void *origin(int which) const {  // NULL while the buffer does not exist (host-only contexts)
        return buf[which] ? (char *)buf[which] + origin_offset() * (int64_t)esize() : nullptr;
    }
};

struct Reduction {
    tc_redop op;
    std::string name;
    // host accumulator (double-double for sums)
    double hi = 0.0, lo = 0.0;
    bool touched = false;
};

struct ArgRec {
    int kind;
    int handle;
    int stencil;
    int access;
    bool reads() const { return kind == TC_ARG_DAT && (access == TC_READ || access == TC_RW || access == TC_INC); }
    bool writes() const { return kind == TC_ARG_DAT && (access == TC_WRITE || access == TC_RW || access == TC_INC); }
};

struct LoopRec {
    int op;
    int block;
    int ndim;
    int lo[3], hi[3];  // unused dims: [0,1)
    std::vector<ArgRec> args;
    std::vector<double> params;
    std::string name;
    int64_t points() const {
        int64_t n = 1;
        for (int d = 0; d < 3; ++d) n *= (hi[d] > lo[d]) ? (hi[d] - lo[d]) : 0;
        return n;
    }
};

// ---------------------------------------------------------------------------
// Device-side descriptors (passed by value as kernel arguments)
// ---------------------------------------------------------------------------
struct DArg {
    void *ptr;   // logical (0,0,0) of the buffer to use
    int64_t sy;  // element stride of y
    int64_t sz;  // element stride of z
};

struct LoopDesc {
    int op;
    int ndim;
    int nargs;       // dataset arguments (reductions are not listed here)
    int npts[kMaxArgs];
    int pt0[kMaxArgs];  // first stencil point of each argument in off[]
    DArg arg[kMaxArgs];
    int64_t off[kMaxPts];  // linear element offset of every stencil point
    unsigned char qarg[kMaxPts];  // dataset argument of every stencil point
    double prm[kMaxPts > kMaxParams ? kMaxPts : kMaxParams];  // WSUM: weight of stencil point i at prm[i] (aligned with off[])
    int nred;            // reduction arguments (0..2)
    int red_op[2];
    double *partials[2];  // per-block (hi, lo) partial results, indexed from part_base
};

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------
struct SkewedPlan {
    int ndim = 0;
    int num_tiles[3] = {1, 1, 1};
    // start/end[d][t][l]
    std::vector<int> start[3], end[3];
    int nloops = 0;
    int s(int d, int t, int l) const { return start[d][(size_t)t * nloops + l]; }
    int e(int d, int t, int l) const { return end[d][(size_t)t * nloops + l]; }
};

struct FusedGroup;  // defined in fused.hpp

// One kernel launch of a per-loop schedule: loop index, box, and where its
// workgroups write reduction partials (in units of (hi, lo) pairs).
struct Launch {
    int loop;
    int lo[3], hi[3];
    int nb;
    int64_t part_off[2];
};

// One step of a schedule: a per-loop launch or a fused group.
struct Step {
    int kind;   // 0: launches[index], 1: groups[index]
    int index;
};

struct CachedPlan {
    tc_tiling mode;
    SkewedPlan skewed;
    std::vector<Step> steps;
    std::vector<Launch> launches;
    std::vector<int> red_handles;      // reductions used by the chain, slot order
    std::vector<int64_t> red_base;     // first partial of each slot
    std::vector<int64_t> red_count;    // partials of each slot
    int64_t partials_total = 0;
    std::vector<std::shared_ptr<FusedGroup>> groups;  // fused mode
    double build_seconds = 0.0;
    int max_skew[3] = {0, 0, 0};
    // per-loop schedules replayed as a HIP graph once the same launch
    // arguments have been seen on two consecutive flushes
    hipGraphExec_t gexec = nullptr;
    uint64_t ghash = 0, ghash_prev = 0;
};

// One schedule the autotuner can pick: mode, tile (as for tc_set_tiling) and,
// for fused groups, the columns each lane holds (1 or 2).
struct TuneCand {
    tc_tiling mode;
    int tile[3];
    int cpl;
};

// Workgroup shapes of the register-window (marching) kernels: in 2D, rows
// per workgroup (TC_MARCH_TY); in 3D, rows per workgroup, one wavefront each
// (TC_MARCH3_ROWS: 4 or 8), and planes each workgroup marches
// (TC_MARCH3_TZ); 0: chosen by the launcher from the box.
struct MarchShape {
    int ty = 8;
    int rows3 = 0;
    int tz3 = 0;
};

struct Ctx {
    int device = 0;
    bool host_only = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    tc_alloc_fn alloc = nullptr;
    tc_free_fn free = nullptr;
    void *alloc_user = nullptr;
    bool poisoned = false;
    std::string last_error;

    std::vector<Block> blocks;
    std::vector<Dataset> dats;
    std::vector<Stencil> stencils;
    std::vector<Reduction> reds;
    std::vector<LoopRec> chain;

    tc_tiling mode = TC_TILING_NONE;
    int tile[3] = {0, 0, 0};

    std::unordered_map<uint64_t, std::shared_ptr<CachedPlan>> plans;
    // AUTO mode: per chain structure, the candidates tried so far, their
    // measured device times and the choice once every candidate has run
    struct Tune {
        int next = 0;
        int warm = 0;  // untimed flushes of candidate `next` so far
        int best = -1;
        std::vector<std::vector<double>> samples;  // timed flushes per candidate
        std::vector<double> seconds;               // median per finished candidate
    };
    std::unordered_map<uint64_t, Tune> tuned;
    std::unordered_map<uint64_t, TuneCand> tune_saved;  // choices read from / written to TC_TUNE_CACHE
    bool tune_cache_loaded = false;
    int tune_cand = -1;          // candidate being timed by the current flush
    uint64_t tune_key = 0;
    hipEvent_t tune_ev[2] = {nullptr, nullptr};

    // reduction partials (device) and host staging
    double *partials = nullptr;
    int64_t partials_cap = 0;  // in doubles
    double *red_out = nullptr;  // device: 2 doubles per reduction
    int64_t red_out_cap = 0;
    double *red_host = nullptr;      // pinned, coherent host memory: the flush's reduction results
    double *red_host_dev = nullptr;  // its device address (the combining kernel writes it directly)

    tc_stats stats{};

    // weighted-sum loops on canonical 2D star stencils use the register-window
    // kernel (TC_WSUM_MARCH=0 in the environment selects the generic kernel)
    bool march_enabled = true;
    MarchShape march;             // workgroup shapes of the register-window kernels
    int64_t stagger_unit = 0;     // dataset i's base is offset by (i % 16) * stagger_unit bytes

    bool use_graphs = true;              // TC_GRAPHS=0 disables graph replay
    hipStream_t cap_stream = nullptr;    // private stream used only for graph capture

    // fused groups: generated kernels compiled at plan time, cached by source
    std::unordered_map<uint64_t, hipModule_t> jit_modules;
    int jit_unroll = 3;      // steps per iteration of the generated march loop (TC_JIT_UNROLL)
    int jit_prefetch = 1;    // rows loaded ahead of their arrival step (TC_JIT_PREFETCH)
    int jit_edge_div = 4;  // TC_JIT_EDGE_DIV: edge wavefronts march Hseg / this many rows
    int jit_wpe = 2;         // wavefronts per SIMD asked of the interior fused kernels (TC_JIT_WPE, 0: compiler's choice)
    int jit_max_window = 0;  // split the readers of a loaded dataset above this window (TC_JIT_MAXWIN, 0: never)
    bool jit_cse_steps = true;  // TC_JIT_CSE=0: shifted values recomputed per loop
    bool jit_sched_fence = false;  // TC_JIT_FENCE=1: scheduling barrier between loops
    bool jit_align_store = true;   // TC_JIT_ALIGN=0: owned strips of any width (else whole 128-byte lines)
    int jit_cpl = 1;         // consecutive columns per lane in fused kernels (TC_JIT_CPL: 1 or 2)
    bool jit_test_short_windows = false;  // TC_JIT_TEST_SHORT_WINDOWS=1: fault injection for error-path tests
    bool jit_bake = true;    // compile the weights into the kernels (TC_JIT_BAKE=0: read them from arguments)
    // staged groups (overlapped tiles in LDS for loops of any op and range):
    // TC_STAGED=0 disables them, TC_STAGED=2 takes every one the analysis
    // accepts whatever the cost model says, TC_STAGED_TILE=x,y,z fixes the
    // owned box
    int staged_mode = 1;
    bool cheb_enabled = true;  // TC_CHEB=0: no fused Chebyshev-step groups
    int cheb_steps = 0;        // TC_CHEB_STEPS=k: Chebyshev groups of exactly k steps (or a run's shorter rest)
    int staged_threads = 0;  // TC_STAGED_THREADS=256|1024: workgroup size of staged tiles (0: by box size)
    int staged_tile[3] = {0, 0, 0};
    std::vector<void *> staged_allocs;  // device tables of staged groups (freed at finalize)
    double jit_compile_seconds = 0.0;

    // calls that must not allocate device memory (tc_reduction_result_static):
    // while set, reduction partials and outputs live in the library's static
    // device scratch array, graphs and profiling are off, and any path that
    // would allocate, compile or load code fails with TC_ERR_STATE instead
    bool noalloc = false;
    double *scratch = nullptr;  // device address of this device's scratch array

    // per-launch kernel timing (tc_set_profiling)
    bool profiling = false;
    std::vector<hipEvent_t> events;
};

// No C++ exception crosses the C ABI: every exported call runs its body
// through this guard, which turns std::bad_alloc into TC_ERR_NOMEM and any
// other exception into TC_ERR_STATE, keeping the text as the context's last
// error (when there is a context).
inline void note_abi_error(Ctx *c, const char *msg) noexcept {
    if (!c) return;
    try {
        c->last_error = msg;
    } catch (...) {
    }
}

template <class F>
tc_status guard_abi(Ctx *c, F &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        note_abi_error(c, "host memory allocation failed");
        return TC_ERR_NOMEM;
    } catch (const std::exception &e) {
        note_abi_error(c, e.what());
        return TC_ERR_STATE;
    } catch (...) {
        note_abi_error(c, "internal error");
        return TC_ERR_STATE;
    }
}

// plan.cpp
SkewedPlan build_skewed_plan(const Ctx &c, const std::vector<LoopRec> &chain, const int tile[3]);
uint64_t chain_key(const Ctx &c, const std::vector<LoopRec> &chain, int mode, const int tile[3], int cpl);

}  // namespace tc

// The C ABI's context object.
struct tc_ctx {
    tc::Ctx c;
};
