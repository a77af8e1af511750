// Fused execution of a loop chain: overlapped tiles (Section 4.4 of the
// paper, applied to GPU workgroups instead of MPI ranks) streamed through
// LDS.
//
// A fusion group is a run of consecutive 2D weighted-sum loops.  Every
// workgroup owns a block of W columns by Hseg rows of the group's domain and
// marches up y two rows per step.  At every step each loop of the group
// computes one row pair at its own lag, reading its inputs from per-dataset
// ring buffers in LDS; loaders bring chain-start values of datasets into their
// rings ahead of their first readers, storers write each dataset's final
// values for the owned block back to HBM.  A loop recomputes the points its
// later readers need beyond the owned block (its x and y extents), so blocks
// run concurrently with no communication; datasets the group writes are
// written to a second buffer (ping-pong) so that no workgroup overwrites
// values another one still loads.
#pragma once

#include "tc_internal.hpp"

namespace tc {

constexpr int kFMaxLoops = 16;
constexpr int kFMaxRings = 16;
constexpr int kFMaxLoaded = 12;  // rings with a loader (register buffers per thread)
constexpr int kFMaxEnt = 384;
constexpr int kFCols = 128;     // ring width in columns = threads per row
// Workgroup: 128 columns x TR thread rows (256, 512 or 1024 threads); every
// thread computes P consecutive rows per step: rows per step 2 (TR 2), 4
// (TR 4), 8 (TR 8) or 16 (TR 8, P 2).

struct FLoopD {
    int out_ring;
    int ent0, nent;      // stencil-point entries of the inputs, listed order
    int in0, nin;        // inputs (for per-input slot computation)
    int lag;
    int xlo, xhi, ylo, yhi;  // iteration range
    int hlo, hhi, vlo, vhi;  // columns left/right and rows below/above the owned block it computes
};

struct FInD {   // one input of a loop: ring and its entries
    int ring, ent0, nent;
    int star;   // 1 or 2: canonical radius-1/2 star (centre, -x, +x, [-2x, +2x,] -y, +y, [-2y, +2y]); 0: entries
};

struct FRingD {
    void *src;    // logical (0,0) of the buffer holding the chain-start values
    void *dst;    // logical (0,0) of the buffer receiving the final values
    int64_t sy;   // row pitch (elements)
    int depth;    // rows
    int lds_off;  // elements
    float inv_depth;
    int load;     // 0: none, 1: every point, 2: points outside the first write's range
    int load_lag, ld_below, ld_above;
    int fw_xlo, fw_xhi, fw_ylo, fw_yhi;
    int store, store_lag;
    int hull_xlo, hull_xhi, hull_ylo, hull_yhi;  // store region
    int ext_xlo, ext_xhi, ext_ylo, ext_yhi;      // allocated extent
};

struct FEnt {
    short ring;
    signed char dx, dy;
};

// Flat per-step records read by the kernel (built per flush): one record per
// loop, per loaded ring and per stored ring, so that a step reads each with a
// few wide scalar loads and no indirection.
constexpr int kFMaxIn = 4;  // inputs of a fused loop
struct FInRec {
    int off, depth;
    float inv;
    int star;  // 1 or 2: canonical star, weights in FLoopRec::w; 0: entries ent0..ent0+nent
    int ent0, nent;
};
struct FLoopRec {
    int lag, ylo, yhi, vlo, vhi;
    int out_off, out_depth;
    float out_inv;
    int nin, pad[3];
    FInRec in[kFMaxIn];
    double w[kFMaxIn][9];
};
struct FLoadRec {
    const void *src;
    int64_t sy;
    int off, depth;
    float inv;
    int lag;
    int ext_ylo, ext_yhi, ld_below, ld_above;
    int ext_xlo, ext_xhi;
    int fw, fw_xlo, fw_xhi, fw_ylo, fw_yhi;
    int alloc_xlo;  // first column of the allocated row (aligned to 16 elements)
};
struct FStoreRec {
    void *dst;
    int64_t sy;
    int off, depth;
    float inv;
    int lag;
    int hxlo, hxhi, hylo, hyhi;
};

// bytes of LDS after the rings holding the step records (copied there at
// kernel start: LDS broadcast reads are much cheaper than scalar loads that
// miss the scalar cache)
constexpr int kFDescLds = ((int)(sizeof(FLoopRec) * kFMaxLoops + sizeof(FLoadRec) * kFMaxLoaded +
                                 sizeof(FStoreRec) * kFMaxRings) + 255) / 256 * 256;

struct FGroupD {
    int nloops, nrings, nin;
    int R;           // rows per step
    int ring_bytes;  // LDS bytes of the rings (step records follow)
    int nload, nstore;
    int load_list[kFMaxRings], store_list[kFMaxRings];  // rings with a loader / a storer
    FLoopRec lrec[kFMaxLoops];
    FLoadRec ld[kFMaxLoaded];
    FStoreRec st[kFMaxRings];
    int W, HR, Hseg;
    int dom_xlo, dom_ylo, nbx, nby;
    FLoopD loops[kFMaxLoops];
    FRingD rings[kFMaxRings];
    FInD ins[kFMaxLoops * 8];
    FEnt ent[kFMaxEnt];
    double w[kFMaxEnt];
};

// Static analysis of one fusion group (cached with the plan).
struct FusedGroup {
    int g0, g1;               // loops [g0, g1) of the chain
    int dtype;
    int rows = 2;             // rows per step (2 or 4)
    int hseg_req = 0;         // requested rows per workgroup (0: automatic)
    std::vector<int> ring_dat;  // dataset of every ring
    std::vector<int> ring_store;
    FGroupD tmpl;             // descriptor without pointers, store regions or weights
    int lds_bytes = 0;
    int nblocks = 0;
    // per-group staging: pinned host copy and device copy of the descriptor,
    // and an event marking the end of the last upload from the host copy
    FGroupD *host = nullptr;
    FGroupD *dev = nullptr;
    hipEvent_t uploaded = nullptr;
};

// Split a chain into fusion groups; loops outside any group run one kernel
// each.  Returns the groups in chain order.
std::vector<std::shared_ptr<FusedGroup>> fused_split(const Ctx &c, const std::vector<LoopRec> &chain,
                                                     const int tile[3]);

// Run one fusion group on the context's stream (ping-pong buffers are
// prepared and swapped here).
tc_status fused_run(Ctx &c, const std::vector<LoopRec> &chain, FusedGroup &g);

// Kernel launch (fused_kernel.hip).
hipError_t launch_fused(const FGroupD *dev_desc, int dtype, int rows, int nblocks, int lds_bytes, hipStream_t s);

// Release device memory held for fused execution.
void fused_release(Ctx &c);

// AUTO mode: the execution mode (and tile, written back) to use for this
// chain; while candidates are being measured, autotune_record receives the
// flush's device time and autotune_finish picks the fastest when all ran.
tc_tiling autotune_choose(Ctx &c, const std::vector<LoopRec> &chain, int tile[3]);
void autotune_record(Ctx &c, double seconds);
void autotune_finish(Ctx &c, size_t ncand);
size_t autotune_candidates(const std::vector<LoopRec> &chain);

// shared helpers (api.cpp)
int canonical_star2(const Stencil &st);
double now_s();
tc_status fail(Ctx &c, tc_status s, const char *fmt, ...);
void *dev_alloc(Ctx &c, size_t bytes);
void dev_free(Ctx &c, void *p);

}  // namespace tc
