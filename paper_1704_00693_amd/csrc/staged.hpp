// Staged tiles: overlapped tiles (Section 4.4 of the paper) for runs of loops
// of any op, dimension and iteration range, executed by one workgroup per
// tile with the working set staged in LDS.
//
// The union of the group's loop ranges is cut into owned boxes (tiles).  For
// every tile the analysis walks the group backwards from its owned box: a
// loop computes the hull of the points where a later loop of the group, or
// the final state on the owned box, needs a value it writes (clipped to its
// range), and the points it reads there through its stencils are then
// needed from the loops before it.  A loop with a reduction also computes
// the owned part of its range, and only owned points contribute to the
// reduction, so each point counts once.
//
// Every dataset the group writes lives in LDS for the tile's lifetime, over
// the hull of everything the tile reads or writes of it; its chain-start
// values are loaded where they are needed, the loops run one after the
// other (one barrier between loops) in place, and the owned box is written
// back.  Datasets the group only reads are staged in LDS over their read
// hull too while they fit (the most accessed first), else read from device
// memory directly.  A written dataset whose chain-start values a tile loads beyond
// its own owned box is written to the dataset's second buffer (ping-pong),
// so no tile overwrites a value another still loads.  The point arithmetic
// is the per-loop kernels' own functors (ops.hpp), so results are
// bit-identical to untiled execution; reductions differ only in summation
// order.
#pragma once

#include <array>
#include <vector>

#include "tc_internal.hpp"

namespace tc {

constexpr int kSMaxDat = 24;        // datasets one staged group names
constexpr int kSMaxLoops = 128;     // loops of one staged group
constexpr int kSMaxPrm = 256;       // scalar parameters of one group (kernel arguments)
constexpr int kSThreads = 1024;     // most threads per tile workgroup (the default is 256)
constexpr int64_t kSLdsBudget = 150 * 1024;  // bytes of LDS for the staged datasets and one descriptor

// Per dataset slot of a group (device copy in the group's table).
struct SSlot {
    int resident;    // written by the group: staged in LDS and written back
    int staged;      // held in LDS (every written dataset; read-only ones while they fit)
    int twin;        // write back to the second buffer
    int pad;
    int64_t lds_off;  // element offset of the slot's LDS box
    int64_t lsy, lsz;  // element strides of the LDS box
    int wlo[3], whi[3];  // hull of the ranges of the loops writing it (write-back region within a tile)
};

// Per loop of a group (device copy).
struct SLoop {
    int slot[kMaxArgs];  // slot of every dataset argument
    int prm_off, nprm;   // parameters in the kernel-argument array (LoopDesc prm layout)
    int prm_skip;        // leading entries of that layout the loop's parameters skip (a weighted
                         // sum's output stencil points)
    int all_lds;         // every dataset argument is staged: LDS-addressed accesses
    int64_t part[2];     // first partial of each reduction argument (one per tile follows)
};

struct StagedGroup {
    int g0 = 0, g1 = 0;
    int ndim = 2;
    int dtype = TC_F64;
    int tile[3] = {1, 1, 1};       // owned box extent per dimension
    int ulo[3] = {0, 0, 0}, uhi[3] = {1, 1, 1};  // union of the loop ranges
    int nt[3] = {1, 1, 1};
    int ntot = 0;                  // tiles
    int threads = kSThreads;       // workgroup size: 256 or 1024
    std::vector<int> dats;         // dataset of every slot
    std::vector<SSlot> slots;
    std::vector<SLoop> loops;
    int64_t lds_bytes = 0;         // staged datasets (descriptor excluded)
    int64_t desc_off = 0;          // byte offset of the loop descriptor in LDS
    int rec = 0;                   // ints per tile record
    std::vector<int> table;        // tile records (built for the chosen tiling)
    int nprm = 0;
    int nred_loops = 0;
    // per loop, the computed box of an interior tile relative to its owned
    // box (lo: points below the owned box, hi: points above), -1 if the
    // interior tile does not compute it
    std::vector<std::array<int, 6>> ext;
    std::vector<char> computed;    // per loop: computed by some tile
    double cost = 0.0;             // modelled seconds per run
    int64_t alg_bytes = 0;         // chain-start values of written datasets over their write regions, the
                                   // datasets only read over the union range, and the write-backs
    void *dev = nullptr;           // device copy: descriptors, loops, slots, table
    size_t dev_bytes = 0;
    int64_t off_loops = 0, off_slots = 0, off_table = 0;
};

// Analyse loops [g0, g1) of the chain as one staged group.  tile: owned box
// extents (0: choose).  With full == false only representative tiles are
// walked (enough to size LDS and model the cost; used by the split search);
// with full == true every tile is walked and the table is built.  False if
// the loops cannot form a staged group (mixed element types or blocks, too
// many datasets or parameters, LDS too small for any tile shape).
bool staged_analyse(const Ctx &c, const std::vector<LoopRec> &chain, int g0, int g1, const int tile[3], bool full,
                    StagedGroup &G);

// Build the descriptor templates and upload the group's tables (device
// contexts); partial offsets must be final.
tc_status staged_upload(Ctx &c, const std::vector<LoopRec> &chain, StagedGroup &G);

// Run the group on the context's stream.
tc_status staged_run(Ctx &c, const std::vector<LoopRec> &chain, StagedGroup &G);

// For a call that allocates nothing: TC_ERR_STATE if running the group would
// allocate (its second buffers do not all exist yet).
tc_status staged_check_noalloc(Ctx &c, const StagedGroup &G);

// Device side (staged.hip): launch one group.
struct SArgs {
    const LoopDesc *loops;
    const SLoop *sl;
    const SSlot *slots;
    const int *table;
    double *partials;
    int nloops, nslots, rec, ntot;
    int64_t desc_off;
    void *src[kSMaxDat];  // chain-start buffer of every slot (logical origin)
    void *dst[kSMaxDat];  // write-back buffer of every resident slot (logical origin)
    int64_t gsy[kSMaxDat], gsz[kSMaxDat];  // device strides of every slot
    double prm[kSMaxPrm];
};
// threads: 256 or 1024 (one workgroup per tile)
hipError_t launch_staged(const SArgs &a, int dtype, size_t lds_bytes, int threads, hipStream_t s);

}  // namespace tc
