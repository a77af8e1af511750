// Fused execution of a loop chain with overlapped tiles (Section 4.4 of the
// paper, applied to GPU wavefronts instead of MPI ranks).
//
// A fusion group is a run of consecutive 2D weighted-sum loops over one
// common range.  The library generates a HIP kernel for the group at plan
// time and compiles it with hipRTC.  Every wavefront owns a strip of Wo
// columns by Hseg rows of the range; its 64 lanes hold 64 consecutive
// columns (the owned ones plus HL to the left and HR to the right) and it
// marches up the rows.  At every step each loop of the group computes one
// row at its own lag, reading its inputs from per-version register windows
// (x neighbours through cross-lane moves, y neighbours from older window
// entries); chain-start values of datasets are loaded a few rows ahead of
// their first reader and the final value of every written dataset is stored
// for the owned columns.  A loop computes the columns and rows its later
// readers need beyond the owned block, so wavefronts run with no
// communication at all.  A dataset whose chain-start value is read and which
// is also written is written to its second buffer (ping-pong), so that no
// wavefront overwrites a value another one still loads.
//
// Wavefronts whose reads stay inside the range run the "interior" kernel;
// those near the range boundary run the "edge" kernel, which additionally
// keeps the chain-start value of every written dataset where the range does
// not cover a point (such points are never written by the group).
#pragma once

#include <string>
#include <vector>

#include "staged.hpp"
#include "tc_internal.hpp"

namespace tc {

constexpr int kJLanes = 64;      // columns held by one wavefront
constexpr int kJMaxSrc = 24;     // datasets loaded by one group
constexpr int kJMaxDst = 16;     // datasets stored by one group
constexpr int kJMaxW = 384;      // weights of one group (kernel arguments)
constexpr int kJMaxOff = 8;      // largest stencil offset in x or y

struct JPt {
    int dx, dy, w;  // offset and index of the weight in the group's weight list
};

struct JRead {
    int ver;
    std::vector<JPt> pts;
    int dxmin, dxmax, dymin, dymax;
};

struct JLoop {
    int loop;  // chain index
    int out;   // version written
    std::vector<JRead> in;
    int lag = 0;
    bool needed = false;
    int extL = -1, extR = -1, extB = -1, extT = -1;  // extra columns/rows computed (-1: not needed)
};

struct JVer {
    int dat;
    int producer = -1;   // group loop index, -1 for the chain-start value
    int lag = 0;         // produced: loop lag; loaded: row y arrives at step y + lag
    bool stored = false;
    bool needed = false;
    bool sel = false;    // read at a non-zero offset (edge kernel keeps the chain-start value outside the range)
    int extL = -1, extR = -1, extB = -1, extT = -1;
};

// Per-variant schedule: which chain-start versions are loaded and the
// register window (rows) of every version.
struct JVariant {
    std::vector<int> win;         // per version, 0 if not held
    std::vector<int> load_lag;    // per version (loaded only)
    std::vector<char> loaded;     // per version
    std::vector<std::pair<int, int>> pseudo;  // (producer loop, chain-start version): edge selects
    int pre = 0, post = 0;        // steps before / after the owned rows
    int regs = 0;                 // estimated VGPRs of the windows
    int PF = 2;                   // steps loads run ahead
};

struct FusedGroup {
    int g0 = 0, g1 = 0;  // loops [g0, g1) of the chain
    int dtype = TC_F64;
    int xlo = 0, xhi = 0, ylo = 0, yhi = 0;
    std::vector<JLoop> loops;
    std::vector<JVer> vers;
    JVariant var[2];  // 0 interior, 1 edge
    int cpl = 1;      // consecutive columns held by one lane (1 or 2); a wavefront holds 64 * cpl
    int wpe = 2;      // wavefronts per SIMD requested for the interior kernel
    bool cse_steps = true;  // shifted values shared by all loops of a step (else per loop)
    bool sched_fence = false;  // scheduling barrier between the loops of a step
    int HL = 0, HR = 0, Wo = 0;
    int BMAX = 0, TMAX = 0;  // rows below / above the owned rows that are read
    int Hseg = 0, U = 3, PF = 1;
    int nstrips = 0, nsegs = 0;  // a plain grid of Wo-column strips and Hseg-row segments over the range
    // interior waves: in_ns strips by in_ng segments from (xlo + in_x, ylo + in_y)
    int in_x = 0, in_y = 0, in_ns = 0, in_ng = 0;
    int nwaves_in = 0, nwaves_edge = 0;
    int Hedge = 0;  // rows per edge wavefront
    // edge bands (relative to xlo, ylo): bottom rows [0, e_yb) and top rows
    // [e_yt, height) over the whole width; left columns [0, in_x) and right
    // columns [e_xr, width) of rows [in_y, e_yt).  Strips of Wo columns from
    // each band's left end, segments of Hedge rows from its bottom.
    int e_yb = 0, e_yt = 0, e_xr = 0;
    int e_ns = 0, e_nsl = 0, e_nsr = 0;   // strips: whole width, left band, right band
    int e_ngb = 0, e_ngt = 0, e_ngm = 0;  // segments: bottom, top and middle bands
    int nblocks = 0;
    std::vector<int> src_dat;   // datasets loaded (kernel argument order)
    std::vector<int> dst_dat;   // datasets stored
    std::vector<char> dst_twin; // store to the second buffer
    int nweights = 0;
    std::vector<double> wvals;  // weights at analysis time
    bool baked = false;         // weights compiled into the kernels
    double cost = 0.0;          // modelled seconds per flush (split choice)
    int64_t alg_bytes = 0;      // chain-start datasets read plus datasets written, once over the range
    std::string source;         // generated kernels
    std::string kname_in, kname_edge;
    hipFunction_t fin = nullptr, fedge = nullptr;
    // set for a staged group (any ops, dimensions and ranges; staged.hpp):
    // the loops run as staged tiles instead of generated register windows
    std::shared_ptr<StagedGroup> staged;
    // set for a 3D Runge-Kutta stage (EULER_RHS for the five components,
    // then RK_STAGE for the five): one z-marching kernel (euler.hip)
    std::shared_ptr<struct EulerStage> estage;
    // set for a run of 2D Chebyshev steps of the heat-conduction
    // preconditioner: one launch of cheb.hip
    std::shared_ptr<struct ChebGroup> cheb;
};

struct EulerStage {
    int q[5], q0[5], r[5], u[3], p;  // datasets
    bool r_live[5];                  // R_c read by a later loop before it is overwritten
    bool prim = false;               // the stage's EULER_PRIM loop is in the group
    bool copy0 = false;              // the group starts with the five copies Q0_c = Q_c
    int lo[3], hi[3];
};

// A run of Chebyshev steps on a 2D grid: per step the four reflective ghost
// fills of sd (x sides over the interior rows, then y sides over all
// columns, depth h), TEA_P1 (kx, ky, sd, rt, z) over the interior [0, n) and
// TEA_P2 (sd, rt) over it; the last step may end after TEA_P1.
struct ChebGroup {
    int kx, ky, sd, rt, z;  // datasets
    int r = -1, init_loop = -1;  // with the preconditioner's TEA_PRECON_INIT first: r and that loop
    // with TEA_CG_UPDATE (x, r, p, w; alpha) before the set-up: its datasets and loop
    int x = -1, p = -1, w = -1, update_loop = -1;
    int steps = 0;
    bool last_p2 = true;
    int n[2] = {0, 0}, h = 0;
    std::vector<int> p2_loop;  // chain index of each step's TEA_P2 (-1: none)
};
// The longest run of such steps starting at loop i (at most kChebMaxSteps
// steps): fills C and returns the number of loops, else 0.  Every prefix of
// whole steps is a run too.
int cheb_match(const Ctx &c, const std::vector<LoopRec> &chain, int i, ChebGroup &C);

// Loops [i, i + 10) as a 3D Runge-Kutta stage (the five right-hand sides,
// then the five updates over one range, sharing Q, the velocities and the
// pressure): fills E and returns true, else false.
bool euler_stage_match(const Ctx &c, const std::vector<LoopRec> &chain, int i, EulerStage &E);
// Loops [i, i + 11): the stage's EULER_PRIM loop (over a range that covers
// the right-hand sides' reads) and the stage, with every primitive variable
// overwritten by a later loop before any read (so none reaches memory).
bool euler_stage_match_prim(const Ctx &c, const std::vector<LoopRec> &chain, int i, EulerStage &E);
// Loops [i, i + 5 + n) with n = 11 (prim) or 10: five copies Q0_c = Q_c (one
// per component, any order, each over the stage's range) and then the stage.
bool euler_stage_match_copy(const Ctx &c, const std::vector<LoopRec> &chain, int i, bool prim, EulerStage &E);

// Split a chain into fusion groups (loops outside any group run one kernel
// each) and generate their kernels; returns the groups in chain order.
std::vector<std::shared_ptr<FusedGroup>> fused_split(Ctx &c, const std::vector<LoopRec> &chain, const int tile[3],
                                                     int cpl);

// Whether a loop can be part of a fusion group at all (its op and dimension).
bool fused_op_supported(const LoopRec &lp);

// Compile (and, on a device context, load) the kernels of a plan's groups;
// staged groups get their device tables uploaded.
tc_status fused_compile(Ctx &c, const std::vector<LoopRec> &chain, std::vector<std::shared_ptr<FusedGroup>> &groups);

// Run one fusion group on the context's stream (ping-pong buffers are
// prepared and swapped here).
tc_status fused_run(Ctx &c, const std::vector<LoopRec> &chain, FusedGroup &g);

// For a call that allocates nothing: TC_ERR_STATE if running the group would
// compile kernels or allocate its second buffers (checked before anything runs).
tc_status fused_check_noalloc(Ctx &c, const std::vector<LoopRec> &chain, const FusedGroup &G);

// Release modules held for fused execution.
void fused_release(Ctx &c);

// AUTO mode: the schedule to use for this chain; while candidates are being
// measured, autotune_record receives the flush's device time and
// autotune_finish picks the fastest when all ran.
TuneCand autotune_choose(Ctx &c, const std::vector<LoopRec> &chain);
void autotune_record(Ctx &c, double seconds);
void autotune_finish(Ctx &c, const std::vector<LoopRec> &chain);
uint64_t autotune_key(const Ctx &c, const std::vector<LoopRec> &chain);
// The autotuner's choice for this chain structure if it has one (measured in
// this context or read from the choice cache); no measurement state changes.
bool autotune_lookup(Ctx &c, const std::vector<LoopRec> &chain, TuneCand &out);

// shared helpers (api.cpp)
void build_desc(const Ctx &c, const LoopRec &lp, LoopDesc &d);
int canonical_star2(const Stencil &st);
double now_s();
tc_status fail(Ctx &c, tc_status s, const char *fmt, ...);
void *dev_alloc(Ctx &c, size_t bytes);
void dev_free(Ctx &c, void *p);

}  // namespace tc
