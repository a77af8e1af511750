// Batched heat-conduction solves: many independent PPCG solves of uneven
// sizes advanced together, one kernel launch per solver phase for all of them
// (the phase sequence of one iteration is captured once in a HIP graph and
// replayed).  Every instance is a small state machine kept on the device:
//
//   INIT         generate density/energy (counter-based SplitMix64), u0 = u = e*rho,
//                face coefficients, Gershgorin bound, Chebyshev scalars
//   RESID/OUTER  r = b - A x in FP64 (mixed: also the FP32 copy of r, d = 0,
//                and the refinement test on the true residual)
//   INNER_START  preconditioner on the new residual, rz
//   INNER        PPCG iterations (FP64 sweeps, or FP32 sweeps in mixed mode)
//   VERIFY       FP64: the true residual of the converged solution
//   DONE / FREE
//
// The solver arithmetic is the per-cell arithmetic of the library's TEA_*
// loops (same operations in the same order), with the reflective ghost cells
// read by mirroring the index instead of being stored.
#pragma once

#include <cstdint>

namespace tc {

enum BState : int {
    B_FREE = 0,
    B_INIT = 1,
    B_RESID = 2,
    B_INNER_START = 3,
    B_INNER = 4,
    B_OUTER = 5,
    B_VERIFY = 6,
    B_DONE = 7,
};

constexpr int kBTX = 64, kBTY = 4;  // cells of one tile: one workgroup of 256 threads
// 2D Chebyshev steps run up to FH at a time on tiles of kFTX x FTY owned
// cells (plus FH cells around them, recomputed), with the direction in LDS;
// (FH, FTY) is one of the compiled shapes below (default kFH, kFTY)
constexpr int kFTX = 64, kFTY = 16, kFH = 3;
// 3D Chebyshev steps run up to three at a time in a march up the planes of
// z-segments of kF3Z planes, on tiles of kF3X x kF3Y owned cells (plus a
// border of one cell per step, recomputed)
constexpr int kF3X = 64, kF3Y = 8, kF3Z = 32;
constexpr int kBMaxCheb = 32;

struct BInst {
    int32_t ndim, n, state, mixed;
    int32_t iters, outer, max_iter, max_outer;
    int32_t cheb_steps, converged, inner_k, pad1;  // inner_k: iterations of the current (correction) solve
    int64_t tile0, ntile;  // tiles [tile0, tile0 + ntile) of the current tile list
    int64_t sy, sz, org;   // padded layout: cell (x,y,z) at org + x + y*sy + z*sz
    uint64_t seed;
    double tol, inner_tol, rx;
    double bnorm, lmax, theta, rz, beta, alpha, r0, rr, true_rr;
    double al[kBMaxCheb], be[kBMaxCheb];
    double *u, *u0, *r, *kx, *ky, *kz;  // FP64 fields
    // fields of the PPCG sweeps (FP64 mode: double, aliasing u, r, kx..;
    // mixed mode: float)
    void *xi, *ri, *p, *w, *z, *rt, *sd0, *sd1, *kxi, *kyi, *kzi;
    void *rt2;  // the second rt buffer of the fused Chebyshev steps (neighbouring tiles read rt around theirs)
};

struct BTile {
    int32_t inst, tx, ty, tz;
};

// A tile list on the device (length read by the kernels) and its host copy.
struct BTileList {
    BTile *d = nullptr, *h = nullptr;
    int64_t *dn = nullptr, *hn = nullptr;
};

}  // namespace tc
