// Launch interface of the per-loop kernels (kernels.hip).
#pragma once

#include "tc_internal.hpp"

namespace tc {

constexpr int kBlockThreads = 256;

// A box of points handed to one launch, with its workgroup decomposition.
struct Box {
    int lo[3], hi[3];
    int bw, bh;        // workgroup footprint: bw points in x by bh rows in y
    int nbx, nby, nb;  // workgroups along x, along y, total (z: nb / (nbx*nby))
};

Box make_box(int ndim, const int lo[3], const int hi[3]);

// Launch one loop over a box.  dtype0 / dtype1: element types of dataset
// arguments 0 and 1 (they differ only for a converting TC_OP_COPY).
// march_mask: for TC_OP_WSUM, -1 or the radius mask of the register-window
// variant (bit a set: input a uses the radius-2 canonical star, else radius 1).
// ms: workgroup shapes of that variant.
hipError_t launch_loop(const LoopDesc &d, const Box &b, int dtype0, int dtype1, int march_mask, const MarchShape &ms,
                       hipStream_t s);

// Weighted-sum kernels (wsum.hip).
hipError_t launch_wsum(const LoopDesc &d, const Box &b, int dtype, int march_mask, const MarchShape &ms, hipStream_t s);
// 3D EULER_RHS marching up z (same arithmetic as the per-point kernel)
hipError_t launch_euler_rhs3(const LoopDesc &d, const Box &b, int dtype, hipStream_t s);

// One 3D Runge-Kutta stage: EULER_RHS for the five components and RK_STAGE
// for the five components, fused (euler.hip), optionally with the stage's
// EULER_PRIM loop before them (its results then never reach memory) and the
// step's five copies Q0_c = Q_c over the stage's range before that (Q0 is
// then taken from Q in registers and written out).
// Arrays (logical origins and strides): kQ + c the stage's Q_c (read at
// +-2 along every axis), kQ0 + c the step's Q0_c, kU + d the velocities, kP
// the pressure; out[c] receives the new Q_c, rout[c] (may be NULL) R_c.
enum { kQ = 0, kQ0 = 5, kU = 10, kP = 13, kEulerArrays = 14 };
struct EulerStageArgs {
    const void *ptr[kEulerArrays];
    int64_t sy[kEulerArrays], sz[kEulerArrays];
    void *out[5];
    int64_t osy[5], osz[5];
    void *rout[5];
    int64_t rsy[5], rsz[5];
    double s, a, b, dt;
    double gm1;            // prim: gamma - 1
    int prim;              // 1: the primitives are computed from Q (their loop is fused in)
    int copy0;             // 1: Q0_c = Q_c is fused in; q0out[c] receives it (kQ0 + c is not read)
    void *q0out[5];
    int64_t q0sy[5], q0sz[5];
    int lo[3], hi[3];
    int rows, tz;          // workgroup rows (4 or 8) and planes; 0: chosen by the launcher
    int nbx, nby, nb;      // set by the launcher
};
hipError_t launch_euler_stage3(const EulerStageArgs &a, int dtype, hipStream_t s);

// Chebyshev steps of the heat-conduction preconditioner on a 2D grid, fused
// (cheb.hip): `steps` repetitions of [reflective ghost fill of sd to depth h,
// TEA_P1, TEA_P2], the last TEA_P2 left out when last_p2 is 0.  A workgroup
// owns kChebTX x kChebTY cells and recomputes `steps` cells around them.
// Arrays by logical origin and row stride: kx, ky read; sd and rt read from
// *_in and written to *_out (other workgroups still read the old values);
// z read and written in place (only ever read at its own cell).  The ghost
// cells of sd are written as the last step's fill leaves them.  Optionally
// the preconditioner's set-up (TEA_PRECON_INIT) comes first, and the CG
// update of x and r (TEA_CG_UPDATE) before it.
constexpr int kChebMaxSteps = 9;
constexpr int kChebTX = 64, kChebTY = 16;
struct ChebArgs {
    const void *kx, *ky, *sd_in, *rt_in;
    void *sd_out, *rt_out, *z;
    int64_t skx, sky, ssd_in, srt_in, ssd_out, srt_out, sz;  // row strides (elements)
    // start != 0: TEA_PRECON_INIT first (rt = r, sd = r / theta, z = 0);
    // sd_in, rt_in and z are then not read
    const void *r;
    int64_t sr;
    double theta;
    int start;
    // update != 0 (with start): TEA_CG_UPDATE first, x = fma(alpha, p, x)
    // and r = fma(-alpha, w, r) (x in place, the new r to r_out)
    const void *p, *w;
    void *x, *r_out;
    int64_t sp, sw, sx, sro;
    double alpha;
    int update;
    double al[kChebMaxSteps], be[kChebMaxSteps];
    int n0, n1;            // interior extent along x and y
    int h;                 // ghost depth of the fills
    int steps, last_p2;
    int ntx, nty;          // set by the launcher
};
hipError_t launch_cheb2(const ChebArgs &a, int dtype, hipStream_t s);
// Cells recomputed around a tile for a group of `steps` steps (3, 5, 7 or 9).
inline int cheb_halo(int steps) { return steps <= 3 ? 3 : steps <= 5 ? 5 : steps <= 7 ? 7 : 9; }

// Combine the (hi, lo) partials of n reductions, one workgroup each, in a
// fixed order: reduction r's count[r] pairs start at part + 2 * base[r] and
// its result goes to out[2r], out[2r+1].  base, count, op: host arrays.
hipError_t launch_finalize_many(const double *part, const int64_t *base, const int64_t *count, const int *op, int n,
                                double *out, hipStream_t s);

}  // namespace tc
