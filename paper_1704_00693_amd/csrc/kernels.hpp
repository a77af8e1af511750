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
// march_ty: rows per workgroup of that variant.
hipError_t launch_loop(const LoopDesc &d, const Box &b, int dtype0, int dtype1, int march_mask, int march_ty,
                       hipStream_t s);

// Weighted-sum kernels (wsum.hip).
hipError_t launch_wsum(const LoopDesc &d, const Box &b, int dtype, int march_mask, int march_ty, hipStream_t s);
// 3D EULER_RHS marching up z (same arithmetic as the per-point kernel)
hipError_t launch_euler_rhs3(const LoopDesc &d, const Box &b, int dtype, hipStream_t s);

// Combine `count` (hi, lo) partials into out[0..1] with one workgroup.
hipError_t launch_finalize(const double *part, int64_t count, int op, double *out, hipStream_t s);

}  // namespace tc
