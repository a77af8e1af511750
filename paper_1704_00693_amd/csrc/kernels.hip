// Per-loop HIP kernels for gfx950: one launch runs one loop over one box of
// its iteration range (the whole range when untiled, a tile's range in the
// skewed schedule of Algorithm 2).  Each op is a small device functor; the
// kernel maps workgroups to boxes of 64 x 4 points (x fastest, one FP64 row
// segment of 512 bytes per wavefront) and orders the workgroup index so that
// each of the 8 XCDs gets one contiguous band of rows (vertical stencil
// neighbours then hit in that XCD's own L2).
//
// Reductions accumulate in FP64 as double-double (error-free transforms:
// TwoSum, and fma for the exact product), per thread, then across the
// workgroup, and each workgroup writes one (hi, lo) partial.
#include <hip/hip_runtime.h>

#include "dd.hpp"
#include "kernels.hpp"
#include "ops.hpp"

namespace tc {

static_assert(kRedThreads == kBlockThreads, "reductions combine one value per thread of a workgroup");

// ---------------------------------------------------------------------------
// the loop kernel
// ---------------------------------------------------------------------------
template <class Op>
__global__ void __launch_bounds__(kBlockThreads) loop_kernel(LoopDesc d, Box b) {
    // XCD-aware order: hardware block i runs on XCD i % 8; give XCD k the
    // contiguous block range [k*q + min(k, r), ...).
    const int nb = b.nb;
    const int i = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, xcd = i & 7, k = i >> 3;
    const int lin = xcd * q + (xcd < r ? xcd : r) + k;
    const int bx = lin % b.nbx;
    const int rest = lin / b.nbx;
    const int by = rest % b.nby;
    const int bz = rest / b.nby;
    const int x = b.lo[0] + bx * b.bw + (int)(threadIdx.x % b.bw);
    const int y = b.lo[1] + by * b.bh + (int)(threadIdx.x / b.bw);
    const int z = b.lo[2] + bz;
    // the accumulators are indexed with constants only (the loop below is
    // unrolled), so they stay in registers rather than in scratch or LDS
    DD red[2];
    red[0] = red_identity(d.red_op[0]);
    red[1] = red_identity(d.red_op[1]);
    if (x < b.hi[0] && y < b.hi[1]) Op::run(d, x, y, z, red);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (j >= d.nred) break;
        DD v = block_reduce(d.red_op[j], red[j]);
        if (threadIdx.x == 0) {
            d.partials[j][2 * (int64_t)lin] = v.hi;
            d.partials[j][2 * (int64_t)lin + 1] = v.lo;
        }
    }
}

constexpr int kFinMax = 16;  // reductions per launch of finalize_many_kernel
struct FinalizeMany {
    const double *part;
    double *out;
    int64_t base[kFinMax], count[kFinMax];
    int op[kFinMax];
};

// Workgroup r combines reduction r's partials in a fixed order.
__global__ void __launch_bounds__(kBlockThreads) finalize_many_kernel(FinalizeMany f) {
    const int r = blockIdx.x;
    const int op = f.op[r];
    const double *part = f.part + 2 * f.base[r];
    DD a = red_identity(op);
    for (int64_t i = threadIdx.x; i < f.count[r]; i += kBlockThreads) {
        DD b;
        b.hi = part[2 * i];
        b.lo = part[2 * i + 1];
        a = red_combine(op, a, b);
    }
    a = block_reduce(op, a);
    if (threadIdx.x == 0) {
        f.out[2 * r] = a.hi;
        f.out[2 * r + 1] = a.lo;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
Box make_box(int ndim, const int lo[3], const int hi[3]) {
    Box b;
    for (int k = 0; k < 3; ++k) {
        b.lo[k] = lo[k];
        b.hi[k] = hi[k];
    }
    int nx = hi[0] - lo[0], ny = hi[1] - lo[1], nz = hi[2] - lo[2];
    if (ndim == 1 || ny == 1) {
        b.bw = kBlockThreads;
        b.bh = 1;
    } else if (nx <= 4) {
        b.bw = 4;
        b.bh = kBlockThreads / 4;
    } else if (nx <= 16) {
        b.bw = 16;
        b.bh = kBlockThreads / 16;
    } else {
        b.bw = 64;
        b.bh = kBlockThreads / 64;
    }
    b.nbx = (nx + b.bw - 1) / b.bw;
    b.nby = (ny + b.bh - 1) / b.bh;
    b.nb = b.nbx * b.nby * nz;
    return b;
}

template <class Op>
static hipError_t go(const LoopDesc &d, const Box &b, hipStream_t s) {
    hipLaunchKernelGGL(loop_kernel<Op>, dim3(b.nb), dim3(kBlockThreads), 0, s, d, b);
    return hipGetLastError();
}

template <typename T>
static hipError_t dispatch_t(const LoopDesc &d, const Box &b, hipStream_t s) {
    switch (d.op) {
    case TC_OP_WSUM: return go<OpWsum<T>>(d, b, s);
    case TC_OP_AXPBY: return go<OpAxpby<T>>(d, b, s);
    case TC_OP_DOT: return go<OpDot<T>>(d, b, s);
    case TC_OP_SUM: return go<OpSum<T>>(d, b, s);
    case TC_OP_HALO_REFLECT: return go<OpHaloReflect<T>>(d, b, s);
    case TC_OP_TEA_INIT: return go<OpTeaInit<T>>(d, b, s);
    case TC_OP_TEA_K: return go<OpTeaK<T>>(d, b, s);
    case TC_OP_TEA_RESID: return go<OpTeaResid<T>>(d, b, s);
    case TC_OP_TEA_MATVEC_DOT: return go<OpTeaMatvecDot<T>>(d, b, s);
    case TC_OP_TEA_P1: return go<OpTeaP1<T>>(d, b, s);
    case TC_OP_TEA_P2: return go<OpTeaP2<T>>(d, b, s);
    case TC_OP_TEA_PRECON_INIT: return go<OpTeaPreconInit<T>>(d, b, s);
    case TC_OP_TEA_CG_UPDATE: return go<OpTeaCgUpdate<T>>(d, b, s);
    case TC_OP_TEA_CG_P: return go<OpTeaCgP<T>>(d, b, s);
    case TC_OP_TEA_GERSH: return go<OpTeaGersh<T>>(d, b, s);
    case TC_OP_EULER_PRIM: return go<OpEulerPrim<T>>(d, b, s);
    case TC_OP_EULER_RHS: return go<OpEulerRhs<T>>(d, b, s);
    case TC_OP_RK_STAGE: return go<OpRkStage<T>>(d, b, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_loop(const LoopDesc &d, const Box &b, int dtype0, int dtype1, int march_mask, const MarchShape &ms,
                       hipStream_t s) {
    if (b.nb <= 0) return hipSuccess;
    if (d.op == TC_OP_WSUM) return launch_wsum(d, b, dtype0, march_mask, ms, s);
    if (d.op == TC_OP_EULER_RHS && d.ndim == 3 && march_mask >= 0) return launch_euler_rhs3(d, b, dtype0, s);
    if (d.op == TC_OP_COPY) {
        if (dtype0 == TC_F64 && dtype1 == TC_F64) return go<OpCopy<double, double>>(d, b, s);
        if (dtype0 == TC_F32 && dtype1 == TC_F32) return go<OpCopy<float, float>>(d, b, s);
        if (dtype0 == TC_F64 && dtype1 == TC_F32) return go<OpCopy<double, float>>(d, b, s);
        return go<OpCopy<float, double>>(d, b, s);
    }
    return dtype0 == TC_F64 ? dispatch_t<double>(d, b, s) : dispatch_t<float>(d, b, s);
}

hipError_t launch_finalize_many(const double *part, const int64_t *base, const int64_t *count, const int *op, int n,
                                double *out, hipStream_t s) {
    for (int r0 = 0; r0 < n; r0 += kFinMax) {
        FinalizeMany f;
        const int m = std::min(kFinMax, n - r0);
        f.part = part;
        f.out = out + 2 * r0;
        for (int k = 0; k < kFinMax; ++k) {
            f.base[k] = k < m ? base[r0 + k] : 0;
            f.count[k] = k < m ? count[r0 + k] : 0;
            f.op[k] = k < m ? op[r0 + k] : 0;
        }
        hipLaunchKernelGGL(finalize_many_kernel, dim3(m), dim3(kBlockThreads), 0, s, f);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tc
