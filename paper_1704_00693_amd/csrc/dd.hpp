// Double-double accumulation for FP64 reductions (error-free transforms:
// TwoSum for additions, fma for the exact product) and the workgroup-wide
// combine used by every reduction kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "tilechain.h"

namespace tc {

constexpr int kRedThreads = 256;

// ---------------------------------------------------------------------------
// double-double helpers
// ---------------------------------------------------------------------------
struct DD {
    double hi, lo;
};

__device__ __forceinline__ void dd_add(DD &a, double v) {
    double s = a.hi + v;
    double bb = s - a.hi;
    double e = (a.hi - (s - bb)) + (v - bb);
    a.hi = s;
    a.lo += e;
}

__device__ __forceinline__ void dd_add_prod(DD &a, double x, double y) {
    double p = x * y;
    double pe = __builtin_fma(x, y, -p);
    dd_add(a, p);
    a.lo += pe;
}

__device__ __forceinline__ DD dd_merge(DD a, DD b) {
    double s = a.hi + b.hi;
    double bb = s - a.hi;
    double e = (a.hi - (s - bb)) + (b.hi - bb);
    DD r;
    r.hi = s;
    r.lo = (a.lo + b.lo) + e;
    return r;
}

__device__ __forceinline__ DD red_combine(int op, DD a, DD b) {
    if (op == TC_RED_SUM) return dd_merge(a, b);
    DD r;
    r.lo = 0.0;
    if (op == TC_RED_MIN)
        r.hi = fmin(a.hi, b.hi);
    else
        r.hi = fmax(a.hi, b.hi);
    return r;
}

__device__ __forceinline__ DD red_identity(int op) {
    DD r;
    r.lo = 0.0;
    r.hi = op == TC_RED_SUM ? 0.0 : (op == TC_RED_MIN ? __builtin_inf() : -__builtin_inf());
    return r;
}

// Workgroup-wide combine of one DD value per thread; thread 0 gets the result.
__device__ inline DD block_reduce(int op, DD v) {
    __shared__ double sh_hi[kRedThreads / 64], sh_lo[kRedThreads / 64];
    for (int o = 32; o > 0; o >>= 1) {
        DD w;
        w.hi = __shfl_xor(v.hi, o);
        w.lo = __shfl_xor(v.lo, o);
        v = red_combine(op, v, w);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sh_hi[wv] = v.hi;
        sh_lo[wv] = v.lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        DD a;
        a.hi = sh_hi[0];
        a.lo = sh_lo[0];
        for (int i = 1; i < kRedThreads / 64; ++i) {
            DD b;
            b.hi = sh_hi[i];
            b.lo = sh_lo[i];
            a = red_combine(op, a, b);
        }
        v = a;
    }
    __syncthreads();
    return v;
}

}  // namespace tc
