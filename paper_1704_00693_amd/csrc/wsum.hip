// Weighted-sum loop kernels (TC_OP_WSUM) for one box of the iteration range.
//
// Two variants, both with the arithmetic order of the op's definition
// (acc = fma(w, v, acc) over inputs and stencil points in listed order):
//
//  * march: 2D, every input read through a radius-1 or radius-2 star stencil
//    listed in the canonical order (centre, -x, +x, [-2x, +2x,] -y, +y,
//    [-2y, +2y]).  A workgroup covers 256 consecutive x and marches TY rows
//    up y; each thread keeps the vertical window of every input in
//    registers (one new row load per input per output row) and takes its x
//    neighbours from adjacent lanes with cross-lane shuffles, so global
//    loads per output point drop from sum(stencil points) to about the
//    number of inputs.
//  * generic: any stencils and dimensions; all loads of a point are issued
//    before its fma chain so one memory latency covers the whole point.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace tc {

namespace {

constexpr int kMarchTY = 16;  // rows per workgroup in the march kernel
constexpr int kMarchW = 256;  // columns per workgroup (4 wavefronts)

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

template <typename T>
__device__ __forceinline__ T shfl_up(T v, int d) {
    return __shfl_up(v, d, 64);
}
template <typename T>
__device__ __forceinline__ T shfl_down(T v, int d) {
    return __shfl_down(v, d, 64);
}

// XCD-aware workgroup order: hardware block i runs on XCD i % 8; XCD k gets
// the contiguous logical block range starting at k*q + min(k, r).
__device__ __forceinline__ int xcd_linear(int i, int nb) {
    const int q = nb >> 3, r = nb & 7, xcd = i & 7, k = i >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

template <typename T, int K, int MASK>
__global__ void __launch_bounds__(kMarchW) wsum_march_kernel(LoopDesc d, int lo0, int hi0, int lo1, int hi1, int nbx,
                                                             int nb) {
    const int lin = xcd_linear(blockIdx.x, nb);
    const int bx = lin % nbx, by = lin / nbx;
    const int lane = threadIdx.x & 63;
    const int x = lo0 + bx * kMarchW + (int)threadIdx.x;
    const bool active = x < hi0;
    const int xc = active ? x : hi0 - 1;  // inactive lanes load a valid address
    const int y0 = lo1 + by * kMarchTY;
    const int y1 = min(y0 + kMarchTY, hi1);

    const T *ptr[K];
    int64_t sy[K];
    T win[K][5];  // vertical window rows y-2 .. y+2 (radius 1 uses 1..3)
    T pf[K];      // next row of every input, loaded one step ahead
#pragma unroll
    for (int a = 0; a < K; ++a) {
        ptr[a] = (const T *)d.arg[a + 1].ptr;
        sy[a] = d.arg[a + 1].sy;
        const int r = (MASK >> a) & 1 ? 2 : 1;
        const T *col = ptr[a] + xc + (int64_t)y0 * sy[a];
#pragma unroll
        for (int j = -2; j < 2; ++j)
            if (j >= -r && j < r) win[a][j + 2] = col[(int64_t)j * sy[a]];
        pf[a] = col[(int64_t)r * sy[a]];
    }
    T *out = (T *)d.arg[0].ptr;
    const int64_t osy = d.arg[0].sy;
    for (int y = y0; y < y1; ++y) {
        T acc = (T)0;
        const bool more = y + 1 < y1;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int r = (MASK >> a) & 1 ? 2 : 1;
            win[a][2 + r] = pf[a];
            if (more) pf[a] = ptr[a][(int64_t)(y + 1 + r) * sy[a] + xc];
        }
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int r = (MASK >> a) & 1 ? 2 : 1;
            const T *row = ptr[a] + (int64_t)y * sy[a];
            const T c = win[a][2];
            T xm1 = shfl_up(c, 1), xp1 = shfl_down(c, 1);
            if (lane < 1) xm1 = row[xc - 1];
            if (lane > 62 || x + 1 >= hi0) xp1 = row[xc + 1];
            const int q = d.pt0[a + 1];
            if (r == 1) {
                acc = fmaT<T>((T)d.prm[q + 0], c, acc);
                acc = fmaT<T>((T)d.prm[q + 1], xm1, acc);
                acc = fmaT<T>((T)d.prm[q + 2], xp1, acc);
                acc = fmaT<T>((T)d.prm[q + 3], win[a][1], acc);
                acc = fmaT<T>((T)d.prm[q + 4], win[a][3], acc);
            } else {
                T xm2 = shfl_up(c, 2), xp2 = shfl_down(c, 2);
                if (lane < 2) xm2 = row[xc - 2];
                if (lane > 61 || x + 2 >= hi0) xp2 = row[xc + 2];
                acc = fmaT<T>((T)d.prm[q + 0], c, acc);
                acc = fmaT<T>((T)d.prm[q + 1], xm1, acc);
                acc = fmaT<T>((T)d.prm[q + 2], xp1, acc);
                acc = fmaT<T>((T)d.prm[q + 3], xm2, acc);
                acc = fmaT<T>((T)d.prm[q + 4], xp2, acc);
                acc = fmaT<T>((T)d.prm[q + 5], win[a][1], acc);
                acc = fmaT<T>((T)d.prm[q + 6], win[a][3], acc);
                acc = fmaT<T>((T)d.prm[q + 7], win[a][0], acc);
                acc = fmaT<T>((T)d.prm[q + 8], win[a][4], acc);
            }
            // shift the window one row up
#pragma unroll
            for (int j = 0; j < 4; ++j) win[a][j] = win[a][j + 1];
        }
        if (active) out[(int64_t)y * osy + x] = acc;
    }
}

constexpr int kGenericMaxQ = 40;  // stencil points handled by the unrolled generic path

template <typename T>
__global__ void __launch_bounds__(kBlockThreads) wsum_generic_kernel(LoopDesc d, Box b) {
    const int lin = xcd_linear(blockIdx.x, b.nb);
    const int bx = lin % b.nbx;
    const int rest = lin / b.nbx;
    const int by = rest % b.nby;
    const int bz = rest / b.nby;
    const int x = b.lo[0] + bx * b.bw + (int)(threadIdx.x % b.bw);
    const int y = b.lo[1] + by * b.bh + (int)(threadIdx.x / b.bw);
    const int z = b.lo[2] + bz;
    if (x >= b.hi[0] || y >= b.hi[1]) return;
    const int q0 = d.npts[0];  // points of the output argument come first
    const int nq = d.pt0[d.nargs - 1] + d.npts[d.nargs - 1];
    T acc = (T)0;
    if (nq - q0 <= kGenericMaxQ) {
        T v[kGenericMaxQ];
#pragma unroll
        for (int k = 0; k < kGenericMaxQ; ++k) {
            const int q = q0 + k;
            if (q < nq) {
                const int a = d.qarg[q];
                const T *p = (const T *)d.arg[a].ptr;
                v[k] = p[(int64_t)x + (int64_t)y * d.arg[a].sy + (int64_t)z * d.arg[a].sz + d.off[q]];
            }
        }
#pragma unroll
        for (int k = 0; k < kGenericMaxQ; ++k)
            if (q0 + k < nq) acc = fmaT<T>((T)d.prm[q0 + k], v[k], acc);
    } else {
        for (int a = 1; a < d.nargs; ++a) {
            const T *p = (const T *)d.arg[a].ptr + (int64_t)x + (int64_t)y * d.arg[a].sy + (int64_t)z * d.arg[a].sz;
            for (int k = 0; k < d.npts[a]; ++k) acc = fmaT<T>((T)d.prm[d.pt0[a] + k], p[d.off[d.pt0[a] + k]], acc);
        }
    }
    T *o = (T *)d.arg[0].ptr;
    o[(int64_t)x + (int64_t)y * d.arg[0].sy + (int64_t)z * d.arg[0].sz] = acc;
}

template <typename T, int K, int MASK>
hipError_t go_march(const LoopDesc &d, const int lo[3], const int hi[3], hipStream_t s) {
    const int nbx = (hi[0] - lo[0] + kMarchW - 1) / kMarchW;
    const int nby = (hi[1] - lo[1] + kMarchTY - 1) / kMarchTY;
    const int nb = nbx * nby;
    hipLaunchKernelGGL((wsum_march_kernel<T, K, MASK>), dim3(nb), dim3(kMarchW), 0, s, d, lo[0], hi[0], lo[1], hi[1],
                       nbx, nb);
    return hipGetLastError();
}

template <typename T, int K>
hipError_t march_k(const LoopDesc &d, int mask, const int lo[3], const int hi[3], hipStream_t s) {
    switch (mask) {
#define M(m)                                                                     \
    case m:                                                                      \
        if constexpr ((m >> K) == 0) return go_march<T, K, m>(d, lo, hi, s);      \
        break;
        M(0) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15)
#undef M
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t wsum_t(const LoopDesc &d, const Box &b, int march_mask, hipStream_t s) {
    const int k = d.nargs - 1;
    if (march_mask >= 0 && d.ndim == 2 && b.hi[2] - b.lo[2] == 1) {
        switch (k) {
        case 1: return march_k<T, 1>(d, march_mask, b.lo, b.hi, s);
        case 2: return march_k<T, 2>(d, march_mask, b.lo, b.hi, s);
        case 3: return march_k<T, 3>(d, march_mask, b.lo, b.hi, s);
        case 4: return march_k<T, 4>(d, march_mask, b.lo, b.hi, s);
        default: break;
        }
    }
    hipLaunchKernelGGL(wsum_generic_kernel<T>, dim3(b.nb), dim3(kBlockThreads), 0, s, d, b);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_wsum(const LoopDesc &d, const Box &b, int dtype, int march_mask, hipStream_t s) {
    if (b.nb <= 0) return hipSuccess;
    return dtype == TC_F64 ? wsum_t<double>(d, b, march_mask, s) : wsum_t<float>(d, b, march_mask, s);
}

}  // namespace tc
