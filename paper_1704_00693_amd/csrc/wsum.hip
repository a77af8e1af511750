// Weighted-sum loop kernels (TC_OP_WSUM) for one box of the iteration range.
//
// Two variants, both with the arithmetic order of the op's definition
// (acc = fma(w, v, acc) over inputs and stencil points in listed order):
//
//  * march: 2D, every input read through a radius-1 or radius-2 star stencil
//    listed in the canonical order (centre, -x, +x, [-2x, +2x,] -y, +y,
//    [-2y, +2y]).  A workgroup covers 240 consecutive x (four wavefronts of
//    60 output columns plus two halo columns per side) and marches TY rows
//    up y; each lane keeps the vertical window of every input in registers
//    (one new row load per input per output row, issued one row ahead) and
//    takes its x neighbours from adjacent lanes with DPP lane moves, so
//    global loads per output point drop from sum(stencil points) to about
//    the number of inputs and no load is conditional.
//  * point: 2D or 3D, every input read at its centre only (a scaled copy
//    or a pointwise combination of up to four datasets).  Each lane computes
//    kPointRows rows of one column and issues all their loads before the
//    first fma chain, so four loads per input are in flight per lane.
//  * generic: any stencils and dimensions; all loads of a point are issued
//    before its fma chain so one memory latency covers the whole point.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "lanes.hpp"

namespace tc {

namespace {

constexpr int kMarchW = 256;                 // threads per workgroup (4 wavefronts side by side in x)
constexpr int kWaveOut = 60;                 // output columns per wavefront
constexpr int kMarchOut = 4 * kWaveOut;      // output columns per workgroup
constexpr int kMarchBatch = 4;               // rows computed per batch (loaded one batch ahead)

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}


// XCD-aware workgroup order: hardware block i runs on XCD i % 8; XCD k gets
// the contiguous logical block range starting at k*q + min(k, r).
__device__ __forceinline__ int xcd_linear(int i, int nb) {
    const int q = nb >> 3, r = nb & 7, xcd = i & 7, k = i >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

template <typename T, int K, int MASK>
__global__ void __launch_bounds__(kMarchW) wsum_march_kernel(LoopDesc d, int lo0, int hi0, int lo1, int hi1, int nbx,
                                                             int nb, int ty) {
    constexpr int TB = kMarchBatch;
    const int lin = xcd_linear(blockIdx.x, nb);
    const int bx = lin % nbx, by = lin / nbx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // each wavefront produces 60 columns; lanes 0-1 and 62-63 hold the x halo
    const int xw = lo0 + bx * kMarchOut + wave * kWaveOut;
    const int x = xw - 2 + lane;
    const bool active = lane >= 2 && lane < 62 && x < hi0;
    const int y0 = lo1 + by * ty;
    const int y1 = min(y0 + ty, hi1);

    const T *ptr[K];
    int64_t sy[K];
    // win[a][j] holds row y - 2 + j of input a for the batch starting at y;
    // pf[a][t] holds row y + TB + r + t, loaded while batch y is computed
    T win[K][TB + 4];
    T pf[K][TB];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const int r = (MASK >> a) & 1 ? 2 : 1;
        // columns outside this input's reach are clamped; no output uses them
        const int xc = min(max(x, lo0 - r), hi0 - 1 + r);
        sy[a] = d.arg[a + 1].sy;
        ptr[a] = (const T *)d.arg[a + 1].ptr + xc;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j >= 2 - r && j < 2 + r) win[a][j] = ptr[a][(int64_t)(y0 - 2 + j) * sy[a]];
#pragma unroll
        for (int t = 0; t < TB; ++t)
            if (y0 + r + t <= y1 - 1 + r) pf[a][t] = ptr[a][(int64_t)(y0 + r + t) * sy[a]];
    }
    T *out = (T *)d.arg[0].ptr + x;
    const int64_t osy = d.arg[0].sy;
    for (int y = y0; y < y1; y += TB) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int r = (MASK >> a) & 1 ? 2 : 1;
#pragma unroll
            for (int t = 0; t < TB; ++t) win[a][2 + r + t] = pf[a][t];
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const int row = y + TB + r + t;
                if (row <= y1 - 1 + r) pf[a][t] = ptr[a][(int64_t)row * sy[a]];
            }
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            T acc = (T)0;
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const int r = (MASK >> a) & 1 ? 2 : 1;
                const T c = win[a][2 + t];
                const T xm1 = lane_prev(c), xp1 = lane_next(c);
                const int q = d.pt0[a + 1];
                if (r == 1) {
                    acc = fmaT<T>((T)d.prm[q + 0], c, acc);
                    acc = fmaT<T>((T)d.prm[q + 1], xm1, acc);
                    acc = fmaT<T>((T)d.prm[q + 2], xp1, acc);
                    acc = fmaT<T>((T)d.prm[q + 3], win[a][1 + t], acc);
                    acc = fmaT<T>((T)d.prm[q + 4], win[a][3 + t], acc);
                } else {
                    const T xm2 = lane_prev(xm1), xp2 = lane_next(xp1);
                    acc = fmaT<T>((T)d.prm[q + 0], c, acc);
                    acc = fmaT<T>((T)d.prm[q + 1], xm1, acc);
                    acc = fmaT<T>((T)d.prm[q + 2], xp1, acc);
                    acc = fmaT<T>((T)d.prm[q + 3], xm2, acc);
                    acc = fmaT<T>((T)d.prm[q + 4], xp2, acc);
                    acc = fmaT<T>((T)d.prm[q + 5], win[a][1 + t], acc);
                    acc = fmaT<T>((T)d.prm[q + 6], win[a][3 + t], acc);
                    acc = fmaT<T>((T)d.prm[q + 7], win[a][t], acc);
                    acc = fmaT<T>((T)d.prm[q + 8], win[a][4 + t], acc);
                }
            }
            if (active && y + t < y1) out[(int64_t)(y + t) * osy] = acc;
        }
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) win[a][j] = win[a][j + TB];
    }
}

// 3D: a workgroup covers 60 columns x NW rows (one wavefront per row, lanes
// as in the 2D march) and marches up z over `tz` planes.  Each lane keeps the
// z window of its own column for every input in registers; x neighbours come
// from adjacent lanes.  For the y neighbours every wavefront puts the centre
// value of its own row into LDS, and wavefronts 0-3 also that of one of the
// four rows just outside the workgroup (y0-2, y0-1, y0+NW, y0+NW+1; loaded
// one batch ahead), where the workgroup's rows read them (one barrier per
// plane, two LDS buffers).  Taller workgroups load fewer outside rows per
// output row (4 per NW).
template <typename T, int K, int MASK, int NW>
__global__ void __launch_bounds__(64 * NW) wsum_march3_kernel(LoopDesc d, int lo0, int hi0, int lo1, int hi1, int lo2,
                                                              int hi2, int nbx, int nby, int nb, int tz) {
    constexpr int TB = kMarchBatch;
    static_assert(TB % 2 == 0, "the LDS buffer of a plane alternates with its parity");
    static_assert(NW >= 4, "wavefronts 0-3 carry the four outside rows");
    __shared__ T yl[2][K][NW + 4][64];
    const int lin = xcd_linear(blockIdx.x, nb);
    const int bx = lin % nbx, rest = lin / nbx, by = rest % nby, bz = rest / nby;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: branches on it stay scalar
    const int x = lo0 + bx * kWaveOut - 2 + lane;
    const int y0 = lo1 + by * NW;
    const int y = y0 + wave;
    const bool active = lane >= 2 && lane < 62 && x < hi0 && y < hi1;
    const int z0 = lo2 + bz * tz;
    const int z1 = min(z0 + tz, hi2);
    const bool outer = wave < 4;                    // this wavefront also carries an outside row
    const int hslot = wave < 2 ? wave : NW + wave;  // its LDS row (rows y0-2, y0-1, y0+NW, y0+NW+1)

    const T *ptr[K];
    const T *optr[K];
    int64_t sz[K];
    T win[K][TB + 4];
    T pf[K][TB];
    T ob[K][TB];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const int r = (MASK >> a) & 1 ? 2 : 1;
        // rows y0-2 and y0+NW+1 are read through radius-2 stencils only
        const bool oa = outer && (r == 2 || (hslot != 0 && hslot != NW + 3));
        // Positions are clamped to the input's reach [lo - r, hi - 1 + r]:
        // whenever an output reads a position, it lies in that reach and is
        // not moved; clamped ones feed no output.
        const int xc = min(max(x, lo0 - r), hi0 - 1 + r);
        const int yc = min(y, hi1 - 1 + r);
        const int yh = min(y0 - 2 + hslot, hi1 - 1 + r);
        const int64_t sy = d.arg[a + 1].sy;
        sz[a] = d.arg[a + 1].sz;
        ptr[a] = (const T *)d.arg[a + 1].ptr + xc + (int64_t)yc * sy;
        optr[a] = (const T *)d.arg[a + 1].ptr + xc + (int64_t)yh * sy;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j >= 2 - r && j < 2 + r) win[a][j] = ptr[a][(int64_t)(z0 - 2 + j) * sz[a]];
        // planes past the input's reach are clamped onto its last plane: no
        // output reads them, and no load is conditional on the plane
#pragma unroll
        for (int t = 0; t < TB; ++t) pf[a][t] = ptr[a][(int64_t)min(z0 + r + t, z1 - 1 + r) * sz[a]];
#pragma unroll
        for (int t = 0; t < TB; ++t)
            if (oa) ob[a][t] = optr[a][(int64_t)min(z0 + t, z1 - 1) * sz[a]];
    }
    T *out = (T *)d.arg[0].ptr + x + (int64_t)min(y, hi1 - 1) * d.arg[0].sy;
    const int64_t osz = d.arg[0].sz;
    for (int z = z0; z < z1; z += TB) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int r = (MASK >> a) & 1 ? 2 : 1;
#pragma unroll
            for (int t = 0; t < TB; ++t) win[a][2 + r + t] = pf[a][t];
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                pf[a][t] = ptr[a][(int64_t)min(z + TB + r + t, z1 - 1 + r) * sz[a]];
            }
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const int buf = t & 1;
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const int r = (MASK >> a) & 1 ? 2 : 1;
                const bool oa = outer && (r == 2 || (hslot != 0 && hslot != NW + 3));
                yl[buf][a][wave + 2][lane] = win[a][2 + t];
                if (outer) yl[buf][a][hslot][lane] = ob[a][t];
                // the outside row of plane z + t is in LDS: load the one TB planes on
                if (oa) ob[a][t] = optr[a][(int64_t)min(z + TB + t, z1 - 1) * sz[a]];
            }
            __syncthreads();
            T acc = (T)0;
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const int r = (MASK >> a) & 1 ? 2 : 1;
                const T c = win[a][2 + t];
                const T xm1 = lane_prev(c), xp1 = lane_next(c);
                const T ym1 = yl[buf][a][wave + 1][lane], yp1 = yl[buf][a][wave + 3][lane];
                const int q = d.pt0[a + 1];
                if (r == 1) {
                    acc = fmaT<T>((T)d.prm[q + 0], c, acc);
                    acc = fmaT<T>((T)d.prm[q + 1], xm1, acc);
                    acc = fmaT<T>((T)d.prm[q + 2], xp1, acc);
                    acc = fmaT<T>((T)d.prm[q + 3], ym1, acc);
                    acc = fmaT<T>((T)d.prm[q + 4], yp1, acc);
                    acc = fmaT<T>((T)d.prm[q + 5], win[a][1 + t], acc);
                    acc = fmaT<T>((T)d.prm[q + 6], win[a][3 + t], acc);
                } else {
                    const T xm2 = lane_prev(xm1), xp2 = lane_next(xp1);
                    const T ym2 = yl[buf][a][wave][lane], yp2 = yl[buf][a][wave + 4][lane];
                    acc = fmaT<T>((T)d.prm[q + 0], c, acc);
                    acc = fmaT<T>((T)d.prm[q + 1], xm1, acc);
                    acc = fmaT<T>((T)d.prm[q + 2], xp1, acc);
                    acc = fmaT<T>((T)d.prm[q + 3], xm2, acc);
                    acc = fmaT<T>((T)d.prm[q + 4], xp2, acc);
                    acc = fmaT<T>((T)d.prm[q + 5], ym1, acc);
                    acc = fmaT<T>((T)d.prm[q + 6], yp1, acc);
                    acc = fmaT<T>((T)d.prm[q + 7], ym2, acc);
                    acc = fmaT<T>((T)d.prm[q + 8], yp2, acc);
                    acc = fmaT<T>((T)d.prm[q + 9], win[a][1 + t], acc);
                    acc = fmaT<T>((T)d.prm[q + 10], win[a][3 + t], acc);
                    acc = fmaT<T>((T)d.prm[q + 11], win[a][t], acc);
                    acc = fmaT<T>((T)d.prm[q + 12], win[a][4 + t], acc);
                }
            }
            if (active && z + t < z1) out[(int64_t)(z + t) * osz] = acc;
        }
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) win[a][j] = win[a][j + TB];
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

constexpr int kPointRows = 4;  // rows per lane of the point variant

// b: the launch box with nby counting groups of bh * kPointRows rows.
template <typename T, int K>
__global__ void __launch_bounds__(kBlockThreads) wsum_point_kernel(LoopDesc d, Box b) {
    const int lin = xcd_linear(blockIdx.x, b.nb);
    const int bx = lin % b.nbx;
    const int rest = lin / b.nbx;
    const int by = rest % b.nby;
    const int bz = rest / b.nby;
    const int x = b.lo[0] + bx * b.bw + (int)(threadIdx.x % b.bw);
    const int y0 = b.lo[1] + by * b.bh * kPointRows + (int)(threadIdx.x / b.bw);
    const int z = b.lo[2] + bz;
    if (x >= b.hi[0]) return;
    T v[kPointRows][K];
#pragma unroll
    for (int r = 0; r < kPointRows; ++r) {
        const int y = y0 + r * b.bh;
        if (y < b.hi[1]) {
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const T *p = (const T *)d.arg[a + 1].ptr;
                v[r][a] = p[(int64_t)x + (int64_t)y * d.arg[a + 1].sy + (int64_t)z * d.arg[a + 1].sz];
            }
        }
    }
    T *o = (T *)d.arg[0].ptr;
#pragma unroll
    for (int r = 0; r < kPointRows; ++r) {
        const int y = y0 + r * b.bh;
        if (y < b.hi[1]) {
            T acc = (T)0;
#pragma unroll
            for (int a = 0; a < K; ++a) acc = fmaT<T>((T)d.prm[d.pt0[a + 1]], v[r][a], acc);
            o[(int64_t)x + (int64_t)y * d.arg[0].sy + (int64_t)z * d.arg[0].sz] = acc;
        }
    }
}

// True if every input of the weighted sum is read at its centre only.
bool centre_only_inputs(const LoopDesc &d) {
    for (int a = 1; a < d.nargs; ++a)
        if (d.npts[a] != 1 || d.off[d.pt0[a]] != 0) return false;
    return d.nargs >= 2;
}

template <typename T, int K>
hipError_t go_point(const LoopDesc &d, const Box &b, hipStream_t s) {
    Box p = b;
    const int ny = b.hi[1] - b.lo[1], nz = b.hi[2] - b.lo[2];
    p.nby = (ny + b.bh * kPointRows - 1) / (b.bh * kPointRows);
    p.nb = p.nbx * p.nby * nz;
    hipLaunchKernelGGL((wsum_point_kernel<T, K>), dim3(p.nb), dim3(kBlockThreads), 0, s, d, p);
    return hipGetLastError();
}

template <typename T, int K, int MASK>
hipError_t go_march(const LoopDesc &d, const int lo[3], const int hi[3], int ty, hipStream_t s) {
    const int nbx = (hi[0] - lo[0] + kMarchOut - 1) / kMarchOut;
    const int nby = (hi[1] - lo[1] + ty - 1) / ty;
    const int nb = nbx * nby;
    hipLaunchKernelGGL((wsum_march_kernel<T, K, MASK>), dim3(nb), dim3(kMarchW), 0, s, d, lo[0], hi[0], lo[1], hi[1],
                       nbx, nb, ty);
    return hipGetLastError();
}

// Planes per workgroup: the given count, or (0) the largest of 128, 64, 32
// that still makes about 1000 workgroups (four per CU).  Longer marches
// re-read fewer z-halo planes; measured on a 384^3 chain: 128 planes 27.9 ms,
// 64 28.2, 32 28.7, 192 29.8 (too few workgroups to balance).
template <typename T, int K, int MASK, int NW>
hipError_t go_march3_nw(const LoopDesc &d, const int lo[3], const int hi[3], int tz, hipStream_t s) {
    const int nbx = (hi[0] - lo[0] + kWaveOut - 1) / kWaveOut;
    const int nby = (hi[1] - lo[1] + NW - 1) / NW;
    const int nz = hi[2] - lo[2];
    if (tz <= 0) {
        tz = 128;
        while (tz > 32 && (int64_t)nbx * nby * ((nz + tz - 1) / tz) < 1000) tz /= 2;
    }
    const int nbz = (nz + tz - 1) / tz;
    const int nb = nbx * nby * nbz;
    hipLaunchKernelGGL((wsum_march3_kernel<T, K, MASK, NW>), dim3(nb), dim3(64 * NW), 0, s, d, lo[0], hi[0], lo[1],
                       hi[1], lo[2], hi[2], nbx, nby, nb, tz);
    return hipGetLastError();
}

template <typename T, int K, int MASK>
hipError_t go_march3(const LoopDesc &d, const int lo[3], const int hi[3], const MarchShape &ms, hipStream_t s) {
    // rows: the given 4 or 8, or (0) 8 unless that leaves fewer than about
    // 1000 workgroups of 32 planes (thin boxes, as skewed tiles launch)
    int rows = ms.rows3;
    if (rows != 4 && rows != 8) {
        const int64_t nb8 = (int64_t)((hi[0] - lo[0] + kWaveOut - 1) / kWaveOut) * ((hi[1] - lo[1] + 7) / 8) *
                            ((hi[2] - lo[2] + 31) / 32);
        rows = nb8 >= 1000 ? 8 : 4;
    }
    return rows == 4 ? go_march3_nw<T, K, MASK, 4>(d, lo, hi, ms.tz3, s)
                     : go_march3_nw<T, K, MASK, 8>(d, lo, hi, ms.tz3, s);
}

template <typename T, int K, int MASK>
hipError_t go_march_nd(const LoopDesc &d, const int lo[3], const int hi[3], const MarchShape &ms, hipStream_t s) {
    return d.ndim == 3 ? go_march3<T, K, MASK>(d, lo, hi, ms, s) : go_march<T, K, MASK>(d, lo, hi, ms.ty, s);
}

template <typename T, int K>
hipError_t march_k(const LoopDesc &d, int mask, const int lo[3], const int hi[3], const MarchShape &ms, hipStream_t s) {
    switch (mask) {
#define M(m)                                                                        \
    case m:                                                                         \
        if constexpr ((m >> K) == 0) return go_march_nd<T, K, m>(d, lo, hi, ms, s);  \
        break;
        M(0) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15)
#undef M
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t wsum_t(const LoopDesc &d, const Box &b, int march_mask, const MarchShape &ms, hipStream_t s) {
    const int k = d.nargs - 1;
    if (march_mask >= 0 && ((d.ndim == 2 && b.hi[2] - b.lo[2] == 1) || d.ndim == 3)) {
        switch (k) {
        case 1: return march_k<T, 1>(d, march_mask, b.lo, b.hi, ms, s);
        case 2: return march_k<T, 2>(d, march_mask, b.lo, b.hi, ms, s);
        case 3: return march_k<T, 3>(d, march_mask, b.lo, b.hi, ms, s);
        case 4: return march_k<T, 4>(d, march_mask, b.lo, b.hi, ms, s);
        default: break;
        }
    }
    if (d.ndim >= 2 && b.hi[1] - b.lo[1] > 1 && b.bw * b.bh == kBlockThreads && centre_only_inputs(d)) {
        switch (d.nargs - 1) {
        case 1: return go_point<T, 1>(d, b, s);
        case 2: return go_point<T, 2>(d, b, s);
        case 3: return go_point<T, 3>(d, b, s);
        case 4: return go_point<T, 4>(d, b, s);
        default: break;
        }
    }
    hipLaunchKernelGGL(wsum_generic_kernel<T>, dim3(b.nb), dim3(kBlockThreads), 0, s, d, b);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_wsum(const LoopDesc &d, const Box &b, int dtype, int march_mask, const MarchShape &ms, hipStream_t s) {
    if (b.nb <= 0) return hipSuccess;
    return dtype == TC_F64 ? wsum_t<double>(d, b, march_mask, ms, s) : wsum_t<float>(d, b, march_mask, ms, s);
}

}  // namespace tc
