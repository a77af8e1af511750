// The fused-group kernel: one workgroup streams its owned block of the group's
// domain through every loop of the group, with each dataset's rows held in a
// ring buffer in LDS (see fused.hpp for the scheme).
//
// Workgroup: 128 columns x 2 thread rows; each thread computes P = 1, 2 or 4
// consecutive rows, so a step covers R = 2P rows.  Per step:
//   1. loaders issue the global loads for the NEXT step's rows (two register
//      sets alternate, so a load has a whole step to arrive),
//   2. every loop computes its R rows from the rings and writes its output
//      ring (lags guarantee no loop reads a row written in the same step),
//   3. storers write final rows of the owned block to the destination buffers,
//   4. the rows loaded during the previous step are written into their rings,
//   5. one workgroup barrier.
// Inputs read through a canonical radius-1/2 star take a fixed access
// pattern; other stencils walk their list of points.
#include <hip/hip_runtime.h>

#include <climits>

#include "fused.hpp"

namespace tc {

namespace {

__device__ __forceinline__ int xcd_linear(int i, int nb) {
    const int q = nb >> 3, r = nb & 7, xcd = i & 7, k = i >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

// row -> ring slot (row mod depth, non-negative) via a float estimate and
// one correction each way; rows stay far below 2^24.
__device__ __forceinline__ int slot_of(int row, int depth, float inv) {
    int q = (int)floorf((float)row * inv);
    int m = row - q * depth;
    m += (m < 0) ? depth : 0;
    m -= (m >= depth) ? depth : 0;
    return m;
}

__device__ __forceinline__ int wrap(int sl, int depth) {
    sl += (sl < 0) ? depth : 0;
    sl -= (sl >= depth) ? depth : 0;
    return sl;
}

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

// Global-memory views of descriptor pointers (so the compiler emits global,
// not flat, loads and stores and tracks their counters precisely).
template <typename T>
using gconst = const T __attribute__((address_space(1))) *;
template <typename T>
using gmut = T __attribute__((address_space(1))) *;

struct Blk {
    int X0, Y0, W, Hseg, HR, x, col, sub;
    uint32_t cload, cfw, cstore, cloop;  // per-thread column tests, one bit per ring / loop
};

// Rows handled by a thread at step s: R*s + sub*P + p - lag, p in [0, P).
template <typename T, int P>
__device__ __forceinline__ void issue_loads(const FGroupD *__restrict__ g, const Blk &b, int base,
                                            T (&buf)[kFMaxLoaded][P]) {
    // every lane loads a clamped, always valid address; write_loads decides
    // which values enter the ring
    const int nload = g->nload;
#pragma unroll
    for (int i = 0; i < kFMaxLoaded; ++i) {
        if (i < nload) {
            const FRingD &Rg = g->rings[g->load_list[i]];
            const int xc = min(max(b.x, Rg.ext_xlo), Rg.ext_xhi - 1);
            gconst<T> src = (gconst<T>)Rg.src + xc;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int y = min(max(base + p - Rg.load_lag, Rg.ext_ylo), Rg.ext_yhi - 1);
                buf[i][p] = src[(int64_t)y * Rg.sy];
            }
        }
    }
}

template <typename T, int P>
__device__ __forceinline__ void write_loads(const FGroupD *__restrict__ g, const Blk &b, int base, T *lds,
                                            const T (&buf)[kFMaxLoaded][P]) {
    const int nload = g->nload;
#pragma unroll
    for (int i = 0; i < kFMaxLoaded; ++i) {
        if (i < nload) {
            const int r = g->load_list[i];
            const FRingD &Rg = g->rings[r];
            const int ra = max(Rg.ext_ylo, b.Y0 - Rg.ld_below), rb = min(Rg.ext_yhi, b.Y0 + b.Hseg + Rg.ld_above);
            const bool col = (b.cload >> r) & 1u;
            const bool fwc = Rg.load == 2 && ((b.cfw >> r) & 1u);
            const int y0 = base - Rg.load_lag;
            int sl = slot_of(y0, Rg.depth, Rg.inv_depth);
            T *ring = lds + Rg.lds_off + b.col;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int y = y0 + p;
                const bool ok = col && y >= ra && y < rb && !(fwc && y >= Rg.fw_ylo && y < Rg.fw_yhi);
                if (ok) ring[sl * kFCols] = buf[i][p];
                sl = wrap(sl + 1, Rg.depth);
            }
        }
    }
}

template <typename T, int P>
__device__ __forceinline__ void compute_and_store(const FGroupD *__restrict__ g, const Blk &b, int base, T *lds) {
    const int nloops = g->nloops;
    for (int l = 0; l < nloops; ++l) {
        const FLoopD &L = g->loops[l];
        const int ya = max(L.ylo, b.Y0 - L.vlo), yb = min(L.yhi, b.Y0 + b.Hseg + L.vhi);
        const int y0 = base - L.lag;
        if (y0 + P <= ya || y0 >= yb) continue;  // uniform across the thread row
        const bool col = (b.cloop >> l) & 1u;
        T acc[P];
#pragma unroll
        for (int p = 0; p < P; ++p) acc[p] = (T)0;
        for (int i = 0; i < L.nin; ++i) {
            const FInD I = g->ins[L.in0 + i];
            const FRingD &Rg = g->rings[I.ring];
            const int depth = Rg.depth;
            const int s0 = slot_of(y0, depth, Rg.inv_depth);
            const T *ring = lds + Rg.lds_off + b.col;
            const double *w = g->w + I.ent0;
            if (I.star) {
                const int r = I.star;
                // column values of rows y0-r .. y0+P-1+r, then the x neighbours of each row
                T cv[P + 4];
#pragma unroll
                for (int j = 0; j < P + 4; ++j)
                    if (j < P + 2 * r) cv[j] = ring[wrap(s0 + j - r, depth) * kFCols];
                T xn[P][4];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const T *c = ring + wrap(s0 + p, depth) * kFCols;
                    xn[p][0] = c[-1];
                    xn[p][1] = c[1];
                    if (r == 2) {
                        xn[p][2] = c[-2];
                        xn[p][3] = c[2];
                    }
                }
                const T w0 = (T)w[0], w1 = (T)w[1], w2 = (T)w[2], w3 = (T)w[3], w4 = (T)w[4];
                if (r == 1) {
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        T a = acc[p];
                        a = fmaT<T>(w0, cv[p + 1], a);
                        a = fmaT<T>(w1, xn[p][0], a);
                        a = fmaT<T>(w2, xn[p][1], a);
                        a = fmaT<T>(w3, cv[p], a);
                        a = fmaT<T>(w4, cv[p + 2], a);
                        acc[p] = a;
                    }
                } else {
                    const T w5 = (T)w[5], w6 = (T)w[6], w7 = (T)w[7], w8 = (T)w[8];
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        T a = acc[p];
                        a = fmaT<T>(w0, cv[p + 2], a);
                        a = fmaT<T>(w1, xn[p][0], a);
                        a = fmaT<T>(w2, xn[p][1], a);
                        a = fmaT<T>(w3, xn[p][2], a);
                        a = fmaT<T>(w4, xn[p][3], a);
                        a = fmaT<T>(w5, cv[p + 1], a);
                        a = fmaT<T>(w6, cv[p + 3], a);
                        a = fmaT<T>(w7, cv[p], a);
                        a = fmaT<T>(w8, cv[p + 4], a);
                        acc[p] = a;
                    }
                }
            } else {
                for (int k = 0; k < I.nent; ++k) {
                    const FEnt E = g->ent[I.ent0 + k];
                    const T wk = (T)w[k];
#pragma unroll
                    for (int p = 0; p < P; ++p)
                        acc[p] = fmaT<T>(wk, ring[wrap(s0 + p + E.dy, depth) * kFCols + E.dx], acc[p]);
                }
            }
        }
        const FRingD &O = g->rings[L.out_ring];
        T *out = lds + O.lds_off + b.col;
        int so = slot_of(y0, O.depth, O.inv_depth);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int y = y0 + p;
            if (col && y >= ya && y < yb) out[so * kFCols] = acc[p];
            so = wrap(so + 1, O.depth);
        }
    }
    const int nstore = g->nstore;
    for (int i = 0; i < nstore; ++i) {
        const int r = g->store_list[i];
        const FRingD &Rg = g->rings[r];
        const int ya = max(Rg.hull_ylo, b.Y0), yb = min(Rg.hull_yhi, b.Y0 + b.Hseg);
        const int y0 = base - Rg.store_lag;
        if (y0 + P <= ya || y0 >= yb) continue;
        const bool col = (b.cstore >> r) & 1u;
        const T *ring = lds + Rg.lds_off + b.col;
        gmut<T> dst = (gmut<T>)Rg.dst + b.x;
        int sl = slot_of(y0, Rg.depth, Rg.inv_depth);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int y = y0 + p;
            if (col && y >= ya && y < yb) dst[(int64_t)y * Rg.sy] = ring[sl * kFCols];
            sl = wrap(sl + 1, Rg.depth);
        }
    }
}

template <int R>
__device__ __forceinline__ int floor_div(int v) {
    return v >= 0 ? v / R : -((-v + R - 1) / R);
}

template <typename T, int P>
__global__ void __launch_bounds__(kFCols * kFThreadRows) fused_kernel(const FGroupD *__restrict__ g) {
    constexpr int R = kFThreadRows * P;
    extern __shared__ __align__(16) unsigned char smem[];
    T *lds = (T *)smem;
    Blk b;
    b.W = g->W;
    b.HR = g->HR;
    b.Hseg = g->Hseg;
    const int lin = xcd_linear(blockIdx.x, gridDim.x);
    const int bx = lin % g->nbx, by = lin / g->nbx;
    b.X0 = g->dom_xlo + bx * b.W;
    b.Y0 = g->dom_ylo + by * b.Hseg;
    b.col = threadIdx.x & (kFCols - 1);
    b.sub = threadIdx.x / kFCols;
    b.x = b.X0 - b.HR + b.col;

    // per-thread column tests and the step range covering every agent
    b.cload = b.cfw = b.cstore = b.cloop = 0u;
    int s_lo = INT_MAX, s_hi = INT_MIN;
    for (int l = 0; l < g->nloops; ++l) {
        const FLoopD &L = g->loops[l];
        if (b.x >= max(L.xlo, b.X0 - L.hlo) && b.x < min(L.xhi, b.X0 + b.W + L.hhi)) b.cloop |= 1u << l;
        const int a = max(L.ylo, b.Y0 - L.vlo), e = min(L.yhi, b.Y0 + b.Hseg + L.vhi);
        if (a < e) {
            s_lo = min(s_lo, floor_div<R>(a + L.lag));
            s_hi = max(s_hi, floor_div<R>(e - 1 + L.lag));
        }
    }
    for (int r = 0; r < g->nrings; ++r) {
        const FRingD &Rg = g->rings[r];
        if (b.x >= Rg.ext_xlo && b.x < Rg.ext_xhi) b.cload |= 1u << r;
        if (b.x >= Rg.fw_xlo && b.x < Rg.fw_xhi) b.cfw |= 1u << r;
        if (b.x >= max(Rg.hull_xlo, b.X0) && b.x < min(Rg.hull_xhi, b.X0 + b.W)) b.cstore |= 1u << r;
        if (Rg.load) {
            const int a = max(Rg.ext_ylo, b.Y0 - Rg.ld_below), e = min(Rg.ext_yhi, b.Y0 + b.Hseg + Rg.ld_above);
            if (a < e) {
                s_lo = min(s_lo, floor_div<R>(a + Rg.load_lag));
                s_hi = max(s_hi, floor_div<R>(e - 1 + Rg.load_lag));
            }
        }
        if (Rg.store) {
            const int a = max(Rg.hull_ylo, b.Y0), e = min(Rg.hull_yhi, b.Y0 + b.Hseg);
            if (a < e) {
                s_lo = min(s_lo, floor_div<R>(a + Rg.store_lag));
                s_hi = max(s_hi, floor_div<R>(e - 1 + Rg.store_lag));
            }
        }
    }
    if (s_lo > s_hi) return;  // uniform: nothing to do for this block

    const int sub0 = b.sub * P;
    T bufA[kFMaxLoaded][P], bufB[kFMaxLoaded][P];
    issue_loads<T, P>(g, b, R * s_lo + sub0, bufA);
    for (int s = s_lo; s <= s_hi; s += 2) {
        issue_loads<T, P>(g, b, R * (s + 1) + sub0, bufB);
        compute_and_store<T, P>(g, b, R * s + sub0, lds);
        write_loads<T, P>(g, b, R * s + sub0, lds, bufA);
        __syncthreads();
        if (s + 1 > s_hi) break;
        issue_loads<T, P>(g, b, R * (s + 2) + sub0, bufA);
        compute_and_store<T, P>(g, b, R * (s + 1) + sub0, lds);
        write_loads<T, P>(g, b, R * (s + 1) + sub0, lds, bufB);
        __syncthreads();
    }
}

template <typename T, int P>
hipError_t go(const FGroupD *dev_desc, int nblocks, int lds_bytes, hipStream_t s) {
    hipError_t e = hipFuncSetAttribute((const void *)fused_kernel<T, P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fused_kernel<T, P>), dim3(nblocks), dim3(kFCols * kFThreadRows), lds_bytes, s, dev_desc);
    return hipGetLastError();
}

template <typename T>
hipError_t go_rows(const FGroupD *dev_desc, int rows, int nblocks, int lds_bytes, hipStream_t s) {
    switch (rows) {
    case 2: return go<T, 1>(dev_desc, nblocks, lds_bytes, s);
    case 8: return go<T, 4>(dev_desc, nblocks, lds_bytes, s);
    default: return go<T, 2>(dev_desc, nblocks, lds_bytes, s);
    }
}

}  // namespace

hipError_t launch_fused(const FGroupD *dev_desc, int dtype, int rows, int nblocks, int lds_bytes, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    return dtype == TC_F64 ? go_rows<double>(dev_desc, rows, nblocks, lds_bytes, s)
                           : go_rows<float>(dev_desc, rows, nblocks, lds_bytes, s);
}

}  // namespace tc
