// The fused-group kernel: one workgroup streams its owned block of the group's
// domain through every loop of the group, with each dataset's rows held in a
// ring buffer in LDS (see fused.hpp for the scheme).
//
// Workgroup: 256 threads = 128 columns x 2 rows.  Per step (two rows):
//   1. loaders issue the global loads of their next rows (kept in registers),
//   2. every loop computes its row pair from the rings and writes its output
//      ring (lags guarantee no loop reads a row written in the same step),
//   3. storers write final rows of the owned block to the destination buffers,
//   4. loaded values are written into their rings,
//   5. one workgroup barrier.
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

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

template <typename T>
__global__ void __launch_bounds__(kFThreads) fused_kernel(const FGroupD *__restrict__ g) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *lds = (T *)smem;
    const int nloops = g->nloops, nrings = g->nrings;
    const int W = g->W, HR = g->HR, Hseg = g->Hseg;
    const int lin = xcd_linear(blockIdx.x, gridDim.x);
    const int bx = lin % g->nbx, by = lin / g->nbx;
    const int X0 = g->dom_xlo + bx * W, Y0 = g->dom_ylo + by * Hseg;
    const int col = threadIdx.x & (kFCols - 1);
    const int sub = threadIdx.x / kFCols;
    const int x = X0 - HR + col;

    // step range covering every loader, loop and storer of this block
    int s_lo = INT_MAX, s_hi = INT_MIN;
    for (int l = 0; l < nloops; ++l) {
        const FLoopD &L = g->loops[l];
        const int a = max(L.ylo, Y0 - L.vlo), b = min(L.yhi, Y0 + Hseg + L.vhi);
        if (a < b) {
            s_lo = min(s_lo, (a + L.lag) >> 1);
            s_hi = max(s_hi, (b - 1 + L.lag) >> 1);
        }
    }
    for (int r = 0; r < nrings; ++r) {
        const FRingD &Rg = g->rings[r];
        if (Rg.load) {
            const int a = max(Rg.ext_ylo, Y0 - Rg.ld_below), b = min(Rg.ext_yhi, Y0 + Hseg + Rg.ld_above);
            if (a < b) {
                s_lo = min(s_lo, (a + Rg.load_lag) >> 1);
                s_hi = max(s_hi, (b - 1 + Rg.load_lag) >> 1);
            }
        }
        if (Rg.store) {
            const int a = max(Rg.hull_ylo, Y0), b = min(Rg.hull_yhi, Y0 + Hseg);
            if (a < b) {
                s_lo = min(s_lo, (a + Rg.store_lag) >> 1);
                s_hi = max(s_hi, (b - 1 + Rg.store_lag) >> 1);
            }
        }
    }

    T ldv[kFMaxRings];
    for (int s = s_lo; s <= s_hi; ++s) {
        const int base = 2 * s + sub;  // row of an agent with lag 0
        // 1. loaders: global loads of the next rows
#pragma unroll
        for (int r = 0; r < kFMaxRings; ++r) {
            const FRingD &Rg = g->rings[r];
            if (r < nrings && Rg.load) {
                const int y = base - Rg.load_lag;
                bool ok = y >= max(Rg.ext_ylo, Y0 - Rg.ld_below) && y < min(Rg.ext_yhi, Y0 + Hseg + Rg.ld_above) &&
                          x >= Rg.ext_xlo && x < Rg.ext_xhi;
                if (Rg.load == 2)
                    ok = ok && !(x >= Rg.fw_xlo && x < Rg.fw_xhi && y >= Rg.fw_ylo && y < Rg.fw_yhi);
                if (ok) ldv[r] = ((const T *)Rg.src)[(int64_t)y * Rg.sy + x];
            }
        }
        // 2. loops
        for (int l = 0; l < nloops; ++l) {
            const FLoopD &L = g->loops[l];
            const int y = base - L.lag;
            const bool ok = y >= max(L.ylo, Y0 - L.vlo) && y < min(L.yhi, Y0 + Hseg + L.vhi) &&
                            x >= max(L.xlo, X0 - L.hlo) && x < min(L.xhi, X0 + W + L.hhi);
            if (!ok) continue;
            T acc = (T)0;
            for (int i = 0; i < L.nin; ++i) {
                const FInD &I = g->ins[L.in0 + i];
                const FRingD &Rg = g->rings[I.ring];
                const int depth = Rg.depth;
                const int s0 = slot_of(y, depth, Rg.inv_depth);
                const T *ring = lds + Rg.lds_off + col;
                int k = 0;
                // batches of four points: four LDS reads, then four fmas in order
                for (; k + 4 <= I.nent; k += 4) {
                    T v[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const FEnt E = g->ent[I.ent0 + k + j];
                        int sl = s0 + E.dy;
                        sl += (sl < 0) ? depth : 0;
                        sl -= (sl >= depth) ? depth : 0;
                        v[j] = ring[sl * kFCols + E.dx];
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc = fmaT<T>((T)g->w[I.ent0 + k + j], v[j], acc);
                }
                for (; k < I.nent; ++k) {
                    const FEnt E = g->ent[I.ent0 + k];
                    int sl = s0 + E.dy;
                    sl += (sl < 0) ? depth : 0;
                    sl -= (sl >= depth) ? depth : 0;
                    acc = fmaT<T>((T)g->w[I.ent0 + k], ring[sl * kFCols + E.dx], acc);
                }
            }
            const FRingD &O = g->rings[L.out_ring];
            lds[O.lds_off + slot_of(y, O.depth, O.inv_depth) * kFCols + col] = acc;
        }
        // 3. storers
        for (int r = 0; r < nrings; ++r) {
            const FRingD &Rg = g->rings[r];
            if (!Rg.store) continue;
            const int y = base - Rg.store_lag;
            if (y >= max(Rg.hull_ylo, Y0) && y < min(Rg.hull_yhi, Y0 + Hseg) && x >= max(Rg.hull_xlo, X0) &&
                x < min(Rg.hull_xhi, X0 + W))
                ((T *)Rg.dst)[(int64_t)y * Rg.sy + x] = lds[Rg.lds_off + slot_of(y, Rg.depth, Rg.inv_depth) * kFCols + col];
        }
        // 4. loaded rows into their rings
#pragma unroll
        for (int r = 0; r < kFMaxRings; ++r) {
            const FRingD &Rg = g->rings[r];
            if (r < nrings && Rg.load) {
                const int y = base - Rg.load_lag;
                bool ok = y >= max(Rg.ext_ylo, Y0 - Rg.ld_below) && y < min(Rg.ext_yhi, Y0 + Hseg + Rg.ld_above) &&
                          x >= Rg.ext_xlo && x < Rg.ext_xhi;
                if (Rg.load == 2)
                    ok = ok && !(x >= Rg.fw_xlo && x < Rg.fw_xhi && y >= Rg.fw_ylo && y < Rg.fw_yhi);
                if (ok) lds[Rg.lds_off + slot_of(y, Rg.depth, Rg.inv_depth) * kFCols + col] = ldv[r];
            }
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_fused(const FGroupD *dev_desc, int dtype, int nblocks, int lds_bytes, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    if (dtype == TC_F64) {
        hipError_t e = hipFuncSetAttribute((const void *)fused_kernel<double>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(fused_kernel<double>, dim3(nblocks), dim3(kFThreads), lds_bytes, s, dev_desc);
    } else {
        hipError_t e = hipFuncSetAttribute((const void *)fused_kernel<float>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(fused_kernel<float>, dim3(nblocks), dim3(kFThreads), lds_bytes, s, dev_desc);
    }
    return hipGetLastError();
}

}  // namespace tc
