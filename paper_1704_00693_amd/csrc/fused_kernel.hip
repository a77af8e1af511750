// The fused-group kernel: one workgroup streams its owned block of the group's
// domain through every loop of the group, with each dataset's rows held in a
// ring buffer in LDS (see fused.hpp for the scheme).
//
// Workgroup: 128 columns x TR thread rows (TR = 2, 4 or 8 wavefront pairs);
// each thread computes P = 1 or 2 consecutive rows, so a step covers R = TR*P
// rows.  Per step:
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
    const FLoopRec *lrec;   // step records copied into LDS
    const FLoadRec *ld;
    const FStoreRec *st;
    int X0, Y0, W, Hseg, HR, x, col, sub;
    uint32_t cload, cfw, cstore, cloop;  // per-thread column tests, one bit per ring / loop
};

// Rows handled by a thread at step s: R*s + sub*P + p - lag, p in [0, P).
// Loaders: the rows a step needs from the chain-start buffers go straight
// from global memory into their ring slots (global_load_lds, 16 bytes per
// lane: one wave instruction moves one 128-column FP64 row).  Rows are spread
// over the wavefronts; a lane loads only if its column pair is needed.  The
// loads of step s complete before the barrier that ends step s.
template <typename T, int R, int TR>
__device__ __forceinline__ void issue_row_loads(const FGroupD *__restrict__ g, const Blk &b, int s, T *lds) {
    constexpr int EPL = 16 / sizeof(T);           // elements per lane
    constexpr int LANES_PER_ROW = kFCols / EPL;   // 64 (FP64) or 32 (FP32)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwaves = (kFCols * TR) >> 6;
    const int nitems = g->nload * R;
    const int x0 = b.X0 - b.HR;
    for (int it = wave; it < nitems; it += nwaves) {  // one row per wavefront
        const int l = lane;
        const int i = it / R, p = it % R;
        const FLoadRec &Q = b.ld[i];
        const int y = R * s + p - Q.lag;
        const int ra = max(Q.ext_ylo, b.Y0 - Q.ld_below), rb = min(Q.ext_yhi, b.Y0 + b.Hseg + Q.ld_above);
        if (y < ra || y >= rb) continue;
        const int xl = x0 + EPL * l;
        bool act = l < LANES_PER_ROW && xl + EPL > Q.ext_xlo && xl < Q.ext_xhi;
        if (Q.fw && y >= Q.fw_ylo && y < Q.fw_yhi) act = act && !(xl >= Q.fw_xlo && xl + EPL <= Q.fw_xhi);
        if (!act) continue;
        const T __attribute__((address_space(1))) *src =
            (const T __attribute__((address_space(1))) *)Q.src + (int64_t)y * Q.sy + xl;
        T *dst = lds + Q.off + slot_of(y, Q.depth, Q.inv) * kFCols;  // wave-uniform row base
        __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)src,
                                         (void __attribute__((address_space(3))) *)dst, 16, 0, 0);
    }
}

// One input read through a canonical radius-RAD star, for P consecutive rows
// starting at ring slot s0: every LDS read is issued first (rows s0-RAD ..
// s0+P-1+RAD of the thread's column, then the x neighbours of each row), then
// the fmas in the listed order (centre, -x, +x, [-2x, +2x,] -y, +y, [-2y, +2y]).
template <typename T, int P, int RAD>
__device__ __forceinline__ void star_input(const T *ring, int s0, int depth, const double *w, T (&acc)[P]) {
    T cv[P + 2 * RAD];
    int sl[P + 2 * RAD];
#pragma unroll
    for (int j = 0; j < P + 2 * RAD; ++j) sl[j] = wrap(s0 + j - RAD, depth) * kFCols;
#pragma unroll
    for (int j = 0; j < P + 2 * RAD; ++j) cv[j] = ring[sl[j]];
    T xn[P][2 * RAD];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const T *c = ring + sl[p + RAD];
        xn[p][0] = c[-1];
        xn[p][1] = c[1];
        if (RAD == 2) {
            xn[p][2] = c[-2];
            xn[p][3] = c[2];
        }
    }
    T wt[RAD == 1 ? 5 : 9];
#pragma unroll
    for (int k = 0; k < (RAD == 1 ? 5 : 9); ++k) wt[k] = (T)w[k];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        T a = acc[p];
        a = fmaT<T>(wt[0], cv[p + RAD], a);
        a = fmaT<T>(wt[1], xn[p][0], a);
        a = fmaT<T>(wt[2], xn[p][1], a);
        if (RAD == 1) {
            a = fmaT<T>(wt[3], cv[p], a);
            a = fmaT<T>(wt[4], cv[p + 2], a);
        } else {
            a = fmaT<T>(wt[3], xn[p][2], a);
            a = fmaT<T>(wt[4], xn[p][3], a);
            a = fmaT<T>(wt[5], cv[p + 1], a);
            a = fmaT<T>(wt[6], cv[p + 3], a);
            a = fmaT<T>(wt[7], cv[p], a);
            a = fmaT<T>(wt[8], cv[p + 4], a);
        }
        acc[p] = a;
    }
}

template <typename T, int P>
__device__ __forceinline__ void compute_and_store(const FGroupD *__restrict__ g, const Blk &b, int base, T *lds) {
    const int nloops = g->nloops;
    for (int l = 0; l < nloops; ++l) {
        const FLoopRec &L = b.lrec[l];
        const int ya = max(L.ylo, b.Y0 - L.vlo), yb = min(L.yhi, b.Y0 + b.Hseg + L.vhi);
        const int y0 = base - L.lag;
        if (y0 + P <= ya || y0 >= yb) continue;  // uniform across the thread row
        const bool col = (b.cloop >> l) & 1u;
        T acc[P];
#pragma unroll
        for (int p = 0; p < P; ++p) acc[p] = (T)0;
        const int nin = L.nin;
#pragma unroll
        for (int i = 0; i < kFMaxIn; ++i) {
            if (i >= nin) break;
            const FInRec &I = L.in[i];
            const int depth = I.depth;
            const int s0 = slot_of(y0, depth, I.inv);
            const T *ring = lds + I.off + b.col;
            if (I.star == 2) {
                star_input<T, P, 2>(ring, s0, depth, L.w[i], acc);
            } else if (I.star == 1) {
                star_input<T, P, 1>(ring, s0, depth, L.w[i], acc);
            } else {
                for (int k = 0; k < I.nent; ++k) {
                    const FEnt E = g->ent[I.ent0 + k];
                    const T wk = (T)g->w[I.ent0 + k];
#pragma unroll
                    for (int p = 0; p < P; ++p)
                        acc[p] = fmaT<T>(wk, ring[wrap(s0 + p + E.dy, depth) * kFCols + E.dx], acc[p]);
                }
            }
        }
        T *out = lds + L.out_off + b.col;
        int so = slot_of(y0, L.out_depth, L.out_inv);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int y = y0 + p;
            if (col && y >= ya && y < yb) out[so * kFCols] = acc[p];
            so = wrap(so + 1, L.out_depth);
        }
    }
    const int nstore = g->nstore;
    for (int i = 0; i < nstore; ++i) {
        const FStoreRec &Q = b.st[i];
        const int ya = max(Q.hylo, b.Y0), yb = min(Q.hyhi, b.Y0 + b.Hseg);
        const int y0 = base - Q.lag;
        if (y0 + P <= ya || y0 >= yb) continue;
        const bool col = (b.cstore >> i) & 1u;
        const T *ring = lds + Q.off + b.col;
        gmut<T> dst = (gmut<T>)Q.dst + b.x;
        int sl = slot_of(y0, Q.depth, Q.inv);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int y = y0 + p;
            if (col && y >= ya && y < yb) dst[(int64_t)y * Q.sy] = ring[sl * kFCols];
            sl = wrap(sl + 1, Q.depth);
        }
    }
}

template <int R>
__device__ __forceinline__ int floor_div(int v) {
    return v >= 0 ? v / R : -((-v + R - 1) / R);
}

template <typename T, int TR, int P>
__global__ void __launch_bounds__(kFCols * TR) fused_kernel(const FGroupD *__restrict__ g) {
    constexpr int R = TR * P;
    extern __shared__ __align__(16) unsigned char smem[];
    T *lds = (T *)smem;
    Blk b;
    {
        // step records into LDS after the rings
        unsigned char *d = smem + g->ring_bytes;
        const int n0 = g->nloops * (int)sizeof(FLoopRec), n1 = g->nload * (int)sizeof(FLoadRec),
                  n2 = g->nstore * (int)sizeof(FStoreRec);
        const int o1 = (int)sizeof(FLoopRec) * kFMaxLoops, o2 = o1 + (int)sizeof(FLoadRec) * kFMaxLoaded;
        const uint32_t *s0 = (const uint32_t *)g->lrec, *s1 = (const uint32_t *)g->ld, *s2 = (const uint32_t *)g->st;
        for (int k = threadIdx.x; k < n0 / 4; k += blockDim.x) ((uint32_t *)d)[k] = s0[k];
        for (int k = threadIdx.x; k < n1 / 4; k += blockDim.x) ((uint32_t *)(d + o1))[k] = s1[k];
        for (int k = threadIdx.x; k < n2 / 4; k += blockDim.x) ((uint32_t *)(d + o2))[k] = s2[k];
        b.lrec = (const FLoopRec *)d;
        b.ld = (const FLoadRec *)(d + o1);
        b.st = (const FStoreRec *)(d + o2);
        __syncthreads();
    }
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
    for (int i = 0; i < g->nload; ++i) {
        const FLoadRec &Q = b.ld[i];
        if (b.x >= Q.ext_xlo && b.x < Q.ext_xhi) b.cload |= 1u << i;
        if (Q.fw && b.x >= Q.fw_xlo && b.x < Q.fw_xhi) b.cfw |= 1u << i;
        const int a = max(Q.ext_ylo, b.Y0 - Q.ld_below), e = min(Q.ext_yhi, b.Y0 + b.Hseg + Q.ld_above);
        if (a < e) {
            s_lo = min(s_lo, floor_div<R>(a + Q.lag));
            s_hi = max(s_hi, floor_div<R>(e - 1 + Q.lag));
        }
    }
    for (int i = 0; i < g->nstore; ++i) {
        const FStoreRec &Q = b.st[i];
        if (b.x >= max(Q.hxlo, b.X0) && b.x < min(Q.hxhi, b.X0 + b.W)) b.cstore |= 1u << i;
        const int a = max(Q.hylo, b.Y0), e = min(Q.hyhi, b.Y0 + b.Hseg);
        if (a < e) {
            s_lo = min(s_lo, floor_div<R>(a + Q.lag));
            s_hi = max(s_hi, floor_div<R>(e - 1 + Q.lag));
        }
    }
    if (s_lo > s_hi) return;  // uniform: nothing to do for this block

    const int sub0 = b.sub * P;
    for (int s = s_lo; s <= s_hi; ++s) {
        issue_row_loads<T, R, TR>(g, b, s, lds);
        compute_and_store<T, P>(g, b, R * s + sub0, lds);
        __builtin_amdgcn_s_waitcnt(0);  // this step's row loads have landed in LDS
        __syncthreads();
    }
}

template <typename T, int TR, int P>
hipError_t go(const FGroupD *dev_desc, int nblocks, int lds_bytes, hipStream_t s) {
    hipError_t e = hipFuncSetAttribute((const void *)fused_kernel<T, TR, P>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fused_kernel<T, TR, P>), dim3(nblocks), dim3(kFCols * TR), lds_bytes, s, dev_desc);
    return hipGetLastError();
}

template <typename T>
hipError_t go_rows(const FGroupD *dev_desc, int rows, int nblocks, int lds_bytes, hipStream_t s) {
    switch (rows) {
    case 2: return go<T, 2, 1>(dev_desc, nblocks, lds_bytes, s);
    case 8: return go<T, 8, 1>(dev_desc, nblocks, lds_bytes, s);
    case 16: return go<T, 8, 2>(dev_desc, nblocks, lds_bytes, s);
    default: return go<T, 4, 1>(dev_desc, nblocks, lds_bytes, s);
    }
}

}  // namespace

hipError_t launch_fused(const FGroupD *dev_desc, int dtype, int rows, int nblocks, int lds_bytes, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    return dtype == TC_F64 ? go_rows<double>(dev_desc, rows, nblocks, lds_bytes, s)
                           : go_rows<float>(dev_desc, rows, nblocks, lds_bytes, s);
}

}  // namespace tc
