// Staged tiles on gfx950: one workgroup (256 threads) per tile.  The datasets
// the group writes are staged in LDS over the tile's boxes; the loops run in
// order over their computed boxes with the per-loop kernels' functors,
// re-pointed at the LDS copies (the descriptor itself is copied to LDS and
// patched per loop); a barrier separates loops.  Reductions count owned
// points only and write one double-double partial per tile.
#include <hip/hip_runtime.h>

#include "ops.hpp"
#include "staged.hpp"

namespace tc {

static_assert(sizeof(LoopDesc) % 8 == 0, "descriptors are copied to LDS in 8-byte words");
static_assert(sizeof(SArgs) <= 4096, "staged kernel arguments stay within 4 KiB");

namespace {

__device__ __forceinline__ int tile_order(int i, int nb) {
    // XCD-aware order: hardware block i runs on XCD i % 8; XCD k gets a
    // contiguous range of tiles, so neighbouring tiles share that XCD's L2
    const int q = nb >> 3, r = nb & 7, xcd = i & 7, k = i >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

struct Pt {
    int x, y, z;
};

// i-th point of the box [lo, hi) with x fastest
__device__ __forceinline__ Pt box_point(const int *lo, int wx, int wy, int i) {
    Pt p;
    const int q = i / wx;
    p.x = lo[0] + (i - q * wx);
    const int r = q / wy;
    p.y = lo[1] + (q - r * wy);
    p.z = lo[2] + r;
    return p;
}

template <class Op>
__device__ void run_loop_box(const LoopDesc &d, const int *C, const int *O, int nred, double *partials0,
                             double *partials1, int tile) {
    const int wx = C[3] - C[0], wy = C[4] - C[1], wz = C[5] - C[2];
    const int n = wx * wy * wz;
    DD red[2];
    red[0] = red_identity(d.red_op[0]);
    red[1] = red_identity(d.red_op[1]);
    if (nred == 0) {
        for (int i = threadIdx.x; i < n; i += kSThreads) {
            const Pt p = box_point(C, wx, wy, i);
            Op::run(d, p.x, p.y, p.z, red);
        }
        return;
    }
    for (int i = threadIdx.x; i < n; i += kSThreads) {
        const Pt p = box_point(C, wx, wy, i);
        const bool own = p.x >= O[0] && p.x < O[3] && p.y >= O[1] && p.y < O[4] && p.z >= O[2] && p.z < O[5];
        if (own) {
            Op::run(d, p.x, p.y, p.z, red);
        } else {
            DD scratch_red[2];
            scratch_red[0] = red_identity(d.red_op[0]);
            scratch_red[1] = red_identity(d.red_op[1]);
            Op::run(d, p.x, p.y, p.z, scratch_red);
        }
    }
    for (int j = 0; j < 2; ++j) {
        if (j >= nred) break;
        const DD v = block_reduce(d.red_op[j], red[j]);
        double *part = j == 0 ? partials0 : partials1;
        if (threadIdx.x == 0) {
            part[2 * (int64_t)tile] = v.hi;
            part[2 * (int64_t)tile + 1] = v.lo;
        }
    }
}

template <typename T>
__device__ void dispatch(const LoopDesc &d, const int *C, const int *O, int tile) {
    const int nred = d.nred;
    double *p0 = d.partials[0], *p1 = d.partials[1];
    switch (d.op) {
    case TC_OP_WSUM: run_loop_box<OpWsum<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_COPY: run_loop_box<OpCopy<T, T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_AXPBY: run_loop_box<OpAxpby<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_DOT: run_loop_box<OpDot<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_SUM: run_loop_box<OpSum<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_HALO_REFLECT: run_loop_box<OpHaloReflect<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_TEA_INIT: run_loop_box<OpTeaInit<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_TEA_K: run_loop_box<OpTeaK<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_TEA_RESID: run_loop_box<OpTeaResid<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_TEA_MATVEC_DOT: run_loop_box<OpTeaMatvecDot<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_TEA_P1: run_loop_box<OpTeaP1<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_TEA_P2: run_loop_box<OpTeaP2<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_TEA_PRECON_INIT: run_loop_box<OpTeaPreconInit<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_TEA_CG_UPDATE: run_loop_box<OpTeaCgUpdate<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_TEA_CG_P: run_loop_box<OpTeaCgP<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_TEA_GERSH: run_loop_box<OpTeaGersh<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_EULER_PRIM: run_loop_box<OpEulerPrim<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_EULER_RHS: run_loop_box<OpEulerRhs<T>>(d, C, O, nred, p0, p1, tile); break;
    case TC_OP_RK_STAGE: run_loop_box<OpRkStage<T>>(d, C, O, nred, p0, p1, tile); break;
    default: break;
    }
}

template <typename T>
__global__ void __launch_bounds__(kSThreads) staged_kernel(SArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *lds = (T *)smem;
    LoopDesc &d = *(LoopDesc *)(smem + a.desc_off);
    const int tile = tile_order(blockIdx.x, gridDim.x);
    if (tile >= a.ntot) return;
    const int *r = a.table + (int64_t)tile * a.rec;
    const int *O = r;
    const int ns = a.nslots;

    // chain-start values of the staged datasets where the tile needs them
    for (int s = 0; s < ns; ++s) {
        const SSlot &S = a.slots[s];
        if (!S.resident) continue;
        const int *q = r + 6 + 9 * s;
        const int *L = q + 3;
        const int wx = q[6] - L[0], wy = q[7] - L[1], wz = q[8] - L[2];
        if (wx <= 0 || wy <= 0 || wz <= 0) continue;
        const T *src = (const T *)a.src[s];
        const int64_t gsy = a.gsy[s], gsz = a.gsz[s];
        T *box = lds + S.lds_off;
        const int n = wx * wy * wz;
        for (int i = threadIdx.x; i < n; i += kSThreads) {
            const Pt p = box_point(L, wx, wy, i);
            box[(p.x - q[0]) + (p.y - q[1]) * S.lsy + (p.z - q[2]) * S.lsz] =
                src[(int64_t)p.x + (int64_t)p.y * gsy + (int64_t)p.z * gsz];
        }
    }
    __syncthreads();

    for (int l = 0; l < a.nloops; ++l) {
        const int *C = r + 6 + 9 * ns + 6 * l;
        if (C[3] <= C[0] || C[4] <= C[1] || C[5] <= C[2]) {
            // nothing to compute here; a reduction still gets this tile's
            // partial (the identity), since the finalize pass reads one per tile
            const LoopDesc &tmpl = a.loops[l];
            if (threadIdx.x < (unsigned)tmpl.nred) {
                const int j = threadIdx.x;
                const DD e = red_identity(tmpl.red_op[j]);
                double *part = a.partials + 2 * (a.sl[l].part[j] + tile);
                part[0] = e.hi;
                part[1] = e.lo;
            }
            continue;
        }
        // this loop's descriptor into LDS, re-pointed at the tile's boxes
        {
            const uint64_t *from = (const uint64_t *)(a.loops + l);
            uint64_t *to = (uint64_t *)&d;
            for (int i = threadIdx.x; i < (int)(sizeof(LoopDesc) / 8); i += kSThreads) to[i] = from[i];
        }
        __syncthreads();
        const SLoop &SL = a.sl[l];
        if (threadIdx.x < (unsigned)d.nargs) {
            const int k = threadIdx.x;
            const int s = SL.slot[k];
            const SSlot &S = a.slots[s];
            if (S.resident) {
                const int *q = r + 6 + 9 * s;
                d.arg[k].ptr = (void *)(lds + S.lds_off - ((int64_t)q[0] + (int64_t)q[1] * S.lsy + (int64_t)q[2] * S.lsz));
            } else {
                d.arg[k].ptr = a.src[s];
            }
        }
        if (threadIdx.x >= 64 && threadIdx.x < 64u + (unsigned)SL.nprm) {
            const int k = threadIdx.x - 64;
            d.prm[k] = a.prm[SL.prm_off + k];
        }
        if (threadIdx.x >= 192 && threadIdx.x < 194) {
            const int j = threadIdx.x - 192;
            d.partials[j] = a.partials + 2 * SL.part[j];
        }
        __syncthreads();
        dispatch<T>(d, C, O, tile);
        __syncthreads();
    }

    // owned values of the staged datasets
    for (int s = 0; s < ns; ++s) {
        const SSlot &S = a.slots[s];
        if (!S.resident) continue;
        int lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
            lo[k] = max(O[k], S.wlo[k]);
            hi[k] = min(O[3 + k], S.whi[k]);
        }
        const int wx = hi[0] - lo[0], wy = hi[1] - lo[1], wz = hi[2] - lo[2];
        if (wx <= 0 || wy <= 0 || wz <= 0) continue;
        const int *q = r + 6 + 9 * s;
        T *dst = (T *)a.dst[s];
        const int64_t gsy = a.gsy[s], gsz = a.gsz[s];
        const T *box = lds + S.lds_off;
        const int n = wx * wy * wz;
        for (int i = threadIdx.x; i < n; i += kSThreads) {
            const Pt p = box_point(lo, wx, wy, i);
            dst[(int64_t)p.x + (int64_t)p.y * gsy + (int64_t)p.z * gsz] =
                box[(p.x - q[0]) + (p.y - q[1]) * S.lsy + (p.z - q[2]) * S.lsz];
        }
    }
}

template <typename T>
hipError_t go(const SArgs &a, size_t lds, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute((const void *)staged_kernel<T>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(staged_kernel<T>, dim3(a.ntot), dim3(kSThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_staged(const SArgs &a, int dtype, size_t lds_bytes, hipStream_t s) {
    if (a.ntot <= 0) return hipSuccess;
    return dtype == TC_F64 ? go<double>(a, lds_bytes, s) : go<float>(a, lds_bytes, s);
}

}  // namespace tc
