// Staged tiles on gfx950: one workgroup (256 or 1024 threads) per tile.  The datasets
// the group writes are staged in LDS over the tile's boxes; the loops run in
// order over their computed boxes with the per-loop kernels' functors,
// re-pointed at the LDS copies (the descriptor itself is copied to LDS and
// patched per loop); a barrier separates loops.  Reductions count owned
// points only and write one double-double partial per tile.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "ops.hpp"
#include "staged.hpp"

namespace tc {

static_assert(sizeof(LoopDesc) % 8 == 0, "descriptors are copied to LDS in 8-byte words");
static_assert(sizeof(LoopDesc) <= 2 * 8 * 256, "a descriptor is at most two words per thread");
static_assert(sizeof(SArgs) <= 4096, "staged kernel arguments stay within 4 KiB");

namespace {

constexpr int kBatch = 8;  // values per lane loaded before they are stored (staging and write-back)

__device__ __forceinline__ int tile_order(int i, int nb) {
    // XCD-aware order: hardware block i runs on XCD i % 8; XCD k gets a
    // contiguous range of tiles, so neighbouring tiles share that XCD's L2
    const int q = nb >> 3, r = nb & 7, xcd = i & 7, k = i >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

struct Pt {
    int x, y, z;
};

// Workgroup-wide combine of one DD value per thread: within each wavefront
// by butterfly shuffles, then the wavefronts' values in wavefront order by
// thread 0.
__device__ DD tile_reduce(int op, DD v) {
    constexpr int kMaxWaves = kSThreads / 64;
    const int nwaves = (int)blockDim.x / 64;
    __shared__ double sh_hi[kMaxWaves], sh_lo[kMaxWaves];
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
        for (int i = 1; i < nwaves; ++i) {
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

// Quotient of 0 <= i < 2^24 by w > 0 through a float reciprocal (inv =
// 1.0f / w): the product is off by at most one, and one correction step
// makes it exact.
__device__ __forceinline__ int quot(int i, int w, float inv) {
    int q = (int)((float)i * inv);
    const int r = i - q * w;
    q += r < 0 ? -1 : (r >= w ? 1 : 0);
    return q;
}

// The box [lo, lo + (wx, wy, *)) walked with x fastest.
struct BoxWalk {
    int lo0, lo1, lo2, wx, wy;
    float ix, iy;
    __device__ BoxWalk(const int *lo, int wx_, int wy_)
        : lo0(lo[0]), lo1(lo[1]), lo2(lo[2]), wx(wx_), wy(wy_), ix(1.0f / (float)wx_), iy(1.0f / (float)wy_) {}
    __device__ __forceinline__ Pt operator()(int i) const {
        Pt p;
        const int q = quot(i, wx, ix);
        p.x = lo0 + (i - q * wx);
        const int r = quot(q, wy, iy);
        p.y = lo1 + (q - r * wy);
        p.z = lo2 + r;
        return p;
    }
};

template <class Op, class D>
__device__ void run_loop_box(const D &d, const int *C, const int *O, int nred, double *partials0,
                             double *partials1, int tile) {
    const int wx = C[3] - C[0], wy = C[4] - C[1], wz = C[5] - C[2];
    const int n = wx * wy * wz;
    const BoxWalk box_point(C, wx, wy);
    DD red[2];
    red[0] = red_identity(d.red_op[0]);
    red[1] = red_identity(d.red_op[1]);
    if (nred == 0) {
        for (int i = threadIdx.x; i < n; i += (int)blockDim.x) {
            const Pt p = box_point(i);
            Op::run(d, p.x, p.y, p.z, red);
        }
        return;
    }
    for (int i = threadIdx.x; i < n; i += (int)blockDim.x) {
        const Pt p = box_point(i);
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
        const DD v = tile_reduce(d.red_op[j], red[j]);
        double *part = j == 0 ? partials0 : partials1;
        if (threadIdx.x == 0) {
            part[2 * (int64_t)tile] = v.hi;
            part[2 * (int64_t)tile + 1] = v.lo;
        }
    }
}

template <typename T, class D>
__device__ void dispatch(const D &d, const int *C, const int *O, int tile) {
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
    const int nt = (int)blockDim.x;  // 256 or 1024
    T *lds = (T *)smem;
    LoopDesc &d = *(LoopDesc *)(smem + a.desc_off);
    const int tile = tile_order(blockIdx.x, gridDim.x);
    if (tile >= a.ntot) return;
    const int *r = a.table + (int64_t)tile * a.rec;
    const int *O = r;
    const int ns = a.nslots;

    // chain-start values of the staged datasets where the tile needs them
    // (written ones: where their chain-start values are read; read-only
    // ones: their read hull)
    for (int s = 0; s < ns; ++s) {
        const SSlot &S = a.slots[s];
        if (!S.staged) continue;
        const int *q = r + 6 + 9 * s;
        const int *L = q + 3;
        const int wx = q[6] - L[0], wy = q[7] - L[1], wz = q[8] - L[2];
        if (wx <= 0 || wy <= 0 || wz <= 0) continue;
        const T *src = (const T *)a.src[s];
        const int64_t gsy = a.gsy[s], gsz = a.gsz[s];
        T *box = lds + S.lds_off;
        const int n = wx * wy * wz;
        const BoxWalk box_point(L, wx, wy);
        // kBatch loads in flight per lane before their stores
        for (int i0 = threadIdx.x; i0 < n; i0 += kBatch * nt) {
            T v[kBatch];
            int o[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int i = i0 + k * nt;
                o[k] = -1;
                if (i < n) {
                    const Pt p = box_point(i);
                    o[k] = (p.x - q[0]) + (p.y - q[1]) * S.lsy + (p.z - q[2]) * S.lsz;
                    v[k] = src[(int64_t)p.x + (int64_t)p.y * gsy + (int64_t)p.z * gsz];
                }
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k)
                if (o[k] >= 0) box[o[k]] = v[k];
        }
    }
    __syncthreads();

    // Loops in order.  A loop's descriptor is read from device memory while
    // the previous loop computes and written to LDS after it, with the
    // tile's pointers, the flush's parameters and the partial addresses
    // substituted as the words are stored; loops the tile does not compute
    // are skipped (their reductions get an identity partial).
    constexpr int kWords = (int)(sizeof(LoopDesc) / 8);
    constexpr int kArg0 = (int)(offsetof(LoopDesc, arg) / 8);
    constexpr int kPrm0 = (int)(offsetof(LoopDesc, prm) / 8);
    constexpr int kPart0 = (int)(offsetof(LoopDesc, partials) / 8);
    static_assert(sizeof(DArg) == 24 && offsetof(DArg, ptr) == 0, "descriptor argument layout");
    static_assert(offsetof(LoopDesc, arg) % 8 == 0 && offsetof(LoopDesc, prm) % 8 == 0 &&
                      offsetof(LoopDesc, partials) % 8 == 0, "descriptor word layout");
    auto next_loop = [&](int l) {
        for (++l; l < a.nloops; ++l) {
            const int *C = r + 6 + 9 * ns + 6 * l;
            if (C[3] > C[0] && C[4] > C[1] && C[5] > C[2]) break;
            const LoopDesc &tmpl = a.loops[l];
            if (threadIdx.x < (unsigned)tmpl.nred) {
                const int j = threadIdx.x;
                const DD e = red_identity(tmpl.red_op[j]);
                double *part = a.partials + 2 * (a.sl[l].part[j] + tile);
                part[0] = e.hi;
                part[1] = e.lo;
            }
        }
        return l;
    };
    // the word of loop l's descriptor at index wi, with this tile's substitutions
    auto word = [&](int l, int wi, uint64_t v) -> uint64_t {
        const SLoop &SL = a.sl[l];
        if (wi >= kArg0 && wi < kArg0 + 3 * kMaxArgs && (wi - kArg0) % 3 == 0) {
            const int k = (wi - kArg0) / 3;
            if (k < a.loops[l].nargs) {
                const int s = SL.slot[k];
                const SSlot &S = a.slots[s];
                if (!S.staged) return (uint64_t)a.src[s];
                const int *q = r + 6 + 9 * s;
                return (uint64_t)(lds + S.lds_off - ((int64_t)q[0] + (int64_t)q[1] * S.lsy + (int64_t)q[2] * S.lsz));
            }
        } else if (wi >= kPrm0 && wi < kPrm0 + SL.nprm) {
            return __builtin_bit_cast(uint64_t, a.prm[SL.prm_off + (wi - kPrm0)]);
        } else if (wi >= kPart0 && wi < kPart0 + 2) {
            return (uint64_t)(a.partials + 2 * SL.part[wi - kPart0]);
        }
        return v;
    };
    uint64_t *dw = (uint64_t *)&d;
    int l = next_loop(-1);
    if (l < a.nloops) {
        const uint64_t *from = (const uint64_t *)(a.loops + l);
        for (int i = threadIdx.x; i < kWords; i += nt) dw[i] = word(l, i, from[i]);
    }
    __syncthreads();
    while (l < a.nloops) {
        const int ln = next_loop(l);
        uint64_t w0 = 0, w1 = 0;
        if (ln < a.nloops) {  // in flight while this loop computes
            const uint64_t *from = (const uint64_t *)(a.loops + ln);
            if (threadIdx.x < (unsigned)kWords) w0 = from[threadIdx.x];
            if (threadIdx.x + nt < (unsigned)kWords) w1 = from[threadIdx.x + nt];
        }
        if (a.sl[l].all_lds)  // every dataset in LDS: LDS-addressed loads and stores
            dispatch<T>(static_cast<const LdsDesc &>(d), r + 6 + 9 * ns + 6 * l, O, tile);
        else
            dispatch<T>(d, r + 6 + 9 * ns + 6 * l, O, tile);
        __syncthreads();
        if (ln < a.nloops) {
            if (threadIdx.x < (unsigned)kWords) dw[threadIdx.x] = word(ln, threadIdx.x, w0);
            if (threadIdx.x + nt < (unsigned)kWords) dw[threadIdx.x + nt] = word(ln, threadIdx.x + nt, w1);
        }
        __syncthreads();
        l = ln;
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
        const BoxWalk box_point(lo, wx, wy);
        for (int i0 = threadIdx.x; i0 < n; i0 += kBatch * nt) {
            T v[kBatch];
            int64_t o[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int i = i0 + k * nt;
                o[k] = 0;
                if (i < n) {  // logical offsets may be negative (halo points)
                    const Pt p = box_point(i);
                    o[k] = (int64_t)p.x + (int64_t)p.y * gsy + (int64_t)p.z * gsz;
                    v[k] = box[(p.x - q[0]) + (p.y - q[1]) * S.lsy + (p.z - q[2]) * S.lsz];
                }
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k)
                if (i0 + k * nt < n) dst[o[k]] = v[k];
        }
    }
}

template <typename T>
hipError_t go(const SArgs &a, size_t lds, int threads, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute((const void *)staged_kernel<T>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(staged_kernel<T>, dim3(a.ntot), dim3(threads == 256 ? 256 : kSThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_staged(const SArgs &a, int dtype, size_t lds_bytes, int threads, hipStream_t s) {
    if (a.ntot <= 0) return hipSuccess;
    return dtype == TC_F64 ? go<double>(a, lds_bytes, threads, s) : go<float>(a, lds_bytes, threads, s);
}

}  // namespace tc
