// Right-hand side of the compressible Euler equations in 3D (TC_OP_EULER_RHS),
// one conserved component per launch, marching up z.
//
// Arguments as for the op: R (written), Q_c, u, v, w, p; parameters c and
// s = 1 / (12 h).  For each axis the flux of component c is
//   F = Q_c u_axis (+ p if c is the axis's momentum) (then fma(p, u_axis, F)
//   if c is the energy),
// and R = -(g_x + g_y + g_z) s with g = 8 (F(+1) - F(-1)) - (F(+2) - F(-2)),
// the differences taken first and summed in axis order: the same operations
// in the same order as the per-point loop kernel, so the results are equal
// bit for bit.
//
// Layout: a workgroup is four wavefronts, one per y row; a wavefront's lanes
// hold 64 consecutive x columns, 60 of them owned (two halo lanes per side),
// and it walks kRhsTz planes up z.  The x fluxes of the current plane come
// from neighbouring lanes and the z fluxes from a five-plane register window
// fed by one row load per plane and input.  For the y fluxes every wavefront
// computes the flux of its own row and of one of the four rows just outside
// the workgroup (y0-2, y0-1, y0+4, y0+5) and puts both into LDS, where the
// workgroup's rows find their four neighbours (one barrier per plane, two LDS
// buffers).  Loads run one plane ahead.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace tc {

namespace {

constexpr int kRhsThreads = 256;  // four wavefronts, one per y row
constexpr int kRhsOut = 60;       // owned columns per wavefront
constexpr int kRhsRows = 4;       // rows per workgroup
constexpr int kRhsTz = 32;        // planes per workgroup

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

__device__ __forceinline__ int xcd_block(int i, int nb) {
    const int q = nb >> 3, r = nb & 7, xcd = i & 7, k = i >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

// flux of component C along axis AX (0 x, 1 y, 2 z)
template <typename T, int C, int AX>
__device__ __forceinline__ T flux(T q, T ud, T p) {
    T f = q * ud;
    if constexpr (C == AX + 1) f = f + p;
    if constexpr (C == 4) f = fma_t<T>(p, ud, f);
    return f;
}

template <typename T>
__device__ __forceinline__ T diff4(T fm2, T fm1, T fp1, T fp2) {
    const T t1 = fp1 - fm1;
    const T t2 = fp2 - fm2;
    return (T)8 * t1 - t2;
}

template <typename T, int C>
__global__ void __launch_bounds__(kRhsThreads) euler_rhs3_kernel(LoopDesc d, int lo0, int hi0, int lo1, int hi1,
                                                                 int lo2, int hi2, int nbx, int nby, int nb, int tz) {
    constexpr bool PX = C == 1 || C == 4, PY = C == 2 || C == 4, PZ = C == 3 || C == 4;
    constexpr bool P0 = PX || PY;  // pressure of the current plane
    __shared__ T fy_lds[2][kRhsRows + 4][64];
    const int lin = xcd_block(blockIdx.x, nb);
    const int bx = lin % nbx, rest = lin / nbx, by = rest % nby, bz = rest / nby;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = lo0 + bx * kRhsOut - 2 + lane;
    const int y0 = lo1 + by * kRhsRows;
    const int y = y0 + wave;
    const bool active = lane >= 2 && lane < 2 + kRhsOut && x < hi0 && y < hi1;
    const int z0 = lo2 + bz * tz;
    const int z1 = min(z0 + tz, hi2);
    // Every position read lies in [lo - 2, hi + 1] per axis, inside the
    // allocation.  Lanes and rows beyond that are clamped; they feed no
    // output.  Rows up to hi1 + 1 are real neighbours of the last output rows.
    const int xc = min(max(x, lo0 - 2), hi0 + 1);
    const int yr = min(y, hi1 + 1);
    const int hslot = wave < 2 ? wave : wave + kRhsRows;  // LDS row of this wave's outside row
    const int yh = min(y0 - 2 + hslot, hi1 + 1);
    const int64_t qy = d.arg[1].sy, vy = d.arg[3].sy, py = d.arg[5].sy;
    const T *q = (const T *)d.arg[1].ptr + xc + (int64_t)yr * qy;
    const T *u = (const T *)d.arg[2].ptr + xc + (int64_t)yr * d.arg[2].sy;
    const T *v = (const T *)d.arg[3].ptr + xc + (int64_t)yr * vy;
    const T *w = (const T *)d.arg[4].ptr + xc + (int64_t)yr * d.arg[4].sy;
    const T *p = (const T *)d.arg[5].ptr + xc + (int64_t)yr * py;
    const T *hq = (const T *)d.arg[1].ptr + xc + (int64_t)yh * qy;
    const T *hv = (const T *)d.arg[3].ptr + xc + (int64_t)yh * vy;
    const T *hp = (const T *)d.arg[5].ptr + xc + (int64_t)yh * py;
    T *out = (T *)d.arg[0].ptr + xc + (int64_t)yr * d.arg[0].sy;
    const int64_t qz = d.arg[1].sz, uz = d.arg[2].sz, vz = d.arg[3].sz, wz = d.arg[4].sz, pz = d.arg[5].sz;
    const int64_t oz = d.arg[0].sz;
    const T s = (T)d.prm[1];

    // z fluxes of planes z-2 .. z+2
    T fz[5];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t pl = z0 - 2 + k;
        fz[k] = flux<T, C, 2>(q[pl * qz], w[pl * wz], PZ ? p[pl * pz] : (T)0);
    }
    // own row at planes z and z+1 (q, u, p), v at plane z; the leading
    // plane z+2 (q, u, w, p); the outside row at plane z (q, v, p)
    T q0 = q[(int64_t)z0 * qz], u0 = u[(int64_t)z0 * uz], p0 = P0 ? p[(int64_t)z0 * pz] : (T)0;
    T q1 = q[(int64_t)(z0 + 1) * qz], u1 = u[(int64_t)(z0 + 1) * uz];
    T p1 = P0 ? p[(int64_t)(z0 + 1) * pz] : (T)0;
    T v0 = v[(int64_t)z0 * vz];
    T nq = q[(int64_t)(z0 + 2) * qz], nu = u[(int64_t)(z0 + 2) * uz], nw = w[(int64_t)(z0 + 2) * wz];
    T np = (P0 || PZ) ? p[(int64_t)(z0 + 2) * pz] : (T)0;
    T oq = hq[(int64_t)z0 * qz], ov = hv[(int64_t)z0 * vz], op = PY ? hp[(int64_t)z0 * pz] : (T)0;

    int buf = 0;
    for (int z = z0; z < z1; ++z) {
        // y fluxes of this plane: own row and outside row into LDS
        fy_lds[buf][wave + 2][lane] = flux<T, C, 1>(q0, v0, PY ? p0 : (T)0);
        fy_lds[buf][hslot][lane] = flux<T, C, 1>(oq, ov, op);
        // the leading plane completes the z window
        fz[4] = flux<T, C, 2>(nq, nw, PZ ? np : (T)0);
        const T q2 = nq, u2 = nu, p2 = np;
        // loads for the next plane
        if (z + 1 < z1) {
            const int64_t pl = z + 1;
            v0 = v[pl * vz];
            oq = hq[pl * qz];
            ov = hv[pl * vz];
            if (PY) op = hp[pl * pz];
            const int64_t lead = z + 3;
            nq = q[lead * qz];
            nu = u[lead * uz];
            nw = w[lead * wz];
            if (P0 || PZ) np = p[lead * pz];
        }
        // x: fluxes of this lane's column, neighbours from adjacent lanes
        const T fx = flux<T, C, 0>(q0, u0, PX ? p0 : (T)0);
        const T fxm1 = __shfl_up(fx, 1, 64), fxp1 = __shfl_down(fx, 1, 64);
        const T fxm2 = __shfl_up(fx, 2, 64), fxp2 = __shfl_down(fx, 2, 64);
        const T gx = diff4<T>(fxm2, fxm1, fxp1, fxp2);
        const T gz = diff4<T>(fz[0], fz[1], fz[3], fz[4]);
        __syncthreads();
        const T gy = diff4<T>(fy_lds[buf][wave][lane], fy_lds[buf][wave + 1][lane], fy_lds[buf][wave + 3][lane],
                              fy_lds[buf][wave + 4][lane]);
        T acc = gx;
        acc = acc + gy;
        acc = acc + gz;
        if (active) out[(int64_t)z * oz] = -acc * s;
#pragma unroll
        for (int k = 0; k < 4; ++k) fz[k] = fz[k + 1];
        q0 = q1;
        u0 = u1;
        p0 = p1;
        q1 = q2;
        u1 = u2;
        p1 = p2;
        buf ^= 1;
    }
}

template <typename T, int C>
hipError_t go_rhs3(const LoopDesc &d, const Box &b, hipStream_t s) {
    const int nbx = (b.hi[0] - b.lo[0] + kRhsOut - 1) / kRhsOut;
    const int nby = (b.hi[1] - b.lo[1] + kRhsRows - 1) / kRhsRows;
    const int nbz = (b.hi[2] - b.lo[2] + kRhsTz - 1) / kRhsTz;
    const int nb = nbx * nby * nbz;
    hipLaunchKernelGGL((euler_rhs3_kernel<T, C>), dim3(nb), dim3(kRhsThreads), 0, s, d, b.lo[0], b.hi[0], b.lo[1],
                       b.hi[1], b.lo[2], b.hi[2], nbx, nby, nb, kRhsTz);
    return hipGetLastError();
}

template <typename T>
hipError_t rhs3_t(const LoopDesc &d, const Box &b, hipStream_t s) {
    switch ((int)d.prm[0]) {
    case 0: return go_rhs3<T, 0>(d, b, s);
    case 1: return go_rhs3<T, 1>(d, b, s);
    case 2: return go_rhs3<T, 2>(d, b, s);
    case 3: return go_rhs3<T, 3>(d, b, s);
    case 4: return go_rhs3<T, 4>(d, b, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_euler_rhs3(const LoopDesc &d, const Box &b, int dtype, hipStream_t s) {
    if (b.nb <= 0) return hipSuccess;
    return dtype == TC_F64 ? rhs3_t<double>(d, b, s) : rhs3_t<float>(d, b, s);
}

}  // namespace tc
