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
#include "lanes.hpp"

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

// the same flux with the component chosen at run time (a switch the
// compiler resolves when the caller's loop over components is unrolled)
template <typename T, int AX>
__device__ __forceinline__ T flux_c(int c, T q, T ud, T p) {
    T f = q * ud;
    if (c == AX + 1) f = f + p;
    if (c == 4) f = fma_t<T>(p, ud, f);
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
        const T fxm1 = lane_prev(fx), fxp1 = lane_next(fx);
        const T fxm2 = lane_prev(fxm1), fxp2 = lane_next(fxp1);
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

// ---------------------------------------------------------------------------
// One Runge-Kutta stage after the primitive variables: the five right-hand
// sides and the five updates in one z march.  Per plane a lane forms the x,
// y and z fluxes of all five components from Q, u, v, w, p (x neighbours
// from adjacent lanes, y neighbours through LDS as above, z neighbours from
// a five-plane window), then R_c = -(g_x + g_y + g_z) s and
// Q_c = fma(a, Q0_c, b fma(dt, R_c, Q_c)) -- the arithmetic of the RHS and
// RK_STAGE loops, in their order, so the results are their bits.  Q is read
// at stencil offsets by neighbouring workgroups, so the new Q goes to the
// datasets' second buffers; R is written only if a later loop reads it.
// ---------------------------------------------------------------------------
constexpr int kStageOut = 60;

// Primitive variables of one point, as TC_OP_EULER_PRIM computes them.
template <typename T>
__device__ __forceinline__ void prims3(const T q[5], T gm1, T &u, T &v, T &w, T &p) {
    const T ri = (T)1 / q[0];
    const T u0 = q[1] * ri, u1 = q[2] * ri, u2 = q[3] * ri;
    T ke = q[3] * u2;
    ke = fma_t<T>(q[2], u1, ke);
    ke = fma_t<T>(q[1], u0, ke);
    u = u0;
    v = u1;
    w = u2;
    p = gm1 * fma_t<T>((T)-0.5, ke, q[4]);
}

// PRIM: the stage's primitive variables are computed here from Q (its
// primitive-variable loop is fused in) instead of being loaded.  COPY0: the
// step's copies Q0 = Q are fused in: the update takes Q0 from the stage's Q
// (the copy's value) and Q0 is stored at the owned points.
// A workgroup is NW wavefronts, one per y row; wavefronts 0-3 also carry the
// four rows just outside it (y0-2, y0-1, y0+NW, y0+NW+1).
template <typename T, bool PRIM, bool COPY0, int NW>
__global__ void __launch_bounds__(64 * NW) euler_stage3_kernel(EulerStageArgs a) {
    __shared__ T fy_lds[2][NW + 4][5][64];
    const int lin = xcd_block(blockIdx.x, a.nb);
    const int bx = lin % a.nbx, rest = lin / a.nbx, by = rest % a.nby, bz = rest / a.nby;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: branches on it stay scalar
    const bool outer = wave < 4;
    const int x = a.lo[0] + bx * kStageOut - 2 + lane;
    const int y0 = a.lo[1] + by * NW;
    const int y = y0 + wave;
    const bool active = lane >= 2 && lane < 2 + kStageOut && x < a.hi[0] && y < a.hi[1];
    const int z0 = a.lo[2] + bz * a.tz;
    const int z1 = min(z0 + a.tz, a.hi[2]);
    // every position read lies in [lo - 2, hi + 1] per axis (inside the
    // allocation); lanes and rows beyond that are clamped and feed no output
    const int xc = min(max(x, a.lo[0] - 2), a.hi[0] + 1);
    const int yr = min(y, a.hi[1] + 1);
    const int hslot = wave < 2 ? wave : wave + NW;  // LDS row of this wavefront's outside row (wavefronts 0-3)
    const int yh = min(y0 - 2 + hslot, a.hi[1] + 1);
    // row bases: own row (yr) and outside row (yh), column xc
    auto at = [&](int k, int row) { return (const T *)a.ptr[k] + xc + (int64_t)row * a.sy[k]; };
    const T *q[5], *hq[5], *q0[5];
    for (int c = 0; c < 5; ++c) {
        q[c] = at(kQ + c, yr);
        hq[c] = at(kQ + c, yh);
        q0[c] = COPY0 ? nullptr : at(kQ0 + c, yr);
    }
    const T *u = PRIM ? nullptr : at(kU, yr), *v = PRIM ? nullptr : at(kU + 1, yr);
    const T *w = PRIM ? nullptr : at(kU + 2, yr), *p = PRIM ? nullptr : at(kP, yr);
    const T *hv = PRIM ? nullptr : at(kU + 1, yh), *hp = PRIM ? nullptr : at(kP, yh);
    auto ld = [&](const T *base, int k, int z) { return base[(int64_t)z * a.sz[k]]; };
    const T s = (T)a.s, ra = (T)a.a, rb = (T)a.b, dt = (T)a.dt, gm1 = (T)a.gm1;

    // z fluxes of planes z0-2 .. z0+1
    T fz[5][5];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int pl = z0 - 2 + k;
        T qk[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) qk[c] = ld(q[c], kQ + c, pl);
        T wk, pk;
        if constexpr (PRIM) {
            T uk, vk;
            prims3<T>(qk, gm1, uk, vk, wk, pk);
        } else {
            wk = ld(w, kU + 2, pl);
            pk = ld(p, kP, pl);
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) fz[c][k] = flux_c<T, 2>(c, qk[c], wk, pk);
    }
    // own row at planes z (current) and z+1: Q, u, v, p; the leading plane
    // z+2: Q, u, v, w, p; the outside row at plane z: Q, v, p; Q0 at plane z
    T cq[5], nq[5], lq[5], oq[5], cq0[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        cq[c] = ld(q[c], kQ + c, z0);
        nq[c] = ld(q[c], kQ + c, z0 + 1);
        lq[c] = ld(q[c], kQ + c, z0 + 2);
        oq[c] = outer ? ld(hq[c], kQ + c, z0) : (T)1;  // (T)1: no division by zero in prims3
        cq0[c] = COPY0 ? cq[c] : ld(q0[c], kQ0 + c, z0);
    }
    T cu, cv, cp, nu, nv, np_, lu, lv, lw, lp, ov, op;
    if constexpr (PRIM) {
        T t0, t1;
        prims3<T>(cq, gm1, cu, cv, t0, cp);
        prims3<T>(nq, gm1, nu, nv, t1, np_);
        prims3<T>(lq, gm1, lu, lv, lw, lp);
        prims3<T>(oq, gm1, t0, ov, t1, op);
    } else {
        cu = ld(u, kU, z0), cv = ld(v, kU + 1, z0), cp = ld(p, kP, z0);
        nu = ld(u, kU, z0 + 1), nv = ld(v, kU + 1, z0 + 1), np_ = ld(p, kP, z0 + 1);
        lu = ld(u, kU, z0 + 2), lv = ld(v, kU + 1, z0 + 2), lw = ld(w, kU + 2, z0 + 2), lp = ld(p, kP, z0 + 2);
        ov = outer ? ld(hv, kU + 1, z0) : (T)0;
        op = outer ? ld(hp, kP, z0) : (T)0;
    }

    T *qn[5], *rr[5], *q0o[5];
    for (int c = 0; c < 5; ++c) {
        qn[c] = (T *)a.out[c] + xc + (int64_t)yr * a.osy[c];
        rr[c] = a.rout[c] ? (T *)a.rout[c] + xc + (int64_t)yr * a.rsy[c] : nullptr;
        q0o[c] = COPY0 ? (T *)a.q0out[c] + xc + (int64_t)yr * a.q0sy[c] : nullptr;
    }
    int buf = 0;
    for (int z = z0; z < z1; ++z) {
        // y fluxes of this plane: own row and outside row into LDS
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            fy_lds[buf][wave + 2][c][lane] = flux_c<T, 1>(c, cq[c], cv, cp);
            if (outer) fy_lds[buf][hslot][c][lane] = flux_c<T, 1>(c, oq[c], ov, op);
        }
        // the leading plane completes the z windows
#pragma unroll
        for (int c = 0; c < 5; ++c) fz[c][4] = flux_c<T, 2>(c, lq[c], lw, lp);
        // x fluxes of this lane's column, neighbours from adjacent lanes
        T gx[5], gz[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const T fx = flux_c<T, 0>(c, cq[c], cu, cp);
            const T fxm1 = lane_prev(fx), fxp1 = lane_next(fx);
            const T fxm2 = lane_prev(fxm1), fxp2 = lane_next(fxp1);
            gx[c] = diff4<T>(fxm2, fxm1, fxp1, fxp2);
            gz[c] = diff4<T>(fz[c][0], fz[c][1], fz[c][3], fz[c][4]);
        }
        // loads for the next plane (the leading plane z+3, the outside row
        // and Q0 at z+1)
        T iq[5], ioq[5], iq0[5];
        T iu = (T)0, iv = (T)0, iw = (T)0, ip = (T)0, iov = (T)0, iop = (T)0;
        const bool more = z + 1 < z1;
        if (more) {
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                iq[c] = ld(q[c], kQ + c, z + 3);
                ioq[c] = outer ? ld(hq[c], kQ + c, z + 1) : (T)1;
                if constexpr (!COPY0) iq0[c] = ld(q0[c], kQ0 + c, z + 1);
            }
            if constexpr (PRIM) {
                T t0, t1;
                prims3<T>(iq, gm1, iu, iv, iw, ip);
                prims3<T>(ioq, gm1, t0, iov, t1, iop);
            } else {
                iu = ld(u, kU, z + 3);
                iv = ld(v, kU + 1, z + 3);
                iw = ld(w, kU + 2, z + 3);
                ip = ld(p, kP, z + 3);
                if (outer) {
                    iov = ld(hv, kU + 1, z + 1);
                    iop = ld(hp, kP, z + 1);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const T gy = diff4<T>(fy_lds[buf][wave][c][lane], fy_lds[buf][wave + 1][c][lane],
                                  fy_lds[buf][wave + 3][c][lane], fy_lds[buf][wave + 4][c][lane]);
            T acc = gx[c];
            acc = acc + gy;
            acc = acc + gz[c];
            const T r = -acc * s;
            const T t = fma_t<T>(dt, r, cq[c]);
            const T qnew = fma_t<T>(ra, cq0[c], rb * t);
            if (active) {
                qn[c][(int64_t)z * a.osz[c]] = qnew;
                if (rr[c]) rr[c][(int64_t)z * a.rsz[c]] = r;
                if constexpr (COPY0) q0o[c][(int64_t)z * a.q0sz[c]] = cq0[c];
            }
        }
        // advance the windows
#pragma unroll
        for (int c = 0; c < 5; ++c) {
#pragma unroll
            for (int k = 0; k < 4; ++k) fz[c][k] = fz[c][k + 1];
            cq[c] = nq[c];
            nq[c] = lq[c];
            if (more) {
                lq[c] = iq[c];
                oq[c] = ioq[c];
            }
            cq0[c] = COPY0 ? cq[c] : (more ? iq0[c] : cq0[c]);  // cq: already the next plane's
        }
        cu = nu; cv = nv; cp = np_;
        nu = lu; nv = lv; np_ = lp;
        if (more) {
            lu = iu; lv = iv; lw = iw; lp = ip;
            ov = iov; op = iop;
        }
        buf ^= 1;
    }
}

template <typename T, int NW>
hipError_t go_stage3_nw(const EulerStageArgs &in, hipStream_t s) {
    EulerStageArgs a = in;
    a.nbx = (a.hi[0] - a.lo[0] + kStageOut - 1) / kStageOut;
    a.nby = (a.hi[1] - a.lo[1] + NW - 1) / NW;
    const int nz = a.hi[2] - a.lo[2];
    if (a.tz <= 0) {
        // longest march (fewest z-halo planes re-read) that still makes
        // about 1000 workgroups
        a.tz = 128;
        while (a.tz > 32 && (int64_t)a.nbx * a.nby * ((nz + a.tz - 1) / a.tz) < 1000) a.tz /= 2;
    }
    a.nb = a.nbx * a.nby * ((nz + a.tz - 1) / a.tz);
    if (a.nb <= 0 || a.nbx <= 0 || a.nby <= 0 || nz <= 0) return hipSuccess;
    const dim3 g(a.nb), b(64 * NW);
    if (a.prim && a.copy0)
        hipLaunchKernelGGL((euler_stage3_kernel<T, true, true, NW>), g, b, 0, s, a);
    else if (a.prim)
        hipLaunchKernelGGL((euler_stage3_kernel<T, true, false, NW>), g, b, 0, s, a);
    else if (a.copy0)
        hipLaunchKernelGGL((euler_stage3_kernel<T, false, true, NW>), g, b, 0, s, a);
    else
        hipLaunchKernelGGL((euler_stage3_kernel<T, false, false, NW>), g, b, 0, s, a);
    return hipGetLastError();
}

// rows: the given 4 or 8, or (0) 8 unless that leaves fewer than about 1000
// workgroups of 32 planes
template <typename T>
hipError_t go_stage3(const EulerStageArgs &a, hipStream_t s) {
    int rows = a.rows;
    if (rows != 4 && rows != 8) {
        const int64_t nb8 = (int64_t)((a.hi[0] - a.lo[0] + kStageOut - 1) / kStageOut) * ((a.hi[1] - a.lo[1] + 7) / 8) *
                            ((a.hi[2] - a.lo[2] + 31) / 32);
        rows = nb8 >= 1000 ? 8 : 4;
    }
    return rows == 4 ? go_stage3_nw<T, 4>(a, s) : go_stage3_nw<T, 8>(a, s);
}

}  // namespace

hipError_t launch_euler_stage3(const EulerStageArgs &a, int dtype, hipStream_t s) {
    return dtype == TC_F64 ? go_stage3<double>(a, s) : go_stage3<float>(a, s);
}

hipError_t launch_euler_rhs3(const LoopDesc &d, const Box &b, int dtype, hipStream_t s) {
    if (b.nb <= 0) return hipSuccess;
    return dtype == TC_F64 ? rhs3_t<double>(d, b, s) : rhs3_t<float>(d, b, s);
}

}  // namespace tc
