// Fused Chebyshev steps of the heat-conduction preconditioner (2D).
//
// A run of the chain [ghost fill of sd, TEA_P1, TEA_P2] x steps becomes one
// launch.  A workgroup owns kChebTX x kChebTY cells and loads the region H
// cells around them (H >= steps): the face coefficients and rt into
// registers, the direction sd into LDS.  Each step computes, for every
// region cell, A sd with the arithmetic of TEA_P1 (diagonal first, then the
// east, west, north and south terms as fmas), rt -= A sd, z += sd on the
// owned cells, and the next direction al sd + be rt (TEA_P2) into the other
// LDS buffer.  A neighbour outside the domain is the reflective ghost, which
// holds the cell itself; a neighbour outside the region is taken as the cell
// itself too, which is wrong, but the wrong values move one cell inwards per
// step and never reach the owned cells.  The last step's fill is also stored:
// every ghost cell of sd whose mirror cell this workgroup owns.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace tc {

namespace {

__device__ __forceinline__ int cheb_tile(int i, int nb) {
    // XCD-aware order: hardware block i runs on XCD i % 8; XCD k gets a
    // contiguous range of tiles, so neighbouring tiles share its L2
    const int q = nb >> 3, r = nb & 7, xcd = i & 7, k = i >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

template <typename T>
__device__ __forceinline__ T fmaC(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaC<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

// Per-cell flags: inside the domain, owned, and which of the east, west,
// north and south neighbours are other region cells (else the cell itself).
enum : unsigned { kAct = 1, kOwn = 2, kE = 4, kW = 8, kN = 16, kS = 32 };

template <typename T, int H>
__global__ void __launch_bounds__(256) cheb2_kernel(ChebArgs a) {
    constexpr int RW = kChebTX + 2 * H, RH = kChebTY + 2 * H, RC = RW * RH;
    constexpr int PER = (RC + 255) / 256;
    __shared__ T v[2][RC];
    const int t = cheb_tile(blockIdx.x, gridDim.x);
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int rx0 = tx * kChebTX - H, ry0 = ty * kChebTY - H;  // region origin
    const T *kx = (const T *)a.kx, *ky = (const T *)a.ky;
    const T *sd = (const T *)a.sd_in, *rti = (const T *)a.rt_in;
    T *zp = (T *)a.z;
    const int n0 = a.n0, n1 = a.n1;
    T ke[PER], kw[PER], kn[PER], ks[PER], rt[PER], z[PER];
    unsigned fl[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = (int)threadIdx.x + 256 * k;
        const int lx = i % RW, ly = i / RW;
        const int x = rx0 + lx, y = ry0 + ly;
        unsigned f = 0;
        if (i < RC && x >= 0 && x < n0 && y >= 0 && y < n1) {
            f |= kAct;
            if (lx >= H && lx < H + kChebTX && ly >= H && ly < H + kChebTY) f |= kOwn;
            if (x + 1 < n0 && lx + 1 < RW) f |= kE;
            if (x > 0 && lx > 0) f |= kW;
            if (y + 1 < n1 && ly + 1 < RH) f |= kN;
            if (y > 0 && ly > 0) f |= kS;
        }
        fl[k] = f;
        z[k] = (T)0;
        if (f & kAct) {
            ke[k] = kx[(x + 1) + (int64_t)y * a.skx];
            kw[k] = kx[x + (int64_t)y * a.skx];
            kn[k] = ky[x + (int64_t)(y + 1) * a.sky];
            ks[k] = ky[x + (int64_t)y * a.sky];
            if (a.start) {
                // TEA_PRECON_INIT: rt = r, sd = r / theta, z = 0
                T rv = ((const T *)a.r)[x + (int64_t)y * a.sr];
                if (a.update) {
                    // TEA_CG_UPDATE before it: r -= alpha w (every region
                    // cell), x += alpha p (owned cells)
                    const T al = (T)a.alpha;
                    rv = fmaC<T>(-al, ((const T *)a.w)[x + (int64_t)y * a.sw], rv);
                    if (f & kOwn) {
                        T *xp = (T *)a.x + x + (int64_t)y * a.sx;
                        *xp = fmaC<T>(al, ((const T *)a.p)[x + (int64_t)y * a.sp], *xp);
                        ((T *)a.r_out)[x + (int64_t)y * a.sro] = rv;
                    }
                }
                rt[k] = rv;
                v[0][i] = rv / (T)a.theta;
            } else {
                rt[k] = rti[x + (int64_t)y * a.srt_in];
                if (f & kOwn) z[k] = zp[x + (int64_t)y * a.sz];
                v[0][i] = sd[x + (int64_t)y * a.ssd_in];
            }
        }
    }
    __syncthreads();
    T *sdo = (T *)a.sd_out;
    const int h = a.h;
    int buf = 0;
    for (int j = 0; j < a.steps; ++j) {
        const bool p2 = j + 1 < a.steps || a.last_p2;
        const T al = (T)a.al[j], be = (T)a.be[j];
        const T *vv = v[buf];
        T *vn = v[buf ^ 1];
        if (j + 1 == a.steps) {
            // the last step's ghost fill: ghost (gx, gy) holds sd at its
            // mirror cell (x: -1 - g or 2 n - 1 - g, y alike)
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                if (!(fl[k] & kOwn)) continue;
                const int i = (int)threadIdx.x + 256 * k;
                const int x = rx0 + i % RW, y = ry0 + i / RW;
                const bool xl = x < h, xr = x >= n0 - h, yl = y < h, yr = y >= n1 - h;
                if (!(xl || xr || yl || yr)) continue;
                const T val = vv[i];
                const int gx[2] = {x, xl ? -1 - x : 2 * n0 - 1 - x};
                const int gy[2] = {y, yl ? -1 - y : 2 * n1 - 1 - y};
                const int nx = (xl || xr) ? 2 : 1, ny = (yl || yr) ? 2 : 1;
                for (int b = 0; b < ny; ++b)
                    for (int c = 0; c < nx; ++c)
                        if (b + c > 0) sdo[gx[c] + (int64_t)gy[b] * a.ssd_out] = val;
            }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const unsigned f = fl[k];
            if (!(f & kAct)) continue;
            const int i = (int)threadIdx.x + 256 * k;
            T diag = (T)1 + ke[k];
            diag = diag + kw[k];
            diag = diag + kn[k];
            diag = diag + ks[k];
            const T vc = vv[i];
            T av = diag * vc;
            av = fmaC<T>(-ke[k], vv[(f & kE) ? i + 1 : i], av);
            av = fmaC<T>(-kw[k], vv[(f & kW) ? i - 1 : i], av);
            av = fmaC<T>(-kn[k], vv[(f & kN) ? i + RW : i], av);
            av = fmaC<T>(-ks[k], vv[(f & kS) ? i - RW : i], av);
            const T rtv = rt[k] - av;
            rt[k] = rtv;
            if (f & kOwn) z[k] = z[k] + vc;
            if (p2) vn[i] = fmaC<T>(al, vc, be * rtv);
        }
        __syncthreads();
        if (p2) buf ^= 1;
    }
    T *rto = (T *)a.rt_out;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (!(fl[k] & kOwn)) continue;
        const int i = (int)threadIdx.x + 256 * k;
        const int64_t x = rx0 + i % RW, y = ry0 + i / RW;
        rto[x + y * a.srt_out] = rt[k];
        zp[x + y * a.sz] = z[k];
        sdo[x + y * a.ssd_out] = v[buf][i];
    }
}

template <typename T, int H>
hipError_t go_cheb2(const ChebArgs &in, hipStream_t s) {
    ChebArgs a = in;
    a.ntx = (a.n0 + kChebTX - 1) / kChebTX;
    a.nty = (a.n1 + kChebTY - 1) / kChebTY;
    const int nb = a.ntx * a.nty;
    if (nb <= 0 || a.steps <= 0) return hipSuccess;
    hipLaunchKernelGGL((cheb2_kernel<T, H>), dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t cheb2_t(const ChebArgs &a, hipStream_t s) {
    switch (cheb_halo(a.steps)) {
    case 3: return go_cheb2<T, 3>(a, s);
    case 5: return go_cheb2<T, 5>(a, s);
    case 7: return go_cheb2<T, 7>(a, s);
    default: return go_cheb2<T, 9>(a, s);
    }
}

}  // namespace

hipError_t launch_cheb2(const ChebArgs &a, int dtype, hipStream_t s) {
    if (a.steps < 1 || a.steps > kChebMaxSteps || a.h < 1 || a.h > kChebMaxSteps) return hipErrorInvalidValue;
    return dtype == TC_F64 ? cheb2_t<double>(a, s) : cheb2_t<float>(a, s);
}

}  // namespace tc
