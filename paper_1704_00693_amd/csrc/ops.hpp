// Point operations of the closed op vocabulary (see tilechain.h), as device
// functors: Op::run(d, x, y, z, red) evaluates one point of a loop described
// by d, reading and writing through d.arg[a].ptr with the strides d.arg[a].sy
// and d.arg[a].sz (logical coordinates).  The per-loop kernels (kernels.hip)
// pass descriptors of device buffers; the staged tiles (staged.hip) pass the
// same descriptors re-pointed at workgroup-local (LDS) copies, so both run
// exactly the same arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include "dd.hpp"
#include "tc_internal.hpp"

namespace tc {

// ---------------------------------------------------------------------------
// point operations
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T *P(const LoopDesc &d, int a) {
    return (T *)d.arg[a].ptr;
}

// A descriptor whose dataset pointers all address workgroup-local memory
// (LDS): the same layout, but P<T>() returns LDS-qualified pointers, so the
// functors' accesses compile to LDS instructions instead of generic ones.
struct LdsDesc : LoopDesc {};
template <typename T>
using lds_ptr = __attribute__((address_space(3))) T *;
template <typename T>
__device__ __forceinline__ lds_ptr<T> P(const LdsDesc &d, int a) {
    return (lds_ptr<T>)(T *)d.arg[a].ptr;
}

__device__ __forceinline__ int64_t IX(const LoopDesc &d, int a, int x, int y, int z) {
    return (int64_t)x + (int64_t)y * d.arg[a].sy + (int64_t)z * d.arg[a].sz;
}

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

// Weighted sum: acc = fma(w, in[x+q], acc) over inputs and stencil points in
// order.  Common stencil sizes are unrolled so the loads issue together; the
// fma chain keeps its order.
template <typename T, int NP, class Desc, class Ptr>
__device__ __forceinline__ T wsum_input(const Desc &d, Ptr p, int q0, T acc) {
    T v[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) v[k] = p[d.off[q0 + k]];
#pragma unroll
    for (int k = 0; k < NP; ++k) acc = fmaT<T>((T)d.prm[q0 + k], v[k], acc);
    return acc;
}

template <typename T>
struct OpWsum {
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        T acc = (T)0;
        for (int a = 1; a < d.nargs; ++a) {
            const auto p = P<T>(d, a) + IX(d, a, x, y, z);
            const int q0 = d.pt0[a];
            switch (d.npts[a]) {
            case 5: acc = wsum_input<T, 5>(d, p, q0, acc); break;
            case 9: acc = wsum_input<T, 9>(d, p, q0, acc); break;
            case 7: acc = wsum_input<T, 7>(d, p, q0, acc); break;
            case 13: acc = wsum_input<T, 13>(d, p, q0, acc); break;
            default:
                for (int k = 0; k < d.npts[a]; ++k) acc = fmaT<T>((T)d.prm[q0 + k], p[d.off[q0 + k]], acc);
            }
        }
        P<T>(d, 0)[IX(d, 0, x, y, z)] = acc;
    }
};

// COPY with possible conversion: arg0 type TO, arg1 type FROM
template <typename TO, typename FROM>
struct OpCopy {
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        P<TO>(d, 0)[IX(d, 0, x, y, z)] = (TO)P<FROM>(d, 1)[IX(d, 1, x, y, z)];
    }
};

template <typename T>
struct OpAxpby {
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        auto yp = P<T>(d, 0) + IX(d, 0, x, y, z);
        T xv = P<T>(d, 1)[IX(d, 1, x, y, z)];
        *yp = fmaT<T>((T)d.prm[0], xv, (T)d.prm[1] * *yp);
    }
};

template <typename T>
struct OpDot {
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *r) {
        double a = (double)P<T>(d, 0)[IX(d, 0, x, y, z)];
        double b = (double)P<T>(d, 1)[IX(d, 1, x, y, z)];
        dd_add_prod(r[0], a, b);
    }
};

template <typename T>
struct OpSum {
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *r) {
        dd_add(r[0], (double)P<T>(d, 0)[IX(d, 0, x, y, z)]);
    }
};

template <typename T>
struct OpHaloReflect {
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        const int axis = (int)d.prm[0], side = (int)d.prm[1], n = (int)d.prm[2];
        int c[3] = {x, y, z};
        int s[3] = {x, y, z};
        s[axis] = side == 0 ? -1 - c[axis] : 2 * n - 1 - c[axis];
        auto v = P<T>(d, 0);
        v[IX(d, 0, x, y, z)] = v[IX(d, 0, s[0], s[1], s[2])];
    }
};

// ---- heat conduction ------------------------------------------------------
// K arguments are the first ndim dataset arguments.
template <typename T, class Desc>
__device__ __forceinline__ T tea_apply(const Desc &d, int vi, int x, int y, int z) {
    const auto kx = P<T>(d, 0);
        const auto ky = P<T>(d, 1);
    const T ke = kx[IX(d, 0, x + 1, y, z)], kw = kx[IX(d, 0, x, y, z)];
    const T kn = ky[IX(d, 1, x, y + 1, z)], ks = ky[IX(d, 1, x, y, z)];
    const auto v = P<T>(d, vi);
    const int64_t c = IX(d, vi, x, y, z);
    const int64_t sy = d.arg[vi].sy;
    T diag = (T)1 + ke;
    diag = diag + kw;
    diag = diag + kn;
    diag = diag + ks;
    T kt = 0, kb = 0;
    const bool three = d.ndim == 3;
    if (three) {
        const auto kz = P<T>(d, 2);
        kt = kz[IX(d, 2, x, y, z + 1)];
        kb = kz[IX(d, 2, x, y, z)];
        diag = diag + kt;
        diag = diag + kb;
    }
    T av = diag * v[c];
    av = fmaT<T>(-ke, v[c + 1], av);
    av = fmaT<T>(-kw, v[c - 1], av);
    av = fmaT<T>(-kn, v[c + sy], av);
    av = fmaT<T>(-ks, v[c - sy], av);
    if (three) {
        const int64_t sz = d.arg[vi].sz;
        av = fmaT<T>(-kt, v[c + sz], av);
        av = fmaT<T>(-kb, v[c - sz], av);
    }
    return av;
}

template <typename T>
struct OpTeaInit {  // rho, e, u0, u
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        T t = P<T>(d, 1)[IX(d, 1, x, y, z)] * P<T>(d, 0)[IX(d, 0, x, y, z)];
        P<T>(d, 2)[IX(d, 2, x, y, z)] = t;
        P<T>(d, 3)[IX(d, 3, x, y, z)] = t;
    }
};

template <typename T>
struct OpTeaK {  // rho, Kx, Ky[, Kz]; prm r
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        const auto rho = P<T>(d, 0);
        const int64_t c = IX(d, 0, x, y, z);
        const T rc = rho[c];
        const T two_r = (T)2 * (T)d.prm[0];
        P<T>(d, 1)[IX(d, 1, x, y, z)] = two_r / (rho[c - 1] + rc);
        P<T>(d, 2)[IX(d, 2, x, y, z)] = two_r / (rho[c - d.arg[0].sy] + rc);
        if (d.ndim == 3) P<T>(d, 3)[IX(d, 3, x, y, z)] = two_r / (rho[c - d.arg[0].sz] + rc);
    }
};

template <typename T>
struct OpTeaResid {  // K.., x, b, r
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        const int nd = d.ndim;
        T av = tea_apply<T>(d, nd, x, y, z);
        P<T>(d, nd + 2)[IX(d, nd + 2, x, y, z)] = P<T>(d, nd + 1)[IX(d, nd + 1, x, y, z)] - av;
    }
};

template <typename T>
struct OpTeaMatvecDot {  // K.., p, w, red
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *r) {
        const int nd = d.ndim;
        T av = tea_apply<T>(d, nd, x, y, z);
        P<T>(d, nd + 1)[IX(d, nd + 1, x, y, z)] = av;
        dd_add_prod(r[0], (double)P<T>(d, nd)[IX(d, nd, x, y, z)], (double)av);
    }
};

template <typename T>
struct OpTeaP1 {  // K.., sd, rt, z
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        const int nd = d.ndim;
        T av = tea_apply<T>(d, nd, x, y, z);
        auto rt = P<T>(d, nd + 1) + IX(d, nd + 1, x, y, z);
        *rt = *rt - av;
        auto zz = P<T>(d, nd + 2) + IX(d, nd + 2, x, y, z);
        *zz = *zz + P<T>(d, nd)[IX(d, nd, x, y, z)];
    }
};

template <typename T>
struct OpTeaP2 {  // sd, rt; alpha, beta
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        auto sd = P<T>(d, 0) + IX(d, 0, x, y, z);
        T rt = P<T>(d, 1)[IX(d, 1, x, y, z)];
        *sd = fmaT<T>((T)d.prm[0], *sd, (T)d.prm[1] * rt);
    }
};

template <typename T>
struct OpTeaPreconInit {  // r, rt, sd, z; theta
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        T v = P<T>(d, 0)[IX(d, 0, x, y, z)];
        P<T>(d, 1)[IX(d, 1, x, y, z)] = v;
        P<T>(d, 2)[IX(d, 2, x, y, z)] = v / (T)d.prm[0];
        P<T>(d, 3)[IX(d, 3, x, y, z)] = (T)0;
    }
};

template <typename T>
struct OpTeaCgUpdate {  // x, r, p, w; alpha
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        const T al = (T)d.prm[0];
        auto xp = P<T>(d, 0) + IX(d, 0, x, y, z);
        auto rp = P<T>(d, 1) + IX(d, 1, x, y, z);
        *xp = fmaT<T>(al, P<T>(d, 2)[IX(d, 2, x, y, z)], *xp);
        *rp = fmaT<T>(-al, P<T>(d, 3)[IX(d, 3, x, y, z)], *rp);
    }
};

template <typename T>
struct OpTeaCgP {  // p, z; beta
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        auto pp = P<T>(d, 0) + IX(d, 0, x, y, z);
        *pp = fmaT<T>((T)d.prm[0], *pp, P<T>(d, 1)[IX(d, 1, x, y, z)]);
    }
};

template <typename T>
struct OpTeaGersh {  // K.., red(max)
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *r) {
        const auto kx = P<T>(d, 0);
        const auto ky = P<T>(d, 1);
        T s = kx[IX(d, 0, x + 1, y, z)] + kx[IX(d, 0, x, y, z)];
        s = s + ky[IX(d, 1, x, y + 1, z)];
        s = s + ky[IX(d, 1, x, y, z)];
        if (d.ndim == 3) {
            const auto kz = P<T>(d, 2);
            s = s + kz[IX(d, 2, x, y, z + 1)];
            s = s + kz[IX(d, 2, x, y, z)];
        }
        double g = (double)fmaT<T>((T)2, s, (T)1);
        r[0].hi = fmax(r[0].hi, g);
    }
};

// ---- compressible Euler ----------------------------------------------------
template <typename T>
struct OpEulerPrim {  // Q_0..Q_{D+1}, u_1..u_D, p; gm1
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        const int D = d.ndim;
        const T ri = (T)1 / P<T>(d, 0)[IX(d, 0, x, y, z)];
        T u[3], m[3];
        for (int k = 0; k < D; ++k) {
            m[k] = P<T>(d, 1 + k)[IX(d, 1 + k, x, y, z)];
            u[k] = m[k] * ri;
        }
        T ke = m[D - 1] * u[D - 1];
        for (int k = D - 2; k >= 0; --k) ke = fmaT<T>(m[k], u[k], ke);
        for (int k = 0; k < D; ++k) P<T>(d, D + 2 + k)[IX(d, D + 2 + k, x, y, z)] = u[k];
        const T e = P<T>(d, D + 1)[IX(d, D + 1, x, y, z)];
        P<T>(d, 2 * D + 2)[IX(d, 2 * D + 2, x, y, z)] = (T)d.prm[0] * fmaT<T>((T)-0.5, ke, e);
    }
};

template <typename T>
struct OpEulerRhs {  // R, Q_c, u_1..u_D, p; c, s
    template <class Desc>
    static __device__ __forceinline__ T flux(const Desc &d, int c, int ax, int x, int y, int z) {
        const int D = d.ndim;
        const T ud = P<T>(d, 2 + ax)[IX(d, 2 + ax, x, y, z)];
        T f = P<T>(d, 1)[IX(d, 1, x, y, z)] * ud;
        if (c == ax + 1) f = f + P<T>(d, 2 + D)[IX(d, 2 + D, x, y, z)];
        if (c == D + 1) f = fmaT<T>(P<T>(d, 2 + D)[IX(d, 2 + D, x, y, z)], ud, f);
        return f;
    }
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        const int D = d.ndim;
        const int c = (int)d.prm[0];
        T acc = (T)0;
        for (int ax = 0; ax < D; ++ax) {
            const int ex = ax == 0, ey = ax == 1, ez = ax == 2;
            const T fp1 = flux(d, c, ax, x + ex, y + ey, z + ez);
            const T fm1 = flux(d, c, ax, x - ex, y - ey, z - ez);
            const T fp2 = flux(d, c, ax, x + 2 * ex, y + 2 * ey, z + 2 * ez);
            const T fm2 = flux(d, c, ax, x - 2 * ex, y - 2 * ey, z - 2 * ez);
            const T t1 = fp1 - fm1;
            const T t2 = fp2 - fm2;
            const T g = (T)8 * t1 - t2;
            acc = ax == 0 ? g : acc + g;
        }
        P<T>(d, 0)[IX(d, 0, x, y, z)] = -acc * (T)d.prm[1];
    }
};

template <typename T>
struct OpRkStage {  // Q0, Q, R; a, b, dt
    template <class Desc>
    static __device__ __forceinline__ void run(const Desc &d, int x, int y, int z, DD *) {
        auto q = P<T>(d, 1) + IX(d, 1, x, y, z);
        const T t = fmaT<T>((T)d.prm[2], P<T>(d, 2)[IX(d, 2, x, y, z)], *q);
        *q = fmaT<T>((T)d.prm[0], P<T>(d, 0)[IX(d, 0, x, y, z)], (T)d.prm[1] * t);
    }
};

}  // namespace tc
