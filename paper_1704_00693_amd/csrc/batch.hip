// Kernels of the batched heat-conduction solves (scheme in batch.hpp).
//
// Every kernel strides over the current tile list (its length is read from
// device memory, so a captured graph stays valid while the list changes);
// a tile is 64 x 4 cells of one instance, one workgroup, and the workgroup
// skips tiles whose instance is not in a state the kernel serves.  Per-tile
// reduction partials (double-double) go to part[4 * tile + {0,1}] and
// part[4 * tile + {2,3}]; per-instance finalize kernels (one workgroup per
// instance slot) combine them in tile order and advance the state machine.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "dd.hpp"

namespace tc {

namespace {

constexpr unsigned long long kGamma = 0x9E3779B97F4A7C15ull;
constexpr unsigned long long kM1 = 0xBF58476D1CE4E5B9ull;
constexpr unsigned long long kM2 = 0x94D049BB133111EBull;

// Output number k (k >= 1) of the SplitMix64 stream with state s (Steele,
// Lea, Flood 2014), as a double in [0, 1) from its top 53 bits.
__device__ __forceinline__ double splitmix_unit(unsigned long long s, unsigned long long k) {
    unsigned long long z = s + k * kGamma;
    z = (z ^ (z >> 30)) * kM1;
    z = (z ^ (z >> 27)) * kM2;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

template <typename T>
__device__ __forceinline__ T fmaB(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaB<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

struct Cell {
    int x, y, z;
    bool ok;
    int64_t c;
    int64_t e, w, n, s, t, b;  // offsets of the neighbours, mirrored at the domain boundary
};

__device__ __forceinline__ Cell cell_of(const BInst &I, const BTile &tl) {
    Cell k;
    k.x = tl.tx * kBTX + (int)(threadIdx.x & (kBTX - 1));
    k.y = tl.ty * kBTY + (int)(threadIdx.x / kBTX);
    k.z = tl.tz;
    k.ok = k.x < I.n && k.y < I.n;
    k.c = I.org + k.x + (int64_t)k.y * I.sy + (int64_t)k.z * I.sz;
    // a reflective ghost cell holds the value of the cell it mirrors
    k.e = k.x + 1 < I.n ? 1 : 0;
    k.w = k.x > 0 ? -1 : 0;
    k.n = k.y + 1 < I.n ? I.sy : 0;
    k.s = k.y > 0 ? -I.sy : 0;
    k.t = (I.ndim == 3 && k.z + 1 < I.n) ? I.sz : 0;
    k.b = (I.ndim == 3 && k.z > 0) ? -I.sz : 0;
    return k;
}

// (A v) at a cell: diagonal 1 + sum of face coefficients (left to right),
// then the neighbour terms E, W, N, S[, T, B] as fmas.
template <typename T>
__device__ __forceinline__ T apply_A(const BInst &I, const T *kx, const T *ky, const T *kz, const T *v,
                                     const Cell &k) {
    const int64_t c = k.c;
    const T ke = kx[c + 1], kw = kx[c];
    const T kn = ky[c + I.sy], ks = ky[c];
    T diag = (T)1 + ke;
    diag = diag + kw;
    diag = diag + kn;
    diag = diag + ks;
    T kt = 0, kb = 0;
    const bool three = I.ndim == 3;
    if (three) {
        kt = kz[c + I.sz];
        kb = kz[c];
        diag = diag + kt;
        diag = diag + kb;
    }
    T av = diag * v[c];
    av = fmaB<T>(-ke, v[c + k.e], av);
    av = fmaB<T>(-kw, v[c + k.w], av);
    av = fmaB<T>(-kn, v[c + k.n], av);
    av = fmaB<T>(-ks, v[c + k.s], av);
    if (three) {
        av = fmaB<T>(-kt, v[c + k.t], av);
        av = fmaB<T>(-kb, v[c + k.b], av);
    }
    return av;
}

__device__ __forceinline__ bool serves(const BInst &I, unsigned mask) { return (mask >> I.state) & 1u; }

// First tile of a workgroup's grid-stride walk over the tile list.  Hardware
// block b runs on XCD b % 8; when the grid is a multiple of 8, XCD k takes
// the logical blocks [k G/8, (k+1) G/8), so consecutive tiles (neighbours,
// whose borders overlap) are walked by one XCD and share its L2.
__device__ __forceinline__ int64_t first_tile() {
    const unsigned g = gridDim.x, b = blockIdx.x;
    return (g & 7u) ? b : (b & 7u) * (g >> 3) + (b >> 3);
}

__device__ __forceinline__ void write_partial(double *part, int64_t t, int slot, DD v) {
    if (threadIdx.x == 0) {
        part[4 * t + 2 * slot] = v.hi;
        part[4 * t + 2 * slot + 1] = v.lo;
    }
}

// ---- set-up ---------------------------------------------------------------
// density -> r, energy -> u (counter-based draws, density first), then
// u0 = u = e * rho; partial u0 . u0 (slot 0).
__global__ void __launch_bounds__(256) bk_init(BInst *insts, const BTile *tiles, const int64_t *ntiles, double *part) {
    const int64_t nt = *ntiles;
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        if (!serves(I, 1u << B_INIT)) continue;
        const Cell k = cell_of(I, tl);
        DD acc = red_identity(TC_RED_SUM);
        if (k.ok) {
            const unsigned long long cells = (unsigned long long)I.n * I.n * (I.ndim == 3 ? I.n : 1);
            const unsigned long long id = (unsigned long long)k.x + (unsigned long long)I.n * (k.y + (unsigned long long)I.n * k.z);
            const double a0 = 0.1, b0 = 1.0, a1 = 1.0, b1 = 2.0;
            const double rho = a0 + (b0 - a0) * splitmix_unit(I.seed, id + 1);
            const double e = a1 + (b1 - a1) * splitmix_unit(I.seed, cells + id + 1);
            I.r[k.c] = rho;
            const double v = e * rho;
            I.u0[k.c] = v;
            I.u[k.c] = v;
            // the first search direction is p = 0 * p + z
            if (I.mixed)
                ((float *)I.p)[k.c] = 0.0f;
            else
                ((double *)I.p)[k.c] = 0.0;
            dd_add_prod(acc, v, v);
        }
        write_partial(part, t, 0, block_reduce(TC_RED_SUM, acc));
    }
}

// Face coefficients K = 2 rx / (rho_left + rho_right) on faces 0..n of every
// axis (face i lies between cells i-1 and i; ghost densities mirror).
template <typename T>
__global__ void __launch_bounds__(256) bk_faces(BInst *insts, const BTile *tiles, const int64_t *ntiles) {
    const int64_t nt = *ntiles;
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        if (!serves(I, 1u << B_INIT)) continue;
        const Cell k = cell_of(I, tl);
        if (!k.ok) continue;
        const double two_r = 2.0 * I.rx;
        const double *rho = I.r;
        const double rc = rho[k.c];
        T *kxi = (T *)I.kxi, *kyi = (T *)I.kyi, *kzi = (T *)I.kzi;
        const bool mixed = I.mixed != 0;
        auto put = [&](double *K, T *Ki, int64_t at, double v) {
            K[at] = v;
            if (mixed) Ki[at] = (T)v;
        };
        put(I.kx, kxi, k.c, two_r / (rho[k.c + k.w] + rc));
        put(I.ky, kyi, k.c, two_r / (rho[k.c + k.s] + rc));
        if (I.ndim == 3) put(I.kz, kzi, k.c, two_r / (rho[k.c + k.b] + rc));
        // the last face of each axis: both sides are the boundary cell
        if (k.x == I.n - 1) put(I.kx, kxi, k.c + 1, two_r / (rc + rc));
        if (k.y == I.n - 1) put(I.ky, kyi, k.c + I.sy, two_r / (rc + rc));
        if (I.ndim == 3 && k.z == I.n - 1) put(I.kz, kzi, k.c + I.sz, two_r / (rc + rc));
    }
}

// Gershgorin bound of every cell, 1 + 2 * (sum of its face coefficients);
// partial maximum (slot 1).
__global__ void __launch_bounds__(256) bk_gersh(BInst *insts, const BTile *tiles, const int64_t *ntiles, double *part) {
    const int64_t nt = *ntiles;
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        if (!serves(I, 1u << B_INIT)) continue;
        const Cell k = cell_of(I, tl);
        DD m = red_identity(TC_RED_MAX);
        if (k.ok) {
            double s = I.kx[k.c + 1] + I.kx[k.c];
            s = s + I.ky[k.c + I.sy];
            s = s + I.ky[k.c];
            if (I.ndim == 3) {
                s = s + I.kz[k.c + I.sz];
                s = s + I.kz[k.c];
            }
            m.hi = __builtin_fma(2.0, s, 1.0);
        }
        write_partial(part, t, 1, block_reduce(TC_RED_MAX, m));
    }
}

// ---- FP64 residual: r = b - A x; partial r . r (slot 0) -------------------
// Mixed mode also writes the FP32 copy of r and clears the correction d.
template <typename T>
__global__ void __launch_bounds__(256) bk_resid(BInst *insts, const BTile *tiles, const int64_t *ntiles, double *part) {
    const int64_t nt = *ntiles;
    const unsigned mask = (1u << B_RESID) | (1u << B_OUTER) | (1u << B_VERIFY);
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        if (!serves(I, mask)) continue;
        const Cell k = cell_of(I, tl);
        DD acc = red_identity(TC_RED_SUM);
        if (k.ok) {
            const double av = apply_A<double>(I, I.kx, I.ky, I.kz, I.u, k);
            const double rv = I.u0[k.c] - av;
            I.r[k.c] = rv;
            dd_add_prod(acc, rv, rv);
            if (I.mixed && I.state != B_VERIFY) {
                ((T *)I.ri)[k.c] = (T)rv;
                ((T *)I.xi)[k.c] = (T)0;
            }
        }
        write_partial(part, t, 0, block_reduce(TC_RED_SUM, acc));
    }
}

// Mixed mode, start of a refinement step: x += d in FP64.
template <typename T>
__global__ void __launch_bounds__(256) bk_apply_correction(BInst *insts, const BTile *tiles, const int64_t *ntiles) {
    const int64_t nt = *ntiles;
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        if (!serves(I, 1u << B_OUTER)) continue;
        const Cell k = cell_of(I, tl);
        if (!k.ok) continue;
        const double d = (double)((const T *)I.xi)[k.c];
        I.u[k.c] = __builtin_fma(1.0, d, 1.0 * I.u[k.c]);
    }
}

// ---- PPCG sweeps (type T) -------------------------------------------------
// p = beta p + z
template <typename T>
__global__ void __launch_bounds__(256) bk_cg_p(BInst *insts, const BTile *tiles, const int64_t *ntiles) {
    const int64_t nt = *ntiles;
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        if (!serves(I, 1u << B_INNER)) continue;
        const Cell k = cell_of(I, tl);
        if (!k.ok) continue;
        T *p = (T *)I.p;
        p[k.c] = fmaB<T>((T)I.beta, p[k.c], ((const T *)I.z)[k.c]);
    }
}

// w = A p; partial p . w (slot 0)
template <typename T>
__global__ void __launch_bounds__(256) bk_matvec(BInst *insts, const BTile *tiles, const int64_t *ntiles, double *part) {
    const int64_t nt = *ntiles;
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        if (!serves(I, 1u << B_INNER)) continue;
        const Cell k = cell_of(I, tl);
        DD acc = red_identity(TC_RED_SUM);
        if (k.ok) {
            const T *p = (const T *)I.p;
            const T av = apply_A<T>(I, (const T *)I.kxi, (const T *)I.kyi, (const T *)I.kzi, p, k);
            ((T *)I.w)[k.c] = av;
            dd_add_prod(acc, (double)p[k.c], (double)av);
        }
        write_partial(part, t, 0, block_reduce(TC_RED_SUM, acc));
    }
}

// INNER: x += alpha p, r -= alpha w; then (INNER and INNER_START) the
// preconditioner's start: rt = r, sd = rt / theta, z = 0 (skipped for 2D
// instances when skip2d is set: the first fused Chebyshev launch starts from
// r itself).
template <typename T>
__global__ void __launch_bounds__(256) bk_update_init(BInst *insts, const BTile *tiles, const int64_t *ntiles,
                                                      int skip2d) {
    const int64_t nt = *ntiles;
    const unsigned mask = (1u << B_INNER) | (1u << B_INNER_START);
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        if (!serves(I, mask)) continue;
        const Cell k = cell_of(I, tl);
        if (!k.ok) continue;
        T *x = (T *)I.xi, *r = (T *)I.ri;
        T rv = r[k.c];
        if (I.state == B_INNER) {
            const T al = (T)I.alpha;
            x[k.c] = fmaB<T>(al, ((const T *)I.p)[k.c], x[k.c]);
            rv = fmaB<T>(-al, ((const T *)I.w)[k.c], rv);
            r[k.c] = rv;
        }
        if (skip2d && I.ndim == 2) continue;
        ((T *)I.rt)[k.c] = rv;
        ((T *)I.sd0)[k.c] = rv / (T)I.theta;
        ((T *)I.z)[k.c] = (T)0;
    }
}

// Chebyshev step j (1-based): rt -= A sd, z += sd, then for j < steps the
// next direction sd' = al_j sd + be_j rt (into the other sd buffer); the last
// step adds the partials r . z (slot 0) and r . r (slot 1).
template <typename T>
__global__ void __launch_bounds__(256) bk_cheb(BInst *insts, const BTile *tiles, const int64_t *ntiles, double *part,
                                               int j) {
    const int64_t nt = *ntiles;
    const unsigned mask = (1u << B_INNER) | (1u << B_INNER_START);
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        if (!serves(I, mask) || j > I.cheb_steps) continue;
        const bool last = j == I.cheb_steps;
        const Cell k = cell_of(I, tl);
        DD rz = red_identity(TC_RED_SUM), rr = red_identity(TC_RED_SUM);
        if (k.ok) {
            const T *sd = (const T *)((j & 1) ? I.sd0 : I.sd1);
            T *z = (T *)I.z;
            if (!last) {
                T *sdn = (T *)((j & 1) ? I.sd1 : I.sd0);
                const T av = apply_A<T>(I, (const T *)I.kxi, (const T *)I.kyi, (const T *)I.kzi, sd, k);
                T *rt = (T *)I.rt;
                const T rtv = rt[k.c] - av;
                rt[k.c] = rtv;
                z[k.c] = z[k.c] + sd[k.c];
                sdn[k.c] = fmaB<T>((T)I.al[j - 1], sd[k.c], (T)I.be[j - 1] * rtv);
            } else {
                // the last step's rt and direction are never read: only z
                // and the partials
                const T zv = z[k.c] + sd[k.c];
                z[k.c] = zv;
                const T rv = ((const T *)I.ri)[k.c];
                dd_add_prod(rz, (double)rv, (double)zv);
                dd_add_prod(rr, (double)rv, (double)rv);
            }
        }
        if (last) {
            write_partial(part, t, 0, block_reduce(TC_RED_SUM, rz));
            write_partial(part, t, 1, block_reduce(TC_RED_SUM, rr));
        }
    }
}

// Chebyshev steps j0 .. j1-1 (j1 - j0 <= H and odd) of 2D instances; the
// last step, with its reductions, stays with bk_cheb.  A workgroup takes a
// tile of kFTX x FTY owned cells and the H cells around it (inside the
// domain): face coefficients, rt and the direction are loaded once (z for
// the owned cells only: no neighbour needs it), each step exchanges the
// direction through LDS, and rt, z and the last direction are stored for the
// owned cells.  Neighbouring tiles read this tile's cells as their border,
// so rt alternates between two buffers (rt_alt: read rt2, write rt) and the
// direction between sd0 and sd1 (an odd number of steps lands in the other
// one).  A cell at the edge of the loaded region reads itself for a missing
// neighbour, which makes its value wrong, and each step moves the wrong
// values one cell inwards; after at most H steps they have not reached the
// owned cells.  At the domain boundary the mirrored neighbour is the cell
// itself, as in bk_cheb.  Every cell's operations are bk_cheb's, in the same
// order.
template <typename T, int H, int FTY>
__global__ void __launch_bounds__(256) bk_cheb_fused(BInst *insts, const BTile *tiles, const int64_t *ntiles, int j0,
                                                     int j1, int rt_alt, int start) {
    constexpr int RW = kFTX + 2 * H, RH = FTY + 2 * H, RC = RW * RH;
    constexpr int PER = (RC + 255) / 256;
    __shared__ T sdl[2][RC];
    const int64_t nt = *ntiles;
    const unsigned mask = (1u << B_INNER) | (1u << B_INNER_START);
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        const int K = I.cheb_steps;
        if (!serves(I, mask) || I.ndim != 2 || j1 > K) continue;  // the same for the whole workgroup
        const T *rt_in = (const T *)(rt_alt ? I.rt2 : I.rt);
        T *rt_out = (T *)(rt_alt ? I.rt : I.rt2);
        const int rx0 = tl.tx * kFTX - H, ry0 = tl.ty * FTY - H;  // region origin
        const T *kx = (const T *)I.kxi, *ky = (const T *)I.kyi;
        const T *sd = (const T *)((j0 & 1) ? I.sd0 : I.sd1);
        T ke[PER], kw[PER], kn[PER], ks[PER], rt[PER], z[PER];
        int oe[PER], ow[PER], on[PER], os[PER];
        bool act[PER], own[PER];
        int64_t cc[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = (int)threadIdx.x + 256 * k;
            const int lx = i % RW, ly = i / RW;
            const int x = rx0 + lx, y = ry0 + ly;
            act[k] = i < RC && x >= 0 && x < I.n && y >= 0 && y < I.n;
            own[k] = act[k] && lx >= H && lx < H + kFTX && ly >= H && ly < H + FTY;
            cc[k] = I.org + x + (int64_t)y * I.sy;
            oe[k] = (x + 1 < I.n && lx + 1 < RW) ? 1 : 0;
            ow[k] = (x > 0 && lx > 0) ? -1 : 0;
            on[k] = (y + 1 < I.n && ly + 1 < RH) ? RW : 0;
            os[k] = (y > 0 && ly > 0) ? -RW : 0;
            if (act[k]) {
                const int64_t c = cc[k];
                ke[k] = kx[c + 1];
                kw[k] = kx[c];
                kn[k] = ky[c + I.sy];
                ks[k] = ky[c];
                if (start) {
                    // the preconditioner's start, as bk_update_init writes it
                    const T rv = ((const T *)I.ri)[c];
                    rt[k] = rv;
                    z[k] = (T)0;
                    sdl[0][i] = rv / (T)I.theta;
                } else {
                    rt[k] = rt_in[c];
                    if (own[k]) z[k] = ((const T *)I.z)[c];
                    sdl[0][i] = sd[c];
                }
            }
        }
        __syncthreads();
        int buf = 0;
        for (int j = j0; j < j1; ++j) {
            const T al = (T)I.al[j - 1], be = (T)I.be[j - 1];
            const T *v = sdl[buf];
            T *vn = sdl[buf ^ 1];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                if (!act[k]) continue;
                const int i = (int)threadIdx.x + 256 * k;
                T diag = (T)1 + ke[k];
                diag = diag + kw[k];
                diag = diag + kn[k];
                diag = diag + ks[k];
                const T vc = v[i];
                T av = diag * vc;
                av = fmaB<T>(-ke[k], v[i + oe[k]], av);
                av = fmaB<T>(-kw[k], v[i + ow[k]], av);
                av = fmaB<T>(-kn[k], v[i + on[k]], av);
                av = fmaB<T>(-ks[k], v[i + os[k]], av);
                const T rtv = rt[k] - av;
                rt[k] = rtv;
                if (own[k]) z[k] = z[k] + vc;
                vn[i] = fmaB<T>(al, vc, be * rtv);
            }
            __syncthreads();
            buf ^= 1;
        }
        // step j1 - 1 wrote the direction step j1 reads
        T *sdo = (T *)(((j1 - 1) & 1) ? I.sd1 : I.sd0);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (!own[k]) continue;
            const int i = (int)threadIdx.x + 256 * k;
            rt_out[cc[k]] = rt[k];
            ((T *)I.z)[cc[k]] = z[k];
            sdo[cc[k]] = sdl[buf][i];
        }
        __syncthreads();  // the next tile reuses the LDS buffers
    }
}

// Chebyshev steps j0 .. j0+S-1 (S = 1 or 3) of 3D instances; the last step,
// with its reductions, stays with bk_cheb.  A workgroup (f3_threads<T>) takes
// a tile of kF3X x kF3Y owned cells of one z-segment [za, zb) of kF3Z planes
// and marches up the planes: at march m, step s works on plane m - s, so the
// direction a step writes for plane p is there when the next step, one march
// later, needs it as the upper z neighbour of plane p - 1.  Each step level's
// direction lives in LDS, a ring of three planes of the region (the owned
// cells and S cells around them in x and y); rt and z of a cell live in
// registers, a ring of S planes (plane p in slot (p - m0) mod S, so the march
// is unrolled by S and every slot index is a constant), loaded one plane
// ahead.  In FP64 the six face coefficients of a cell join that ring, loaded
// when their plane enters it, with 512-thread workgroups so that two slots
// per thread leave room for them; in FP32 (where the smaller registers keep
// four 256-thread workgroups per CU) every step reads them from memory
// (cached lines by then).  Step s computes the cells within
// S-1-s of the owned ones (in x and y, and in planes around the segment), so
// every neighbour it reads was loaded or written by the step before it.
// Neighbouring tiles and segments read this tile's cells as their border, so
// rt alternates between two buffers (rt_alt: read rt2, write rt) and an odd S
// puts the direction in the other sd buffer.  At the domain boundary the
// mirrored neighbour is the cell itself, as in bk_cheb, and every cell's
// operations are bk_cheb's, in the same order.
template <typename T>
constexpr int f3_threads() {
    return sizeof(T) == 8 ? 512 : 256;
}

template <typename T, int S>
__global__ void __launch_bounds__(f3_threads<T>())
    bk_cheb3_fused(BInst *insts, const BTile *tiles, const int64_t *ntiles, int j0, int rt_alt) {
    constexpr int NT = f3_threads<T>();
    constexpr bool RING = sizeof(T) == 8;  // face coefficients in the register ring
    constexpr int RW = kF3X + 2 * S, RH = kF3Y + 2 * S, RC = RW * RH;
    constexpr int PER = (RC + NT - 1) / NT;
    // per-slot flags: inside the domain, owned, which in-plane neighbours
    // are other region cells (else the cell itself); bits 8..: distance to
    // the owned cells
    enum : unsigned { fAct = 1, fOwn = 2, fE = 4, fW = 8, fN = 16, fS = 32 };
    __shared__ T ring[S][3][RC];
    const int64_t nt = *ntiles;
    const unsigned mask = (1u << B_INNER) | (1u << B_INNER_START);
    for (int64_t t = first_tile(); t < nt; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BInst &I = insts[tl.inst];
        if (!serves(I, mask) || I.ndim != 3 || j0 + S > I.cheb_steps) continue;  // the same for the whole workgroup
        const int n = I.n;
        const int64_t sy = I.sy, sz = I.sz;
        const T *rt_in = (const T *)(rt_alt ? I.rt2 : I.rt);
        T *rt_out = (T *)(rt_alt ? I.rt : I.rt2);
        const T *sdi = (const T *)((j0 & 1) ? I.sd0 : I.sd1);
        T *sdo = (T *)((j0 & 1) ? I.sd1 : I.sd0);
        const T *kx = (const T *)I.kxi, *ky = (const T *)I.kyi, *kz = (const T *)I.kzi;
        T *zp = (T *)I.z;
        const int za = tl.tz * kF3Z, zb = min(n, za + kF3Z);
        int lo[S], hi[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            lo[s] = max(0, za - (S - 1 - s));
            hi[s] = min(n, zb + (S - 1 - s));
        }
        const int ld_lo = max(0, za - S), ld_hi = min(n, zb + S);  // planes of the loaded direction
        const int m0 = lo[0];
        int m_end = m0;
#pragma unroll
        for (int s = 0; s < S; ++s) m_end = max(m_end, hi[s] + s);
        const int rx0 = tl.tx * kF3X - S, ry0 = tl.ty * kF3Y - S;  // region origin
        unsigned fl[PER];
        int64_t cxy[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = (int)threadIdx.x + NT * k;
            const int lx = i % RW, ly = i / RW;
            const int x = rx0 + lx, y = ry0 + ly;
            unsigned f = 0;
            if (i < RC && x >= 0 && x < n && y >= 0 && y < n) {
                const int dx = lx < S ? S - lx : (lx >= S + kF3X ? lx - (S + kF3X - 1) : 0);
                const int dy = ly < S ? S - ly : (ly >= S + kF3Y ? ly - (S + kF3Y - 1) : 0);
                const int d = max(dx, dy);
                f = fAct | ((unsigned)d << 8);
                if (d == 0) f |= fOwn;
                if (x + 1 < n && lx + 1 < RW) f |= fE;
                if (x > 0 && lx > 0) f |= fW;
                if (y + 1 < n && ly + 1 < RH) f |= fN;
                if (y > 0 && ly > 0) f |= fS;
            }
            fl[k] = f;
            cxy[k] = I.org + x + (int64_t)y * sy;
        }
        // the cells step 0 computes (every later step computes a subset)
        auto stepped = [&](int k) { return (fl[k] & fAct) && (int)(fl[k] >> 8) <= S - 1; };
        // planes m0 - 1 and m0 of the direction to LDS; plane m0 + 1 of the
        // direction, and rt and z of plane m0, to the prefetch registers
        T sd_nx[PER], rt_nx[PER], z_nx[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            sd_nx[k] = rt_nx[k] = z_nx[k] = (T)0;
            if (!(fl[k] & fAct)) continue;
            const int i = (int)threadIdx.x + NT * k;
            for (int q = m0 - 1; q <= m0; ++q)
                if (q >= ld_lo && q < ld_hi) ring[0][q % 3][i] = sdi[cxy[k] + q * sz];
            if (m0 + 1 < ld_hi) sd_nx[k] = sdi[cxy[k] + (m0 + 1) * sz];
            if (m0 < hi[0]) rt_nx[k] = rt_in[cxy[k] + m0 * sz];
            if ((fl[k] & fOwn) && m0 >= za && m0 < zb) z_nx[k] = zp[cxy[k] + m0 * sz];
        }
        T rt[S][PER], z[S][PER], cf[RING ? S : 1][6][RING ? PER : 1];
        for (int mb = m0; mb < m_end; mb += S) {
#pragma unroll
            for (int u = 0; u < S; ++u) {
                const int m = mb + u;
                if (m >= m_end) break;
                // plane m + 1 of the direction to LDS, rt and z of plane m to
                // their ring slot, the face coefficients of plane m loaded
                // into theirs; then the loads of the next march
                const bool sd_ok = m + 1 < ld_hi, cf_ok = m < hi[0];
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    if (!(fl[k] & fAct)) continue;
                    const int i = (int)threadIdx.x + NT * k;
                    if (sd_ok) ring[0][(m + 1) % 3][i] = sd_nx[k];
                    rt[u][k] = rt_nx[k];
                    z[u][k] = z_nx[k];
                    if (RING && cf_ok && stepped(k)) {
                        const int64_t c = cxy[k] + m * sz;
                        cf[u][0][k] = kx[c + 1];
                        cf[u][1][k] = kx[c];
                        cf[u][2][k] = ky[c + sy];
                        cf[u][3][k] = ky[c];
                        cf[u][4][k] = kz[c + sz];
                        cf[u][5][k] = kz[c];
                    }
                    if (m + 2 < ld_hi) sd_nx[k] = sdi[cxy[k] + (m + 2) * sz];
                    if (m + 1 < hi[0]) rt_nx[k] = rt_in[cxy[k] + (m + 1) * sz];
                    if ((fl[k] & fOwn) && m + 1 >= za && m + 1 < zb) z_nx[k] = zp[cxy[k] + (m + 1) * sz];
                }
                __syncthreads();
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const int p = m - s;
                    if (p < lo[s] || p >= hi[s]) continue;  // the same for the whole workgroup
                    const int r = (u - s + S) % S;  // ring slot of plane p
                    const T al = (T)I.al[j0 + s - 1], be = (T)I.be[j0 + s - 1];
                    const T *vc_p = ring[s][p % 3];
                    const T *vt_p = ring[s][(p + 1 < n ? p + 1 : p) % 3];
                    const T *vb_p = ring[s][(p > 0 ? p - 1 : p) % 3];
                    const bool own_plane = p >= za && p < zb;
#pragma unroll
                    for (int k = 0; k < PER; ++k) {
                        const unsigned f = fl[k];
                        if (!(f & fAct) || (int)(f >> 8) > S - 1 - s) continue;
                        const int i = (int)threadIdx.x + NT * k;
                        const int64_t c = cxy[k] + p * sz;
                        const T ke = RING ? cf[r][0][k] : kx[c + 1], kw = RING ? cf[r][1][k] : kx[c];
                        const T kn = RING ? cf[r][2][k] : ky[c + sy], ks = RING ? cf[r][3][k] : ky[c];
                        T diag = (T)1 + ke;
                        diag = diag + kw;
                        diag = diag + kn;
                        diag = diag + ks;
                        const T kt = RING ? cf[r][4][k] : kz[c + sz], kb = RING ? cf[r][5][k] : kz[c];
                        diag = diag + kt;
                        diag = diag + kb;
                        const T vc = vc_p[i];
                        T av = diag * vc;
                        av = fmaB<T>(-ke, vc_p[(f & fE) ? i + 1 : i], av);
                        av = fmaB<T>(-kw, vc_p[(f & fW) ? i - 1 : i], av);
                        av = fmaB<T>(-kn, vc_p[(f & fN) ? i + RW : i], av);
                        av = fmaB<T>(-ks, vc_p[(f & fS) ? i - RW : i], av);
                        av = fmaB<T>(-kt, vt_p[i], av);
                        av = fmaB<T>(-kb, vb_p[i], av);
                        const T rtv = rt[r][k] - av;
                        rt[r][k] = rtv;
                        if ((f & fOwn) && own_plane) z[r][k] = z[r][k] + vc;
                        const T vn = fmaB<T>(al, vc, be * rtv);
                        if (s + 1 < S)
                            ring[s + 1 < S ? s + 1 : 0][p % 3][i] = vn;
                        else if ((f & fOwn) && own_plane)
                            sdo[c] = vn;
                    }
                    // the next step reads what this one wrote; with S == 1 the
                    // next march overwrites a plane this step read
                    if (s + 1 < S || S == 1) __syncthreads();
                }
                // rt and z of plane m - S + 1 are final
                const int pf = m - (S - 1);
                if (pf >= za && pf < zb) {
                    const int r = (u + 1) % S;
#pragma unroll
                    for (int k = 0; k < PER; ++k) {
                        if (!(fl[k] & fOwn)) continue;
                        rt_out[cxy[k] + pf * sz] = rt[r][k];
                        zp[cxy[k] + pf * sz] = z[r][k];
                    }
                }
            }
        }
        __syncthreads();  // the next tile reuses the LDS rings
    }
}

// ---- per-instance finalize ------------------------------------------------
// Combine slot `slot` of the instance's tile partials in tile order (the
// same order and grouping as the library's finalize kernel); value = hi + lo
// for sums, hi for max.
__device__ double combine(const BInst &I, const double *part, int slot, int op) {
    DD a = red_identity(op);
    for (int64_t i = threadIdx.x; i < I.ntile; i += kRedThreads) {
        DD b;
        b.hi = part[4 * (I.tile0 + i) + 2 * slot];
        b.lo = part[4 * (I.tile0 + i) + 2 * slot + 1];
        a = red_combine(op, a, b);
    }
    a = block_reduce(op, a);
    return op == TC_RED_SUM ? a.hi + a.lo : a.hi;
}

// phase 0: after the set-up kernels (INIT -> RESID)
// phase 1: after the residual (RESID/OUTER/VERIFY)
// phase 2: after the matrix-vector product (INNER: alpha)
// phase 3: after the preconditioner (INNER_START/INNER: beta, convergence)
__global__ void __launch_bounds__(256) bk_finalize(BInst *insts, int ninst, const double *part, int phase) {
    BInst &I = insts[blockIdx.x];
    const int st = I.state;
    if (phase == 0) {
        if (st != B_INIT) return;
        const double bb = combine(I, part, 0, TC_RED_SUM);
        const double lmax = combine(I, part, 1, TC_RED_MAX);
        if (threadIdx.x == 0) {
            I.bnorm = sqrt(bb);
            I.lmax = lmax;
            // Chebyshev scalars for the spectrum [1, lmax]
            const double lmin = 1.0;
            const double theta = (lmax + lmin) / 2.0;
            const double delta = (lmax - lmin) / 2.0;
            const double sigma = theta / delta;
            double r_old = 1.0 / sigma;
            for (int j = 1; j < I.cheb_steps; ++j) {
                const double r_new = 1.0 / (2.0 * sigma - r_old);
                I.al[j - 1] = r_new * r_old;
                I.be[j - 1] = 2.0 * r_new / delta;
                r_old = r_new;
            }
            I.theta = theta;
            I.state = B_RESID;
        }
    } else if (phase == 1) {
        if (st != B_RESID && st != B_OUTER && st != B_VERIFY) return;
        const double rr = combine(I, part, 0, TC_RED_SUM);
        if (threadIdx.x == 0) {
            I.true_rr = rr;
            const double rn = sqrt(rr);
            if (st == B_VERIFY) {
                I.state = B_DONE;
            } else if (!I.mixed) {
                I.state = B_INNER_START;
            } else if (rn <= I.tol * I.bnorm || I.outer >= I.max_outer) {
                I.converged = rn <= I.tol * I.bnorm;
                I.state = B_DONE;
            } else {
                I.r0 = rn;
                I.outer += 1;
                I.state = B_INNER_START;
            }
        }
    } else if (phase == 2) {
        if (st != B_INNER) return;
        const double pw = combine(I, part, 0, TC_RED_SUM);
        if (threadIdx.x == 0) I.alpha = I.rz / pw;
    } else {
        if (st != B_INNER && st != B_INNER_START) return;
        const double rz_new = combine(I, part, 0, TC_RED_SUM);
        const double rr = combine(I, part, 1, TC_RED_SUM);
        if (threadIdx.x == 0) {
            I.rr = rr;
            if (st == B_INNER_START) {
                I.rz = rz_new;
                I.beta = 0.0;
                I.inner_k = 0;
                I.state = B_INNER;
            } else {
                I.iters += 1;
                I.inner_k += 1;
                const bool done = I.mixed ? sqrt(rr) <= I.inner_tol * I.r0 : sqrt(rr) <= I.tol * I.bnorm;
                if (done) {
                    if (I.mixed) {
                        I.state = B_OUTER;
                    } else {
                        I.converged = 1;
                        I.state = B_VERIFY;
                    }
                } else if (I.inner_k >= I.max_iter) {
                    // iteration cap of one solve (mixed: of one correction)
                    I.state = I.mixed ? B_OUTER : B_VERIFY;
                } else {
                    I.beta = rz_new / I.rz;
                    I.rz = rz_new;
                }
            }
        }
    }
}

template <typename T>
hipError_t enqueue_iteration_t(BInst *insts, int ninst, const BTile *tiles, const int64_t *ntiles,
                               const BTile *tiles3, const int64_t *ntiles3, const BTile *ftiles,
                               const int64_t *nftiles, double *part, int grid, int cheb_steps, bool mixed,
                               int fh, int fty, int f3, bool with3d, bool setup, hipStream_t s) {
    const bool fused = fh > 0;
    const dim3 g(grid), b(256), f(ninst);
    // set-up of newly admitted instances (only the first iteration after an
    // admission has any: left out of the other replays)
    if (setup) {
        hipLaunchKernelGGL(bk_init, g, b, 0, s, insts, tiles, ntiles, part);
        hipLaunchKernelGGL(bk_faces<T>, g, b, 0, s, insts, tiles, ntiles);
        hipLaunchKernelGGL(bk_gersh, g, b, 0, s, insts, tiles, ntiles, part);
        hipLaunchKernelGGL(bk_finalize, f, b, 0, s, insts, ninst, part, 0);
    }
    // refinement step (mixed) / first and verifying residuals
    if (mixed) hipLaunchKernelGGL(bk_apply_correction<T>, g, b, 0, s, insts, tiles, ntiles);
    hipLaunchKernelGGL(bk_resid<T>, g, b, 0, s, insts, tiles, ntiles, part);
    hipLaunchKernelGGL(bk_finalize, f, b, 0, s, insts, ninst, part, 1);
    // one PPCG iteration
    hipLaunchKernelGGL(bk_cg_p<T>, g, b, 0, s, insts, tiles, ntiles);
    hipLaunchKernelGGL(bk_matvec<T>, g, b, 0, s, insts, tiles, ntiles, part);
    hipLaunchKernelGGL(bk_finalize, f, b, 0, s, insts, ninst, part, 2);
    // with fused Chebyshev launches the first one starts 2D instances from r
    const int skip2d = fused && cheb_steps > 1 ? 1 : 0;
    hipLaunchKernelGGL(bk_update_init<T>, g, b, 0, s, insts, tiles, ntiles, skip2d);
    if (fused) {
        // 2D instances: steps 1 .. cheb_steps-1 in launches of at most fh
        // steps (an odd number each), on the fused tiles; 3D instances: in
        // launches of three steps (or one) marching their z-segments (f3), or
        // one launch per step on their own tiles; then everybody's last step
        // (with the r.z and r.r partials)
        int launches = 0;
        for (int j0 = 1; j0 < cheb_steps;) {
            int len = cheb_steps - j0 < fh ? cheb_steps - j0 : fh;
            len -= (len & 1) ^ 1;  // odd, so the direction lands in the other buffer
            const int j1 = j0 + len;
            const int alt = launches & 1, first = launches == 0 ? 1 : 0;
            if (fh == 3 && fty == 16)
                hipLaunchKernelGGL((bk_cheb_fused<T, 3, 16>), g, b, 0, s, insts, ftiles, nftiles, j0, j1, alt, first);
            else if (fh == 3 && fty == 32)
                hipLaunchKernelGGL((bk_cheb_fused<T, 3, 32>), g, b, 0, s, insts, ftiles, nftiles, j0, j1, alt, first);
            else if (fh == 5 && fty == 16)
                hipLaunchKernelGGL((bk_cheb_fused<T, 5, 16>), g, b, 0, s, insts, ftiles, nftiles, j0, j1, alt, first);
            else if (fh == 5 && fty == 32)
                hipLaunchKernelGGL((bk_cheb_fused<T, 5, 32>), g, b, 0, s, insts, ftiles, nftiles, j0, j1, alt, first);
            else
                hipLaunchKernelGGL((bk_cheb_fused<T, 9, 16>), g, b, 0, s, insts, ftiles, nftiles, j0, j1, alt, first);
            ++launches;
            j0 = j1;
        }
        if (with3d && f3 > 0) {
            int l3 = 0;
            for (int j0 = 1; j0 < cheb_steps; ++l3) {
                int len = cheb_steps - j0 < 3 ? cheb_steps - j0 : 3;
                len -= (len & 1) ^ 1;
                if (len == 3)
                    hipLaunchKernelGGL((bk_cheb3_fused<T, 3>), g, dim3(f3_threads<T>()), 0, s, insts, tiles3, ntiles3,
                                       j0, l3 & 1);
                else
                    hipLaunchKernelGGL((bk_cheb3_fused<T, 1>), g, dim3(f3_threads<T>()), 0, s, insts, tiles3, ntiles3,
                                       j0, l3 & 1);
                j0 += len;
            }
        } else if (with3d) {
            for (int j = 1; j < cheb_steps; ++j)
                hipLaunchKernelGGL(bk_cheb<T>, g, b, 0, s, insts, tiles3, ntiles3, part, j);
        }
        hipLaunchKernelGGL(bk_cheb<T>, g, b, 0, s, insts, tiles, ntiles, part, cheb_steps);
    } else {
        for (int j = 1; j <= cheb_steps; ++j)
            hipLaunchKernelGGL(bk_cheb<T>, g, b, 0, s, insts, tiles, ntiles, part, j);
    }
    hipLaunchKernelGGL(bk_finalize, f, b, 0, s, insts, ninst, part, 3);
    return hipGetLastError();
}

}  // namespace

// One round of every solver phase for every resident instance, in order
// (set-up, residual, one PPCG iteration); each instance advances according
// to its own state.
hipError_t batch_enqueue_iteration(BInst *insts, int ninst, const BTileList &all, const BTileList &three,
                                   const BTileList &fused, double *part, int grid, int cheb_steps, bool mixed, int fh,
                                   int fty, int f3, bool with3d, bool setup, hipStream_t s) {
    return mixed ? enqueue_iteration_t<float>(insts, ninst, all.d, all.dn, three.d, three.dn, fused.d, fused.dn, part,
                                              grid, cheb_steps, true, fh, fty, f3, with3d, setup, s)
                 : enqueue_iteration_t<double>(insts, ninst, all.d, all.dn, three.d, three.dn, fused.d, fused.dn, part,
                                               grid, cheb_steps, false, fh, fty, f3, with3d, setup, s);
}

}  // namespace tc
