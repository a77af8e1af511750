// Fusion groups: analysis, split, kernel generation, hipRTC compilation and
// launch (the scheme is described in fused.hpp).
#include "fused.hpp"
#include "kernels.hpp"

#include <hip/hiprtc.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <sstream>
#include <stdexcept>
#include <tuple>
#include <unordered_map>

namespace tc {

namespace {

int esize_of(int dtype) { return dtype == TC_F64 ? 8 : 4; }

struct SplitParams {
    int hseg = 0;      // rows per wavefront segment (0: automatic)
    int regs = 160;    // budget of window registers per lane
    int max_loops = 32;
    int U = 3, PF = 1;
    bool bake = false;
    int cpl = 1;       // columns per lane
    int wpe = 2;       // wavefronts per SIMD requested for the interior kernels (0: compiler's choice)
    int max_window = 0; // longest register window of a loaded version before its readers split (0: never)
    bool cse_steps = true;  // share shifted values between the loops of a step
    bool sched_fence = false;  // keep the instruction scheduler from mixing the loops of a step
    bool align_store = false;  // owned strip width a multiple of 16 columns
    int edge_div = 4;  // edge wavefronts march Hseg / edge_div rows (1: as many as interior ones)
};

// ---------------------------------------------------------------------------
// analysis of one candidate group: versions, liveness, extents (Section 4.4:
// each loop computes what its later readers need beyond the owned block),
// lags, register windows and the wavefront layout.  False if the loops
// cannot form a group.
// ---------------------------------------------------------------------------
bool analyse(const Ctx &c, const std::vector<LoopRec> &chain, int g0, int g1, const SplitParams &sp,
             FusedGroup &G) {
    G = FusedGroup();
    G.g0 = g0;
    G.g1 = g1;
    G.U = sp.U;
    G.PF = sp.PF;
    G.baked = sp.bake;
    G.cpl = sp.cpl;
    G.wpe = sp.wpe;
    G.cse_steps = sp.cse_steps;
    G.sched_fence = sp.sched_fence;
    const LoopRec &f = chain[g0];
    if (f.op != TC_OP_WSUM || f.ndim != 2 || f.points() == 0) return false;
    G.xlo = f.lo[0];
    G.xhi = f.hi[0];
    G.ylo = f.lo[1];
    G.yhi = f.hi[1];
    G.dtype = c.dats[f.args[0].handle].dtype;
    std::unordered_map<int, int> cur;    // dataset -> current version
    std::unordered_map<int, int> first;  // dataset -> chain-start version
    auto start_version = [&](int d) {
        JVer v;
        v.dat = d;
        G.vers.push_back(v);
        const int id = (int)G.vers.size() - 1;
        cur[d] = id;
        first[d] = id;
        return id;
    };
    int wcount = 0;
    for (int l = g0; l < g1; ++l) {
        const LoopRec &lp = chain[l];
        if (lp.op != TC_OP_WSUM || lp.ndim != 2) return false;
        if (lp.lo[0] != G.xlo || lp.hi[0] != G.xhi || lp.lo[1] != G.ylo || lp.hi[1] != G.yhi) return false;
        if (lp.args.size() < 2) return false;
        JLoop J;
        J.loop = l;
        for (size_t a = 1; a < lp.args.size(); ++a) {
            const ArgRec &A = lp.args[a];
            if (c.dats[A.handle].dtype != G.dtype) return false;
            const Stencil &st = c.stencils[A.stencil];
            JRead R;
            R.ver = cur.count(A.handle) ? cur[A.handle] : start_version(A.handle);
            R.dxmin = R.dymin = INT_MAX;
            R.dxmax = R.dymax = INT_MIN;
            for (int k = 0; k < st.npoints(); ++k) {
                const int dx = st.pts[3 * k], dy = st.pts[3 * k + 1];
                if (std::abs(dx) > kJMaxOff || std::abs(dy) > kJMaxOff) return false;
                R.pts.push_back({dx, dy, wcount++});
                R.dxmin = std::min(R.dxmin, dx);
                R.dxmax = std::max(R.dxmax, dx);
                R.dymin = std::min(R.dymin, dy);
                R.dymax = std::max(R.dymax, dy);
            }
            if (R.pts.empty()) return false;
            J.in.push_back(R);
        }
        const int o = lp.args[0].handle;
        if (c.dats[o].dtype != G.dtype) return false;
        if (!cur.count(o)) start_version(o);
        JVer v;
        v.dat = o;
        v.producer = (int)G.loops.size();
        G.vers.push_back(v);
        J.out = (int)G.vers.size() - 1;
        cur[o] = J.out;
        G.loops.push_back(J);
    }
    if (wcount > kJMaxW) return false;
    G.nweights = wcount;
    for (int l = g0; l < g1; ++l) G.wvals.insert(G.wvals.end(), chain[l].params.begin(), chain[l].params.end());
    for (auto &kv : cur)
        if (G.vers[kv.second].producer >= 0) G.vers[kv.second].stored = true;

    // backward: which loops matter and the columns / rows each computes
    // beyond the owned block
    for (auto &v : G.vers)
        if (v.stored) {
            v.needed = true;
            v.extL = v.extR = v.extB = v.extT = 0;
        }
    for (int j = (int)G.loops.size() - 1; j >= 0; --j) {
        JLoop &J = G.loops[j];
        const JVer &o = G.vers[J.out];
        if (!o.needed) continue;
        J.needed = true;
        J.extL = o.extL;
        J.extR = o.extR;
        J.extB = o.extB;
        J.extT = o.extT;
        for (auto &R : J.in) {
            JVer &v = G.vers[R.ver];
            v.needed = true;
            v.extL = std::max(v.extL, std::max(0, J.extL - R.dxmin));
            v.extR = std::max(v.extR, std::max(0, J.extR + R.dxmax));
            v.extB = std::max(v.extB, std::max(0, J.extB - R.dymin));
            v.extT = std::max(v.extT, std::max(0, J.extT + R.dymax));
            for (const auto &p : R.pts)
                if ((p.dx != 0 || p.dy != 0) && v.producer >= 0) v.sel = true;
        }
    }
    int nneeded = 0;
    for (auto &J : G.loops) nneeded += J.needed;
    if (nneeded == 0) return false;

    // forward: lags (a reader runs at least its largest y offset behind the
    // producer of every version it reads)
    for (auto &J : G.loops) {
        if (!J.needed) continue;
        int lag = 0;
        for (const auto &R : J.in) {
            const JVer &v = G.vers[R.ver];
            if (v.producer >= 0) lag = std::max(lag, G.loops[v.producer].lag + R.dymax);
        }
        J.lag = lag;
        G.vers[J.out].lag = lag;
    }

    // load streams: a chain-start version read by loops far apart in lag
    // would need a long register window; its readers are split into groups
    // of nearby lags, each with a window (and loads) of its own -- the extra
    // loads of the same rows are cheaper than the registers
    if (sp.max_window > 0) {
        const size_t nv0 = G.vers.size();
        for (size_t v = 0; v < nv0; ++v) {
            if (G.vers[v].producer >= 0 || !G.vers[v].needed) continue;
            std::vector<std::pair<int, JRead *>> rd;
            for (auto &J : G.loops)
                if (J.needed)
                    for (auto &R : J.in)
                        if (R.ver == (int)v) rd.push_back({J.lag, &R});
            std::sort(rd.begin(), rd.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
            int lo = INT_MAX, hi = INT_MIN, cur = (int)v;
            for (auto &e : rd) {
                const int l2 = std::min(lo, e.first - e.second->dymax), h2 = std::max(hi, e.first - e.second->dymin);
                if (lo != INT_MAX && h2 - l2 + 1 > sp.max_window) {
                    JVer nv = G.vers[v];
                    G.vers.push_back(nv);
                    cur = (int)G.vers.size() - 1;
                    lo = e.first - e.second->dymax;
                    hi = e.first - e.second->dymin;
                } else {
                    lo = l2;
                    hi = h2;
                }
                e.second->ver = cur;
            }
        }
    }

    // lanes: columns loaded left / right of the owned ones; computed extents
    int HL = 0, HR = 0, CL = 0, CR = 0, CB = 0, CT = 0;
    for (const auto &v : G.vers)
        if (v.needed && v.producer < 0) {
            HL = std::max(HL, v.extL);
            HR = std::max(HR, v.extR);
        }
    for (const auto &J : G.loops)
        if (J.needed) {
            CL = std::max(CL, J.extL);
            CR = std::max(CR, J.extR);
            CB = std::max(CB, J.extB);
            CT = std::max(CT, J.extT);
        }
    const int wcols = kJLanes * G.cpl;
    if (G.cpl == 2) {
        // two-column loads stay 16-byte aligned: the first lane column
        // X0 - HL and the strip width are even (the x origin is 16-aligned)
        if (G.xlo % 2 != 0) return false;
        HL += HL & 1;
    }
    G.HL = HL;
    G.HR = HR;
    G.Wo = wcols - HL - HR;
    if (G.cpl == 2) G.Wo -= G.Wo & 1;
    // whole 128-byte lines per stored row: owned strips start and end on
    // multiples of 16 columns (the x origin of every dataset is 16-aligned)
    if (sp.align_store && G.xlo % 16 == 0) G.Wo -= G.Wo % 16;
    if (G.Wo < 8) return false;
    G.BMAX = CB;
    G.TMAX = CT;

    // variants: 0 interior, 1 edge (keeps chain-start values outside the range)
    const int words = esize_of(G.dtype) / 4;
    for (int var = 0; var < 2; ++var) {
        JVariant &V = G.var[var];
        const size_t nv = G.vers.size();
        V.PF = sp.PF;
        V.win.assign(nv, 0);
        V.load_lag.assign(nv, 0);
        V.loaded.assign(nv, 0);
        V.pseudo.clear();
        // per version: smallest (lag - dymax) over its readers bounds the
        // arrival step of a row; largest (lag - dymin) the oldest row kept
        std::vector<int> lo(nv, INT_MAX), hi(nv, INT_MIN), eb(nv, -1), et(nv, -1);
        for (const auto &J : G.loops) {
            if (!J.needed) continue;
            for (const auto &R : J.in) {
                lo[R.ver] = std::min(lo[R.ver], J.lag - R.dymax);
                hi[R.ver] = std::max(hi[R.ver], J.lag - R.dymin);
            }
        }
        if (var == 1) {
            for (size_t j = 0; j < G.loops.size(); ++j) {
                const JLoop &J = G.loops[j];
                if (!J.needed || !G.vers[J.out].sel) continue;
                const int c0 = first.at(G.vers[J.out].dat);
                V.pseudo.push_back({(int)j, c0});
                lo[c0] = std::min(lo[c0], J.lag);
                hi[c0] = std::max(hi[c0], J.lag);
                eb[c0] = std::max(eb[c0], J.extB);
                et[c0] = std::max(et[c0], J.extT);
            }
        }
        int pre = 0, post = 0, regs = 0;
        for (size_t v = 0; v < nv; ++v) {
            const JVer &X = G.vers[v];
            if (X.producer >= 0) {
                if (!X.needed) continue;
                const int oldest = hi[v] == INT_MIN ? X.lag : std::max(hi[v], X.lag);
                V.win[v] = oldest - X.lag + 1;
                regs += V.win[v] * words * G.cpl;
                if (X.stored) post = std::max(post, X.lag);
            } else {
                if (lo[v] == INT_MAX) continue;  // not read in this variant
                V.loaded[v] = 1;
                V.load_lag[v] = lo[v];
                V.win[v] = hi[v] - lo[v] + 1;
                regs += (V.win[v] + V.PF) * words * G.cpl;
                const int b = std::max(X.needed ? X.extB : -1, eb[v]);
                const int t = std::max(X.needed ? X.extT : -1, et[v]);
                pre = std::max(pre, b - lo[v]);
                post = std::max(post, t + lo[v]);
            }
        }
        for (const auto &J : G.loops) {
            if (!J.needed) continue;
            pre = std::max(pre, J.extB - J.lag);
            post = std::max(post, J.extT + J.lag);
        }
        V.pre = pre;
        V.post = post + 1;
        V.regs = regs;
    }
    // The budget bounds the interior variant, which runs on almost every
    // strip.  The edge variant holds extra windows for chain-start versions
    // and may exceed it (it runs on the two edge strips of a row of tiles,
    // where a spill costs little); group length is not cut for it.
    if (G.var[0].regs > sp.regs) return false;
    // datasets loaded / stored, in kernel argument order
    for (size_t v = 0; v < G.vers.size(); ++v)
        if (G.vers[v].producer < 0 && (G.var[0].loaded[v] || G.var[1].loaded[v]) &&
            std::find(G.src_dat.begin(), G.src_dat.end(), G.vers[v].dat) == G.src_dat.end())
            G.src_dat.push_back(G.vers[v].dat);
    for (size_t v = 0; v < G.vers.size(); ++v)
        if (G.vers[v].stored) {
            G.dst_dat.push_back(G.vers[v].dat);
            G.dst_twin.push_back(G.vers[first.at(G.vers[v].dat)].needed ? 1 : 0);
        }
    if ((int)G.src_dat.size() > kJMaxSrc || (int)G.dst_dat.size() > kJMaxDst) return false;

    // wavefront layout: strips of Wo columns by segments of Hseg rows
    const int width = G.xhi - G.xlo, height = G.yhi - G.ylo;
    G.nstrips = (width + G.Wo - 1) / G.Wo;
    int Hseg = sp.hseg;
    const int ediv = std::max(1, sp.edge_div);
    if (Hseg <= 0) {
        const int target = 4096;  // wavefronts: 16 per compute unit
        const int nsegs = std::max(1, (int)std::lround((double)target / G.nstrips));
        Hseg = std::max(48, (height + nsegs - 1) / nsegs);
        Hseg = (Hseg + ediv - 1) / ediv * ediv;
    }
    G.Hseg = std::min(Hseg, height);
    G.nsegs = (height + G.Hseg - 1) / G.Hseg;
    // edge wavefronts are few and run at low occupancy: give them shorter
    // segments
    G.Hedge = std::max(8, G.Hseg / ediv);
    // Interior waves run without bounds logic.  Strip origin X0 = xlo + rx
    // computes columns [X0 - CL, X0 + Wo + CR) and segment origin Y0 = ylo + ry
    // rows [Y0 - CB, Y0 + Hseg + CT): both inside the range.  Every lane
    // column and every row they load must lie inside the allocation.  That
    // bounds rx to [LX, UX] and ry to [LY, UY]; the interior grid starts at a
    // feasible origin and the frame around it goes to edge waves.
    int LX = CL, UX = width - CR - G.Wo, LY = CB, UY = height - CT - G.Hseg;
    {
        const JVariant &V = G.var[0];
        const int nsteps = (G.Hseg + V.pre + V.post + G.U - 1) / G.U * G.U;
        for (size_t v = 0; v < G.vers.size(); ++v) {
            if (!V.loaded[v]) continue;
            const Dataset &ds = c.dats[G.vers[v].dat];
            // columns X0 - HL + [0, wcols)
            LX = std::max(LX, -ds.hneg[0] - G.xlo + HL);
            UX = std::min(UX, ds.size[0] + ds.hpos[0] - wcols - G.xlo + HL);
            // rows Y0 - pre - lag .. Y0 - pre + nsteps - 1 + PF - lag
            LY = std::max(LY, -ds.hneg[1] - G.ylo + V.pre + V.load_lag[v]);
            UY = std::min(UY, ds.size[1] + ds.hpos[1] - 1 - G.ylo + V.pre - nsteps + 1 - V.PF + V.load_lag[v]);
        }
    }
    // owned strips stay on 128-byte lines when the strip width is a multiple of 16
    if (sp.align_store && G.xlo % 16 == 0 && G.Wo % 16 == 0) LX = (LX + 15) / 16 * 16;
    G.in_ns = UX >= LX ? (UX - LX) / G.Wo + 1 : 0;
    G.in_ng = UY >= LY ? (UY - LY) / G.Hseg + 1 : 0;
    if (G.in_ns == 0 || G.in_ng == 0) G.in_ns = G.in_ng = 0;
    if (G.in_ns > 0) {
        // centre the grid in its slack (whole 16-column steps when aligned)
        const int sx = UX - LX - (G.in_ns - 1) * G.Wo, sy = UY - LY - (G.in_ng - 1) * G.Hseg;
        const int step = sp.align_store && G.xlo % 16 == 0 && G.Wo % 16 == 0 ? 16 : 1;
        G.in_x = LX + sx / 2 / step * step;
        G.in_y = LY + sy / 2;
        G.e_yb = G.in_y;
        G.e_yt = G.in_y + G.in_ng * G.Hseg;
        G.e_xr = G.in_x + G.in_ns * G.Wo;
    } else {
        G.in_x = G.in_y = 0;
        G.e_yb = height;  // everything is the bottom band
        G.e_yt = height;
        G.e_xr = width;
    }
    G.nwaves_in = G.in_ns * G.in_ng;
    {
        auto cd = [](int a, int b) { return a <= 0 ? 0 : (a + b - 1) / b; };
        G.e_ns = cd(width, G.Wo);
        G.e_ngb = cd(G.e_yb, G.Hedge);
        G.e_ngt = cd(height - G.e_yt, G.Hedge);
        const bool mid = G.nwaves_in > 0;
        G.e_nsl = mid ? cd(G.in_x, G.Wo) : 0;
        G.e_nsr = mid ? cd(width - G.e_xr, G.Wo) : 0;
        G.e_ngm = mid ? cd(G.e_yt - G.in_y, G.Hedge) : 0;
        G.nwaves_edge = G.e_ns * (G.e_ngb + G.e_ngt) + (G.e_nsl + G.e_nsr) * G.e_ngm;
    }
    G.nblocks = (G.nwaves_in + 3) / 4 + (G.nwaves_edge + 3) / 4;

    // modelled time (split choice): HBM bytes of the loads and stores
    // against VALU work, both scaled by the recomputed lanes and rows
    const double cells = (double)width * height;
    const double fy = (double)(G.Hseg + G.var[0].pre + G.var[0].post) / G.Hseg;
    const double fx = (double)wcols / G.Wo;
    int nload = 0;
    for (size_t v = 0; v < G.vers.size(); ++v) nload += G.var[0].loaded[v];
    double ops = 0.0;
    for (const auto &J : G.loops) {
        if (!J.needed) continue;
        for (const auto &R : J.in)
            for (const auto &p : R.pts) ops += 1.0 + (p.dx != 0 ? (double)words / G.cpl : 0.0);
        ops += 2.0;
    }
    G.alg_bytes = (int64_t)width * height * esize_of(G.dtype) * (int64_t)(nload + (int)G.dst_dat.size());
    const double bytes =
        cells * esize_of(G.dtype) * (nload * (1.0 + 0.5 * (HL + HR) / G.Wo) + (double)G.dst_dat.size()) * fy;
    const double valu = cells * fx * fy * ops / (256.0 * 64.0 * 2.4e9);
    G.cost = std::max(bytes / 5.0e12, valu) + 4e-6;
    return true;
}

// Modelled time of one loop run on its own: its bytes at the HBM rate, or
// at the Infinity Cache's when its datasets together fit well inside the
// 256 MB cache (consecutive loops then mostly hit it), and at least a
// launch.  Measured per-loop PPCG kernels: 3-4 us at 256^2 and 700^2, a
// matrix-vector step over 2000^2 (224 MB moved, 160 MB of datasets) 32 us.
// The streaming part alone: its bytes at that rate.
double loop_stream_time(const Ctx &c, const LoopRec &lp) {
    double b = 0.0, footprint = 0.0;
    for (const auto &a : lp.args)
        if (a.kind == TC_ARG_DAT) {
            b += (a.access == TC_RW || a.access == TC_INC ? 2.0 : 1.0) * c.dats[a.handle].esize();
            footprint += (double)c.dats[a.handle].bytes;
        }
    const double bw = footprint < 192e6 ? 7.0e12 : 4.2e12;
    return (double)lp.points() * b / bw;
}

double single_loop_cost(const Ctx &c, const LoopRec &lp) { return std::max(3e-6, loop_stream_time(c, lp)) + 1e-6; }

// ---------------------------------------------------------------------------
// code generation
// ---------------------------------------------------------------------------
// Cross-lane moves: wave_shr:1 gives every lane the value of the lane below
// it (column x-1), wave_shl:1 the value of the lane above (column x+1).
const char *kPrelude = R"(
typedef long long i64;
typedef const double __attribute__((address_space(4))) *tcj_cw;
typedef const double __attribute__((address_space(1))) *tcj_gcd;
typedef double __attribute__((address_space(1))) *tcj_gd;
typedef const float __attribute__((address_space(1))) *tcj_gcf;
typedef float __attribute__((address_space(1))) *tcj_gf;
typedef double tcj_d2 __attribute__((ext_vector_type(2)));
typedef float tcj_f2 __attribute__((ext_vector_type(2)));
typedef const tcj_d2 __attribute__((address_space(1))) *tcj_gcd2;
typedef const tcj_f2 __attribute__((address_space(1))) *tcj_gcf2;
__device__ __forceinline__ double tcj_shr(double v) {
    const i64 u = __builtin_bit_cast(i64, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)u, 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0x138, 0xf, 0xf, true);
    return __builtin_bit_cast(double, (i64)(unsigned)lo | ((i64)hi << 32));
}
__device__ __forceinline__ double tcj_shl(double v) {
    const i64 u = __builtin_bit_cast(i64, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)u, 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(double, (i64)(unsigned)lo | ((i64)hi << 32));
}
__device__ __forceinline__ float tcj_shr(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float tcj_shl(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double tcj_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float tcj_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ int tcj_lin(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}
)";

// Lane layout: lane l holds columns X0 - HL + cpl*l + e, e < cpl, of every
// row it keeps; window w<v>_<e>[k] is element e of version v's row at slot k.
struct Gen {
    const Ctx &c;
    const FusedGroup &G;
    int var;
    const JVariant &V;
    int cpl;
    std::ostringstream o;
    const char *T, *GC, *GM, *V2;
    std::vector<int> src_index;  // version -> source argument
    std::vector<int> dst_index;  // version -> destination argument
    std::map<std::tuple<int, int, int, int>, std::string> sh;  // shifted values of the current step
    int ntmp = 0;

    Gen(const Ctx &cc, const FusedGroup &g, int v) : c(cc), G(g), var(v), V(g.var[v]), cpl(g.cpl) {
        T = G.dtype == TC_F64 ? "double" : "float";
        GC = G.dtype == TC_F64 ? "tcj_gcd" : "tcj_gcf";
        GM = G.dtype == TC_F64 ? "tcj_gd" : "tcj_gf";
        V2 = G.dtype == TC_F64 ? "tcj_gcd2" : "tcj_gcf2";
        src_index.assign(G.vers.size(), -1);
        dst_index.assign(G.vers.size(), -1);
        for (size_t k = 0; k < G.vers.size(); ++k) {
            const JVer &X = G.vers[k];
            if (X.producer < 0)
                for (size_t i = 0; i < G.src_dat.size(); ++i)
                    if (G.src_dat[i] == X.dat) src_index[k] = (int)i;
            if (X.stored)
                for (size_t i = 0; i < G.dst_dat.size(); ++i)
                    if (G.dst_dat[i] == X.dat) dst_index[k] = (int)i;
        }
    }

    int lag_of(int v) const { return G.vers[v].producer >= 0 ? G.vers[v].lag : V.load_lag[v]; }

    static std::string W(int v, int e) { return "w" + std::to_string(v) + "_" + std::to_string(e); }

    // slot of version v holding the row that a loop at `lag` reads at offset dy
    int slot(int v, int lag, int dy) const {
        const int m = lag - dy - lag_of(v);
        if (m < 0 || m >= V.win[v]) {
            char msg[160];
            std::snprintf(msg, sizeof msg, "fused group [%d,%d): register window of version %d too short (row %d, window %d)",
                          G.g0, G.g1, v, m, V.win[v]);
            throw std::logic_error(msg);
        }
        return V.win[v] - 1 - m;
    }

    std::string entry(int v, int e, int sl) const { return W(v, e) + "[" + std::to_string(sl) + "]"; }

    // element e of the lane `ls` lanes away (ls < 0: lower lanes) at slot sl
    std::string lane_value(int v, int sl, int e, int ls) {
        if (ls == 0) return entry(v, e, sl);
        const auto key = std::make_tuple(v, sl, e, ls);
        auto it = sh.find(key);
        if (it != sh.end()) return it->second;
        const std::string base = lane_value(v, sl, e, ls < 0 ? ls + 1 : ls - 1);
        const std::string name = "x" + std::to_string(ntmp++);
        o << "      const " << T << " " << name << " = " << (ls < 0 ? "tcj_shr(" : "tcj_shl(") << base << ");\n";
        sh[key] = name;
        return name;
    }

    // value of version v at column offset dx, row offset dy, for element e
    std::string term(int v, int lag, int dy, int dx, int e) {
        const int sl = slot(v, lag, dy);
        const int t = e + dx;
        const int ls = t >= 0 ? t / cpl : -((-t + cpl - 1) / cpl);
        return lane_value(v, sl, t - ls * cpl, ls);
    }

    // One row of a loaded version into a window slot.  Interior kernel: a
    // uniform pointer to the row's first lane column, advanced by one row per
    // step (every row it touches lies inside the allocation); two columns per
    // lane load as one 16-byte access.  Edge kernel: row and column clamped to
    // the allocation (clamped values only feed points that are not needed).
    void load_row(int v, const std::string &step, int sl, const char *indent) {
        const Dataset &ds = c.dats[G.vers[v].dat];
        if (var == 0) {
            if (cpl == 2) {
                o << indent << "{ const auto u = *(" << V2 << ")(q" << v << " + 2 * lane); " << entry(v, 0, sl)
                  << " = u.x; " << entry(v, 1, sl) << " = u.y; }";
            } else {
                o << indent << entry(v, 0, sl) << " = q" << v << "[lane];";
            }
            o << " q" << v << " += " << ds.pitch << "; asm volatile(\"\" : \"+s\"(q" << v << "));\n";
        } else {
            o << indent << "{ const int y = __builtin_amdgcn_readfirstlane(min(max(" << step << " - "
              << V.load_lag[v] << ", " << -ds.hneg[1] << "), " << (ds.size[1] + ds.hpos[1] - 1) << ")); " << GC
              << " r = (" << GC << ")(a.s[" << src_index[v] << "] + (i64)y * " << ds.pitch
              << "); asm volatile(\"\" : \"+s\"(r));";
            for (int e = 0; e < cpl; ++e)
                o << " " << entry(v, e, sl) << " = r[cx" << src_index[v] << "_" << e << "];";
            o << " }\n";
        }
    }

    void step(const std::string &tt) {
        sh.clear();
        o << "    {\n      const int tt = " << tt << ";\n";
        // rows arriving PF steps ahead
        for (size_t v = 0; v < G.vers.size(); ++v)
            if (V.loaded[v]) load_row((int)v, "(tt + " + std::to_string(V.PF) + ")", V.win[v] + V.PF - 1, "      ");
        // loops in chain order
        for (size_t j = 0; j < G.loops.size(); ++j) {
            const JLoop &J = G.loops[j];
            if (!J.needed) continue;
            if (!G.cse_steps) sh.clear();  // shifted values are shared within one loop only
            if (G.sched_fence) o << "      __builtin_amdgcn_sched_barrier(0);\n";
            std::vector<std::string> terms[2];
            for (int e = 0; e < cpl; ++e)
                for (const auto &R : J.in)
                    for (const auto &p : R.pts) terms[e].push_back(term(R.ver, J.lag, p.dy, p.dx, e));
            o << "      {\n";
            for (int e = 0; e < cpl; ++e) o << "      " << T << " acc" << e << " = (" << T << ")0;\n";
            size_t q = 0;
            for (const auto &R : J.in) {
                if (G.baked) {
                    for (const auto &p : R.pts) {
                        char lit[64];
                        std::snprintf(lit, sizeof lit, "%a", G.wvals[p.w]);
                        for (int e = 0; e < cpl; ++e)
                            o << "      acc" << e << " = tcj_fma((" << T << ")" << lit << ", " << terms[e][q]
                              << ", acc" << e << ");\n";
                        ++q;
                    }
                    continue;
                }
                // weights read from the kernel arguments right before use
                // (the empty asm hides the pointer's origin, so they are not
                // all kept live in scalar registers)
                o << "      { tcj_cw wl = wk; asm volatile(\"\" : \"+s\"(wl));\n";
                for (const auto &p : R.pts) {
                    for (int e = 0; e < cpl; ++e)
                        o << "      acc" << e << " = tcj_fma((" << T << ")wl[" << p.w << "], " << terms[e][q] << ", acc"
                          << e << ");\n";
                    ++q;
                }
                o << "      }\n";
            }
            const int out = J.out;
            if (var == 1 && G.vers[out].sel) {
                int c0 = -1;
                for (const auto &ps : V.pseudo)
                    if (ps.first == (int)j) c0 = ps.second;
                const int sl = slot(c0, J.lag, 0);
                o << "      { const int y = tt - " << J.lag << "; const bool iny = (unsigned)(y - (" << G.ylo << ")) < "
                  << (unsigned)(G.yhi - G.ylo) << "u;";
                for (int e = 0; e < cpl; ++e)
                    o << " acc" << e << " = (inx" << e << " & iny) ? acc" << e << " : " << entry(c0, e, sl) << ";";
                o << " }\n";
            }
            for (int e = 0; e < cpl; ++e) o << "      " << entry(out, e, V.win[out] - 1) << " = acc" << e << ";\n";
            o << "      }\n";
        }
        // final values of the owned columns (uniform row pointers advanced
        // by one row per step)
        for (size_t v = 0; v < G.vers.size(); ++v) {
            if (!G.vers[v].stored || !G.vers[v].needed) continue;
            const Dataset &ds = c.dats[G.vers[v].dat];
            o << "      { const int y = tt - " << G.vers[v].lag << "; if (y >= Y0 && y < yend) {";
            for (int e = 0; e < cpl; ++e)
                o << " if (own" << e << ") p" << v << "[" << cpl << " * lane + " << e << "] = "
                  << entry((int)v, e, V.win[v] - 1) << ";";
            o << " } p" << v << " += " << ds.pitch << "; asm volatile(\"\" : \"+s\"(p" << v << ")); }\n";
        }
        // advance the windows by one row
        for (size_t v = 0; v < G.vers.size(); ++v) {
            if (!V.win[v]) continue;
            const int n = V.win[v] + (V.loaded[v] ? V.PF : 0);
            for (int e = 0; e < cpl; ++e)
                for (int k = 0; k + 1 < n; ++k) o << "      " << entry((int)v, e, k) << " = " << entry((int)v, e, k + 1) << ";\n";
        }
        o << "    }\n";
    }

    void body() {
        o << "  const tcj_cw wk = (tcj_cw)((const char __attribute__((address_space(4))) *)__builtin_amdgcn_kernarg_segment_ptr() + "
          << 8 * (std::max<size_t>(1, G.src_dat.size()) + std::max<size_t>(1, G.dst_dat.size())) << ");\n";
        o << "  const int lane = threadIdx.x & 63;\n";
        for (int e = 0; e < cpl; ++e) {
            o << "  const int col" << e << " = X0 - " << G.HL << " + " << cpl << " * lane + " << e << ";\n";
            if (var == 0)
                o << "  const bool own" << e << " = (col" << e << " >= X0) & (col" << e << " < X0 + " << G.Wo
                  << ");\n";
            else
                o << "  const bool own" << e << " = (col" << e << " >= X0) & (col" << e << " < XE);\n";
            if (var == 1)
                o << "  const bool inx" << e << " = (col" << e << " >= " << G.xlo << ") & (col" << e << " < " << G.xhi
                  << ");\n";
        }
        const int H = var == 0 ? G.Hseg : G.Hedge;
        if (var == 0)
            o << "  const int yend = Y0 + " << H << ";\n";
        else
            o << "  const int yend = YE;\n";
        const int nsteps = H + V.pre + V.post;
        const int nit = (nsteps + G.U - 1) / G.U;
        o << "  int t = Y0 - " << V.pre << ";\n";
        if (var == 1)
            for (size_t i = 0; i < G.src_dat.size(); ++i) {
                const Dataset &ds = c.dats[G.src_dat[i]];
                for (int e = 0; e < cpl; ++e)
                    o << "  const int cx" << i << "_" << e << " = min(max(col" << e << ", " << -ds.hneg[0] << "), "
                      << (ds.size[0] + ds.hpos[0] - 1) << ");\n";
            }
        for (size_t v = 0; v < G.vers.size(); ++v) {
            const Dataset &ds = c.dats[G.vers[v].dat];
            if (var == 0 && V.loaded[v])
                o << "  " << GC << " q" << v << " = (" << GC << ")(a.s[" << src_index[v] << "] + (i64)(t - "
                  << V.load_lag[v] << ") * " << ds.pitch << " + (X0 - " << G.HL << "));\n";
            if (G.vers[v].stored && G.vers[v].needed)
                o << "  " << GM << " p" << v << " = (" << GM << ")(a.d[" << dst_index[v] << "] + (i64)(t - "
                  << G.vers[v].lag << ") * " << ds.pitch << " + (X0 - " << G.HL << "));\n";
        }
        for (size_t v = 0; v < G.vers.size(); ++v) {
            if (!V.win[v]) continue;
            for (int e = 0; e < cpl; ++e)
                o << "  " << T << " " << W((int)v, e) << "[" << (V.win[v] + (V.loaded[v] ? V.PF : 0)) << "];\n";
        }
        // prologue: rows arriving at the first PF steps
        for (int k = 0; k < V.PF; ++k)
            for (size_t v = 0; v < G.vers.size(); ++v)
                if (V.loaded[v]) load_row((int)v, "(t + " + std::to_string(k) + ")", V.win[v] - 1 + k, "  ");
        o << "  for (int it = 0; it < " << nit << "; ++it, t += " << G.U << ") {\n";
        for (int u = 0; u < G.U; ++u) step("t + " + std::to_string(u));
        o << "  }\n";
    }
};

void gen_group(const Ctx &c, FusedGroup &G, int gi, std::ostringstream &o) {
    const char *T = G.dtype == TC_F64 ? "double" : "float";
    const std::string S = "tcj_args" + std::to_string(gi);
    o << "struct " << S << " { const " << T << "* s[" << std::max<size_t>(1, G.src_dat.size()) << "]; " << T
      << "* d[" << std::max<size_t>(1, G.dst_dat.size()) << "]; double w[" << std::max(1, G.nweights) << "]; };\n";
    G.kname_in = "tcj_g" + std::to_string(gi) + "_in";
    G.kname_edge = "tcj_g" + std::to_string(gi) + "_edge";
    for (int var = 0; var < 2; ++var) {
        if ((var == 0 ? G.nwaves_in : G.nwaves_edge) == 0) continue;
        Gen g(c, G, var);
        // interior kernels: ask for two wavefronts per SIMD (the register
        // windows then fit in 256 registers without spilling, and a second
        // wavefront hides latencies and co-issues scalar work)
        o << "extern \"C\" __global__ void __launch_bounds__(256) ";
        if (var == 0 && G.wpe > 0) o << "__attribute__((amdgpu_waves_per_eu(" << G.wpe << ", " << G.wpe << "))) ";
        o << (var == 0 ? G.kname_in : G.kname_edge) << "(" << S << " a) {\n";
        o << "  const int wid = tcj_lin(blockIdx.x, gridDim.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);\n";
        if (var == 0) {
            const int nsi = G.in_ns;
            o << "  if (wid >= " << G.nwaves_in << ") return;\n";
            o << "  const int strip = wid % " << nsi << ", seg = wid / " << nsi << ";\n";
            o << "  const int X0 = __builtin_amdgcn_readfirstlane(" << G.xlo + G.in_x << " + strip * " << G.Wo
              << "), Y0 = __builtin_amdgcn_readfirstlane(" << G.ylo + G.in_y << " + seg * " << G.Hseg << ");\n";
        } else {
            // the frame around the interior grid: bottom band, top band (both
            // across the whole width), then the left and right bands of the
            // interior rows; owned columns [X0, XE), rows [Y0, YE)
            const int W = G.xhi - G.xlo, Hh = G.yhi - G.ylo, He = G.Hedge;
            const int nB = G.e_ns * G.e_ngb, nT = G.e_ns * G.e_ngt, nL = G.e_nsl * G.e_ngm;
            const int nsl = std::max(1, G.e_nsl), nsr = std::max(1, G.e_nsr);
            o << "  if (wid >= " << G.nwaves_edge << ") return;\n";
            o << "  int xr, xe, yr, ye;\n";
            o << "  if (wid < " << nB << ") { xr = (wid % " << G.e_ns << ") * " << G.Wo << "; xe = min(xr + " << G.Wo
              << ", " << W << "); yr = (wid / " << G.e_ns << ") * " << He << "; ye = min(yr + " << He << ", "
              << G.e_yb << "); }\n";
            o << "  else if (wid < " << nB + nT << ") { const int w = wid - " << nB << "; xr = (w % " << G.e_ns
              << ") * " << G.Wo << "; xe = min(xr + " << G.Wo << ", " << W << "); yr = " << G.e_yt << " + (w / "
              << G.e_ns << ") * " << He << "; ye = min(yr + " << He << ", " << Hh << "); }\n";
            o << "  else if (wid < " << nB + nT + nL << ") { const int w = wid - " << nB + nT << "; xr = (w % " << nsl
              << ") * " << G.Wo << "; xe = min(xr + " << G.Wo << ", " << G.in_x << "); yr = " << G.in_y << " + (w / "
              << nsl << ") * " << He << "; ye = min(yr + " << He << ", " << G.e_yt << "); }\n";
            o << "  else { const int w = wid - " << nB + nT + nL << "; xr = " << G.e_xr << " + (w % " << nsr << ") * "
              << G.Wo << "; xe = min(xr + " << G.Wo << ", " << W << "); yr = " << G.in_y << " + (w / " << nsr
              << ") * " << He << "; ye = min(yr + " << He << ", " << G.e_yt << "); }\n";
            o << "  const int X0 = __builtin_amdgcn_readfirstlane(" << G.xlo << " + xr), XE = "
              << "__builtin_amdgcn_readfirstlane(" << G.xlo << " + xe);\n";
            o << "  const int Y0 = __builtin_amdgcn_readfirstlane(" << G.ylo << " + yr), YE = "
              << "__builtin_amdgcn_readfirstlane(" << G.ylo << " + ye);\n";
        }
        g.body();
        o << g.o.str();
        o << "}\n";
    }
}

// Every cell of the group's range must belong to exactly one wavefront: the
// interior grid's waves plus the edge bands' waves, decoded as the generated
// kernels decode them.  Checked on the owned rectangles over the grid of
// their distinct boundaries.
bool layout_covers_once(const FusedGroup &G) {
    const int W = G.xhi - G.xlo, H = G.yhi - G.ylo, He = G.Hedge;
    struct Rect {
        int x0, x1, y0, y1;
    };
    std::vector<Rect> rects;
    for (int w = 0; w < G.nwaves_in; ++w) {
        const int x0 = G.in_x + (w % G.in_ns) * G.Wo, y0 = G.in_y + (w / G.in_ns) * G.Hseg;
        rects.push_back({x0, x0 + G.Wo, y0, y0 + G.Hseg});
    }
    const int nB = G.e_ns * G.e_ngb, nT = G.e_ns * G.e_ngt, nL = G.e_nsl * G.e_ngm;
    const int nsl = std::max(1, G.e_nsl), nsr = std::max(1, G.e_nsr);
    for (int wid = 0; wid < G.nwaves_edge; ++wid) {
        int xr, xe, yr, ye;
        if (wid < nB) {
            xr = (wid % G.e_ns) * G.Wo;
            xe = std::min(xr + G.Wo, W);
            yr = (wid / G.e_ns) * He;
            ye = std::min(yr + He, G.e_yb);
        } else if (wid < nB + nT) {
            const int w = wid - nB;
            xr = (w % G.e_ns) * G.Wo;
            xe = std::min(xr + G.Wo, W);
            yr = G.e_yt + (w / G.e_ns) * He;
            ye = std::min(yr + He, H);
        } else if (wid < nB + nT + nL) {
            const int w = wid - nB - nT;
            xr = (w % nsl) * G.Wo;
            xe = std::min(xr + G.Wo, G.in_x);
            yr = G.in_y + (w / nsl) * He;
            ye = std::min(yr + He, G.e_yt);
        } else {
            const int w = wid - nB - nT - nL;
            xr = G.e_xr + (w % nsr) * G.Wo;
            xe = std::min(xr + G.Wo, W);
            yr = G.in_y + (w / nsr) * He;
            ye = std::min(yr + He, G.e_yt);
        }
        rects.push_back({xr, xe, yr, ye});
    }
    std::vector<int> xs{0, W}, ys{0, H};
    for (const Rect &r : rects) {
        if (r.x0 < 0 || r.x1 > W || r.y0 < 0 || r.y1 > H || r.x0 >= r.x1 || r.y0 >= r.y1) return false;
        xs.push_back(r.x0);
        xs.push_back(r.x1);
        ys.push_back(r.y0);
        ys.push_back(r.y1);
    }
    std::sort(xs.begin(), xs.end());
    xs.erase(std::unique(xs.begin(), xs.end()), xs.end());
    std::sort(ys.begin(), ys.end());
    ys.erase(std::unique(ys.begin(), ys.end()), ys.end());
    const size_t nx = xs.size() - 1, ny = ys.size() - 1;
    std::vector<int> cnt(nx * ny, 0);
    auto at = [](const std::vector<int> &v, int x) { return (size_t)(std::lower_bound(v.begin(), v.end(), x) - v.begin()); };
    for (const Rect &r : rects)
        for (size_t i = at(xs, r.x0); i < at(xs, r.x1); ++i)
            for (size_t j = at(ys, r.y0); j < at(ys, r.y1); ++j) ++cnt[j * nx + i];
    for (int k : cnt)
        if (k != 1) return false;
    return true;
}

uint64_t fnv1a(const std::string &s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char ch : s) {
        h ^= ch;
        h *= 1099511628211ull;
    }
    return h;
}

// Whether dataset d, written over box [lo, hi) by loop `after` - 1, is read
// by a later loop of the chain before some later loop overwrites all of
// that box (or the chain ends with the value as its final state).
bool live_after(const std::vector<LoopRec> &chain, int after, int d, const int lo[3], const int hi[3]) {
    for (size_t l = after; l < chain.size(); ++l) {
        const LoopRec &lp = chain[l];
        bool reads = false, covers = false;
        for (const auto &a : lp.args) {
            if (a.kind != TC_ARG_DAT || a.handle != d) continue;
            if (a.reads()) reads = true;
            if (a.access == TC_WRITE) {
                covers = true;
                for (int k = 0; k < 3; ++k) covers = covers && lp.lo[k] <= lo[k] && lp.hi[k] >= hi[k];
            }
        }
        if (reads) return true;
        if (covers) return false;
    }
    return true;
}

}  // namespace

bool euler_stage_match(const Ctx &c, const std::vector<LoopRec> &chain, int i, EulerStage &E) {
    if (i + 10 > (int)chain.size()) return false;
    const LoopRec &f = chain[i];
    if (f.ndim != 3) return false;
    int dtype = -1;
    double s = 0.0;
    for (int k = 0; k < 10; ++k) {
        const LoopRec &lp = chain[i + k];
        if (lp.ndim != 3 || lp.block != f.block || lp.op != (k < 5 ? TC_OP_EULER_RHS : TC_OP_RK_STAGE)) return false;
        for (int d = 0; d < 3; ++d)
            if (lp.lo[d] != f.lo[d] || lp.hi[d] != f.hi[d]) return false;
        for (const auto &a : lp.args) {
            if (a.kind != TC_ARG_DAT) return false;
            if (dtype < 0) dtype = c.dats[a.handle].dtype;
            if (c.dats[a.handle].dtype != dtype) return false;
        }
        if (k < 5) {
            // R_c(W), Q_c, u, v, w, p; params (c, s)
            if (lp.args.size() != 6 || (int)lp.params[0] != k || lp.params[0] != (double)k) return false;
            if (k == 0) s = lp.params[1];
            if (lp.params[1] != s) return false;
            E.r[k] = lp.args[0].handle;
            E.q[k] = lp.args[1].handle;
            for (int d = 0; d < 3; ++d) {
                if (k == 0) E.u[d] = lp.args[2 + d].handle;
                if (lp.args[2 + d].handle != E.u[d]) return false;
            }
            if (k == 0) E.p = lp.args[5].handle;
            if (lp.args[5].handle != E.p) return false;
        } else {
            // Q0_c, Q_c(RW), R_c; params (a, b, dt) shared by the five
            const int cc = k - 5;
            if (lp.args.size() != 3 || lp.args[1].handle != E.q[cc] || lp.args[2].handle != E.r[cc]) return false;
            E.q0[cc] = lp.args[0].handle;
            for (int j = 0; j < 3; ++j)
                if (lp.params[j] != chain[i + 5].params[j]) return false;
        }
    }
    // every role a different dataset
    std::vector<int> all;
    for (int k = 0; k < 5; ++k) {
        all.push_back(E.q[k]);
        all.push_back(E.q0[k]);
        all.push_back(E.r[k]);
    }
    for (int d = 0; d < 3; ++d) all.push_back(E.u[d]);
    all.push_back(E.p);
    std::vector<int> sorted = all;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return false;
    for (int d = 0; d < 3; ++d) {
        E.lo[d] = f.lo[d];
        E.hi[d] = f.hi[d];
    }
    for (int k = 0; k < 5; ++k) E.r_live[k] = live_after(chain, i + 10, E.r[k], E.lo, E.hi);
    return true;
}

bool euler_stage_match_prim(const Ctx &c, const std::vector<LoopRec> &chain, int i, EulerStage &E) {
    if (i + 11 > (int)chain.size()) return false;
    const LoopRec &pr = chain[i];
    if (pr.op != TC_OP_EULER_PRIM || pr.ndim != 3 || pr.args.size() != 9) return false;
    if (!euler_stage_match(c, chain, i + 1, E)) return false;
    for (int k = 0; k < 5; ++k)
        if (pr.args[k].kind != TC_ARG_DAT || pr.args[k].handle != E.q[k]) return false;
    for (int d = 0; d < 3; ++d)
        if (pr.args[5 + d].handle != E.u[d]) return false;
    if (pr.args[8].handle != E.p || c.dats[pr.args[0].handle].dtype != c.dats[E.q[0]].dtype) return false;
    // the right-hand sides read the primitives up to 2 points beyond their range
    for (int d = 0; d < 3; ++d)
        if (pr.lo[d] > E.lo[d] - 2 || pr.hi[d] < E.hi[d] + 2) return false;
    const int prims[4] = {E.u[0], E.u[1], E.u[2], E.p};
    for (int v : prims)
        if (live_after(chain, i + 11, v, pr.lo, pr.hi)) return false;
    E.prim = true;
    return true;
}

bool euler_stage_match_copy(const Ctx &c, const std::vector<LoopRec> &chain, int i, bool prim, EulerStage &E) {
    if (i + 5 + (prim ? 11 : 10) > (int)chain.size()) return false;
    if (!(prim ? euler_stage_match_prim(c, chain, i + 5, E) : euler_stage_match(c, chain, i + 5, E))) return false;
    bool seen[5] = {false, false, false, false, false};
    for (int k = 0; k < 5; ++k) {
        const LoopRec &cp = chain[i + k];
        if (cp.op != TC_OP_COPY || cp.ndim != 3 || cp.args.size() != 2) return false;
        for (int d = 0; d < 3; ++d)
            if (cp.lo[d] != E.lo[d] || cp.hi[d] != E.hi[d]) return false;
        const ArgRec &dst = cp.args[0], &src = cp.args[1];
        if (dst.kind != TC_ARG_DAT || src.kind != TC_ARG_DAT) return false;
        if (c.dats[dst.handle].dtype != c.dats[src.handle].dtype) return false;
        int comp = -1;
        for (int cc = 0; cc < 5; ++cc)
            if (E.q[cc] == src.handle && E.q0[cc] == dst.handle) comp = cc;
        if (comp < 0 || seen[comp]) return false;
        seen[comp] = true;
    }
    E.copy0 = true;
    return true;
}

namespace {

// One reflective ghost fill of dataset d along axis `axis`, side `side`,
// depth h, as the 2D heat-conduction chains record them.
bool is_fill(const Ctx &c, const LoopRec &lp, int d, int axis, int side, int h, const int n[2]) {
    if (lp.op != TC_OP_HALO_REFLECT || lp.ndim != 2 || lp.args.size() != 1 || lp.params.size() != 3) return false;
    if (lp.args[0].kind != TC_ARG_DAT || lp.args[0].handle != d) return false;
    if ((int)lp.params[0] != axis || (int)lp.params[1] != side || (int)lp.params[2] != n[axis] ||
        lp.params[0] != (double)axis || lp.params[1] != (double)side || lp.params[2] != (double)n[axis])
        return false;
    const int a = axis, o = 1 - axis;
    const int lo_a = side == 0 ? -h : n[a], hi_a = side == 0 ? 0 : n[a] + h;
    // x fills cover the interior rows, y fills every column (the ghosts too)
    const int lo_o = axis == 0 ? 0 : -h, hi_o = axis == 0 ? n[o] : n[o] + h;
    return lp.lo[a] == lo_a && lp.hi[a] == hi_a && lp.lo[o] == lo_o && lp.hi[o] == hi_o;
}

bool interior_2d(const LoopRec &lp, const int n[2]) {
    return lp.ndim == 2 && lp.lo[0] == 0 && lp.hi[0] == n[0] && lp.lo[1] == 0 && lp.hi[1] == n[1];
}

}  // namespace

int cheb_match(const Ctx &c, const std::vector<LoopRec> &chain, int i, ChebGroup &C) {
    const int L = (int)chain.size();
    C = ChebGroup();
    // the first step's TEA_P1 names the datasets
    if (i + 5 > L) return 0;
    const LoopRec &p1 = chain[i + 4];
    if (p1.op != TC_OP_TEA_P1 || p1.ndim != 2 || p1.args.size() != 5 || !p1.params.empty()) return 0;
    for (const auto &a : p1.args)
        if (a.kind != TC_ARG_DAT) return 0;
    C.kx = p1.args[0].handle;
    C.ky = p1.args[1].handle;
    C.sd = p1.args[2].handle;
    C.rt = p1.args[3].handle;
    C.z = p1.args[4].handle;
    const int ds[5] = {C.kx, C.ky, C.sd, C.rt, C.z};
    for (int a = 0; a < 5; ++a)
        for (int b = a + 1; b < 5; ++b)
            if (ds[a] == ds[b]) return 0;
    const Dataset &S = c.dats[C.sd];
    for (int a = 0; a < 5; ++a)
        if (c.dats[ds[a]].dtype != S.dtype || c.dats[ds[a]].block != S.block) return 0;
    C.n[0] = S.size[0];
    C.n[1] = S.size[1];
    if (!interior_2d(p1, C.n)) return 0;
    const LoopRec &f0 = chain[i];
    if (f0.op != TC_OP_HALO_REFLECT || f0.ndim != 2) return 0;
    C.h = -f0.lo[0];
    if (C.h < 1 || C.h > kChebMaxSteps || C.h > S.hneg[0] || C.h > S.hneg[1] || C.h > S.hpos[0] ||
        C.h > S.hpos[1] || C.n[0] < 2 * C.h || C.n[1] < 2 * C.h)
        return 0;
    int l = i;
    while (C.steps < kChebMaxSteps && l + 5 <= L) {
        bool ok = is_fill(c, chain[l], C.sd, 0, 0, C.h, C.n) && is_fill(c, chain[l + 1], C.sd, 0, 1, C.h, C.n) &&
                  is_fill(c, chain[l + 2], C.sd, 1, 0, C.h, C.n) && is_fill(c, chain[l + 3], C.sd, 1, 1, C.h, C.n);
        const LoopRec &q = chain[l + 4];
        ok = ok && q.op == TC_OP_TEA_P1 && q.args.size() == 5 && interior_2d(q, C.n);
        for (int a = 0; ok && a < 5; ++a) ok = q.args[a].kind == TC_ARG_DAT && q.args[a].handle == ds[a];
        if (!ok) break;
        l += 5;
        ++C.steps;
        const bool p2 = l < L && chain[l].op == TC_OP_TEA_P2 && chain[l].args.size() == 2 &&
                        interior_2d(chain[l], C.n) && chain[l].args[0].kind == TC_ARG_DAT &&
                        chain[l].args[0].handle == C.sd && chain[l].args[1].kind == TC_ARG_DAT &&
                        chain[l].args[1].handle == C.rt && chain[l].params.size() == 2;
        if (!p2) {
            C.last_p2 = false;
            C.p2_loop.push_back(-1);
            break;
        }
        C.p2_loop.push_back(l);
        ++l;
    }
    return C.steps > 0 ? l - i : 0;
}

bool fused_op_supported(const LoopRec &lp) { return lp.op == TC_OP_WSUM && lp.ndim == 2; }

std::vector<std::shared_ptr<FusedGroup>> fused_split(Ctx &c, const std::vector<LoopRec> &chain, const int tile[3],
                                                     int cpl) {
    SplitParams sp;
    sp.bake = c.jit_bake;
    sp.hseg = tile[0] > 0 ? tile[0] : 0;
    sp.regs = tile[1] > 0 ? tile[1] : 160;
    sp.max_loops = tile[2] > 0 ? tile[2] : 32;
    sp.U = std::max(1, c.jit_unroll);
    sp.PF = std::max(1, c.jit_prefetch);
    sp.cpl = cpl == 2 ? 2 : 1;
    sp.wpe = c.jit_wpe;
    sp.max_window = c.jit_max_window;
    sp.cse_steps = c.jit_cse_steps;
    sp.sched_fence = c.jit_sched_fence;
    sp.align_store = c.jit_align_store;
    sp.edge_div = c.jit_edge_div;
    const int L = (int)chain.size();
    // staged candidates [i, j) whose full analysis failed (some tile needs
    // more LDS than the representative ones)
    std::vector<std::pair<int, int>> bad;
    std::vector<std::shared_ptr<FusedGroup>> out;
    for (int attempt = 0; attempt < 8; ++attempt) {
        // best[j]: least modelled time of loops [0, j); from[j]: start of the last piece
        std::vector<double> best(L + 1, 1e300);
        std::vector<int> from(L + 1, -1);
        std::vector<std::shared_ptr<FusedGroup>> piece(L + 1);
        best[0] = 0.0;
        // runs of 2D Chebyshev steps: every whole-step prefix of the longest
        // run from each loop, by the group's end
        std::vector<std::vector<std::shared_ptr<FusedGroup>>> cheb_end(L + 1);
        for (int i = 0; i < L; ++i) {
            ChebGroup C;
            // a run may start with the preconditioner's set-up (TEA_PRECON_INIT:
            // r read, rt, sd and z written over the interior, theta)
            // and the CG update of x and r before that (TEA_CG_UPDATE)
            const bool upd = chain[i].op == TC_OP_TEA_CG_UPDATE && i + 1 < L &&
                             chain[i + 1].op == TC_OP_TEA_PRECON_INIT;
            const int i0 = upd ? i + 1 : i;
            const bool init = chain[i0].op == TC_OP_TEA_PRECON_INIT;
            const int f0 = init ? i0 + 1 : i0;
            if (!c.cheb_enabled || f0 >= L || chain[f0].op != TC_OP_HALO_REFLECT || cheb_match(c, chain, f0, C) == 0)
                continue;
            if (init) {
                const LoopRec &q = chain[i0];
                bool ok = q.ndim == 2 && q.args.size() == 4 && q.params.size() == 1 && q.lo[0] == 0 &&
                          q.hi[0] == C.n[0] && q.lo[1] == 0 && q.hi[1] == C.n[1];
                for (int a = 0; ok && a < 4; ++a) ok = q.args[a].kind == TC_ARG_DAT;
                ok = ok && q.args[1].handle == C.rt && q.args[2].handle == C.sd && q.args[3].handle == C.z;
                if (ok) {
                    const int r = q.args[0].handle;
                    ok = r != C.kx && r != C.ky && r != C.sd && r != C.rt && r != C.z &&
                         c.dats[r].dtype == c.dats[C.sd].dtype && c.dats[r].block == c.dats[C.sd].block;
                    C.r = r;
                    C.init_loop = i0;
                }
                if (!ok) continue;
            }
            if (upd) {
                const LoopRec &q = chain[i];
                bool ok = q.ndim == 2 && q.args.size() == 4 && q.params.size() == 1 && q.lo[0] == 0 &&
                          q.hi[0] == C.n[0] && q.lo[1] == 0 && q.hi[1] == C.n[1];
                for (int a = 0; ok && a < 4; ++a) ok = q.args[a].kind == TC_ARG_DAT;
                ok = ok && q.args[1].handle == C.r;
                if (ok) {
                    C.x = q.args[0].handle;
                    C.p = q.args[2].handle;
                    C.w = q.args[3].handle;
                    const int all[9] = {C.kx, C.ky, C.sd, C.rt, C.z, C.r, C.x, C.p, C.w};
                    for (int a = 0; ok && a < 9; ++a)
                        for (int b = a + 1; ok && b < 9; ++b) ok = all[a] != all[b];
                    for (int d : {C.x, C.p, C.w})
                        ok = ok && c.dats[d].dtype == c.dats[C.sd].dtype && c.dats[d].block == c.dats[C.sd].block;
                    C.update_loop = i;
                }
                if (!ok) continue;
            }
            // at most five steps unless asked: measured on the PPCG solve at
            // 2000^2 (ms per solve) 3 steps 29.3, 4 28.4, 5 24.3, 7 34.1,
            // 9 39.4 (the wider recomputed borders and their registers cost
            // more than the traffic they save)
            for (int m = 1; m <= C.steps; ++m) {
                if (c.cheb_steps > 0 ? m != std::min(C.steps, c.cheb_steps) : m > 5) continue;
                auto P = std::make_shared<ChebGroup>(C);
                P->steps = m;
                P->last_p2 = C.p2_loop[m - 1] >= 0;
                P->p2_loop.resize(m);
                const int len = 5 * m + (P->last_p2 ? m : m - 1) + (init ? 1 : 0) + (upd ? 1 : 0);
                // bytes: face coefficients, rt and sd over the region of a
                // tile, z over the owned cells; rt, z and sd written once.
                // A region's border is mostly read from L2 (the neighbouring
                // tiles load it too): HBM sees about 1.15 times the owned
                // cells of each region-loaded array
                const double f = 1.15;
                const double cells = (double)C.n[0] * C.n[1];
                // (with the set-up first: r over the region instead of rt,
                // sd and z)
                const double arrays = init ? 3.0 * f + 3.0 : 4.0 * f + 1.0 + 3.0;
                const double bytes = cells * c.dats[C.sd].esize() * arrays;
                auto G = std::make_shared<FusedGroup>();
                G->g0 = i;
                G->g1 = i + len;
                G->cost = bytes / 4.5e12 + 6e-6;
                // the update folded in saves its launch but reads w and r
                // over every region and x and p with them: measured, the
                // fold gains on small grids (256^2 5.42 -> 5.20 ms per solve,
                // 700^2 7.10 -> 6.81) and loses on large ones (2000^2 23.31
                // -> 24.62, 4000^2 85.74 -> 88.58), so it is modelled at 1.2
                // times the update's own streaming time
                if (upd) G->cost += 1.2 * loop_stream_time(c, chain[i]);
                G->alg_bytes = (int64_t)(cells * c.dats[C.sd].esize() * 8.0);
                G->cheb = P;
                cheb_end[i + len].push_back(G);
            }
        }
        for (int j = 1; j <= L; ++j) {
            const double s = best[j - 1] + single_loop_cost(c, chain[j - 1]);
            if (s < best[j]) {
                best[j] = s;
                from[j] = j - 1;
                piece[j] = nullptr;
            }
            for (const auto &G : cheb_end[j])
                if (best[G->g0] + G->cost < best[j]) {
                    best[j] = best[G->g0] + G->cost;
                    from[j] = G->g0;
                    piece[j] = G;
                }
            // a 3D Runge-Kutta stage ending here (with its primitive-variable
            // loop when their values die in the chain, and the step's copies
            // Q0 = Q before it): one z-marching kernel
            for (int len : {16, 15, 11, 10}) {
                if (j < len) continue;
                EulerStage E;
                const bool ok = len >= 15 ? euler_stage_match_copy(c, chain, j - len, len == 16, E)
                                : len == 11 ? euler_stage_match_prim(c, chain, j - 11, E)
                                            : euler_stage_match(c, chain, j - 10, E);
                if (!ok) continue;
                const LoopRec &f = chain[j - 10];
                int nlive = 0;
                for (bool b : E.r_live) nlive += b;
                const int arrays = (E.prim ? 15 : 19) + nlive;
                const double cost = (double)f.points() * c.dats[E.q[0]].esize() * arrays / 4.5e12 + 5e-6;
                if (best[j - len] + cost < best[j]) {
                    auto G = std::make_shared<FusedGroup>();
                    G->g0 = j - len;
                    G->g1 = j;
                    G->cost = cost;
                    G->estage = std::make_shared<EulerStage>(E);
                    G->alg_bytes = f.points() * (int64_t)c.dats[E.q[0]].esize() * arrays;
                    best[j] = best[j - len] + cost;
                    from[j] = j - len;
                    piece[j] = G;
                }
            }
            // register-window groups: runs of 2D weighted sums; staged groups:
            // runs that register windows cannot take (any op, dimension, range)
            bool reg_ok = true, stg_ok = c.staged_mode != 0, all_wsum = true;
            for (int i = j - 1; i >= 0; --i) {
                if (!fused_op_supported(chain[i])) {
                    reg_ok = false;
                    all_wsum = false;
                }
                if (j - i < 2) continue;
                if (reg_ok && j - i <= sp.max_loops) {
                    auto G = std::make_shared<FusedGroup>();
                    if (analyse(c, chain, i, j, sp, *G) && best[i] + G->cost < best[j]) {
                        best[j] = best[i] + G->cost;
                        from[j] = i;
                        piece[j] = G;
                    }
                }
                if (stg_ok && !all_wsum) {
                    if (j - i > kSMaxLoops) {
                        stg_ok = false;
                    } else if (std::find(bad.begin(), bad.end(), std::make_pair(i, j)) == bad.end()) {
                        auto S = std::make_shared<StagedGroup>();
                        if (!staged_analyse(c, chain, i, j, c.staged_tile, false, *S)) {
                            stg_ok = false;  // prepending loops only adds datasets, parameters and LDS
                        } else if (c.staged_mode == 2 ? S->cost * 1e-6 < best[j] - best[i]
                                                      : best[i] + S->cost < best[j]) {
                            if (c.staged_mode == 2) S->cost *= 1e-6;
                            auto G = std::make_shared<FusedGroup>();
                            G->g0 = i;
                            G->g1 = j;
                            G->cost = S->cost;
                            G->staged = S;
                            best[j] = best[i] + S->cost;
                            from[j] = i;
                            piece[j] = G;
                        }
                    }
                }
                if (!reg_ok && !stg_ok) break;
            }
        }
        out.clear();
        for (int j = L; j > 0; j = from[j])
            if (piece[j]) out.push_back(piece[j]);
        std::reverse(out.begin(), out.end());
        // staged groups: every tile walked, tables built
        bool ok = true;
        for (auto &g : out) {
            if (!g->staged) continue;
            auto full = std::make_shared<StagedGroup>();
            if (!staged_analyse(c, chain, g->g0, g->g1, c.staged_tile, true, *full)) {
                bad.push_back({g->g0, g->g1});
                ok = false;
                continue;
            }
            g->staged = full;
            g->nblocks = full->ntot;
            g->alg_bytes = full->alg_bytes;
        }
        if (ok) break;
        if (attempt == 7)  // give up on the failing groups: their loops run one kernel each
            out.erase(std::remove_if(out.begin(), out.end(),
                                     [](const std::shared_ptr<FusedGroup> &g) { return g->staged && g->staged->rec == 0; }),
                      out.end());
    }
    if (getenv("TC_JIT_VERBOSE"))
        for (const auto &g : out) {
            if (g->estage) {
                std::fprintf(stderr, "Runge-Kutta stage group [%d,%d): cost %.1f us\n", g->g0, g->g1, g->cost * 1e6);
                continue;
            }
            if (g->cheb) {
                std::fprintf(stderr, "Chebyshev group [%d,%d): %d steps%s, cost %.1f us\n", g->g0, g->g1,
                             g->cheb->steps, g->cheb->last_p2 ? "" : " (last without P2)", g->cost * 1e6);
                continue;
            }
            if (g->staged) {
                const StagedGroup &S = *g->staged;
                std::fprintf(stderr,
                             "staged group [%d,%d): tile %dx%dx%d, %d tiles of %d threads, %d slots, LDS %lld B, cost "
                             "%.1f us\n",
                             g->g0, g->g1, S.tile[0], S.tile[1], S.tile[2], S.ntot, S.threads, (int)S.slots.size(),
                             (long long)(S.desc_off + (int64_t)sizeof(LoopDesc)), S.cost * 1e6);
                continue;
            }
            int nl = 0, nld = 0;
            for (const auto &J : g->loops) nl += J.needed;
            for (char x : g->var[0].loaded) nld += x;
            std::fprintf(stderr,
                         "fused group [%d,%d): %d loops, HL %d HR %d Wo %d, loads %d stores %d, regs %d/%d, "
                         "pre %d post %d, Hseg %d Hedge %d, interior %dx%d at (%d,%d), waves %d+%d, cost %.1f us\n",
                         g->g0, g->g1, nl, g->HL, g->HR, g->Wo, nld, (int)g->dst_dat.size(), g->var[0].regs,
                         g->var[1].regs, g->var[0].pre, g->var[0].post, g->Hseg, g->Hedge, g->in_ns, g->in_ng, g->in_x, g->in_y, g->nwaves_in,
                         g->nwaves_edge, g->cost * 1e6);
        }
    return out;
}

tc_status fused_compile(Ctx &c, const std::vector<LoopRec> &chain, std::vector<std::shared_ptr<FusedGroup>> &all) {
    std::vector<std::shared_ptr<FusedGroup>> groups;
    for (auto &g : all) {
        if (g->estage || g->cheb) continue;  // a precompiled kernel
        if (!g->staged) {
            groups.push_back(g);
            continue;
        }
        if (!g->staged->dev) {
            const tc_status st = staged_upload(c, chain, *g->staged);
            if (st != TC_OK) return st;
        }
    }
    if (groups.empty()) return TC_OK;
    for (const auto &g : groups)
        if (!layout_covers_once(*g))
            return fail(c, TC_ERR_STATE, "fused group [%d,%d): wavefront layout does not cover its range once", g->g0,
                        g->g1);
    std::ostringstream src;
    src << kPrelude;
    try {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            // testing aid: every register window one row short, so that the
            // generator's window check fails and the error reaches the caller
            if (c.jit_test_short_windows)
                for (auto &V : groups[gi]->var)
                    for (int &w : V.win) w = std::max(0, w - 1);
            gen_group(c, *groups[gi], (int)gi, src);
        }
    } catch (const std::logic_error &e) {
        return fail(c, TC_ERR_STATE, "%s", e.what());
    }
    const std::string s = src.str();
    if (const char *dump = getenv("TC_JIT_DUMP")) {
        if (FILE *fp = std::fopen(dump, "w")) {
            std::fwrite(s.data(), 1, s.size(), fp);
            std::fclose(fp);
        }
    }
    const uint64_t key = fnv1a(s) ^ ((uint64_t)c.device << 56);
    hipModule_t mod = nullptr;
    auto it = c.jit_modules.find(key);
    if (it != c.jit_modules.end()) {
        mod = it->second;
    } else {
        const double t0 = now_s();
        hiprtcProgram prog;
        if (hiprtcCreateProgram(&prog, s.c_str(), "tilechain_fused.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
            return fail(c, TC_ERR_DEVICE, "hiprtcCreateProgram failed");
        const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
        const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
        if (r != HIPRTC_SUCCESS) {
            size_t n = 0;
            hiprtcGetProgramLogSize(prog, &n);
            std::string log(n + 1, '\0');
            hiprtcGetProgramLog(prog, &log[0]);
            hiprtcDestroyProgram(&prog);
            return fail(c, TC_ERR_DEVICE, "fused kernel compilation failed: %.2000s", log.c_str());
        }
        size_t n = 0;
        hiprtcGetCodeSize(prog, &n);
        std::vector<char> code(n);
        hiprtcGetCode(prog, code.data());
        hiprtcDestroyProgram(&prog);
        if (const char *dump = getenv("TC_JIT_DUMP_CO")) {
            if (FILE *fp = std::fopen(dump, "wb")) {
                std::fwrite(code.data(), 1, code.size(), fp);
                std::fclose(fp);
            }
        }
        if (!c.host_only && hipModuleLoadData(&mod, code.data()) != hipSuccess)
            return fail(c, TC_ERR_DEVICE, "hipModuleLoadData of the fused kernels failed");
        c.jit_modules[key] = mod;
        c.jit_compile_seconds += now_s() - t0;
    }
    if (c.host_only) return TC_OK;
    for (auto &g : groups) {
        if (g->nwaves_in > 0 && hipModuleGetFunction(&g->fin, mod, g->kname_in.c_str()) != hipSuccess)
            return fail(c, TC_ERR_DEVICE, "fused kernel %s not found", g->kname_in.c_str());
        if (g->nwaves_edge > 0 && hipModuleGetFunction(&g->fedge, mod, g->kname_edge.c_str()) != hipSuccess)
            return fail(c, TC_ERR_DEVICE, "fused kernel %s not found", g->kname_edge.c_str());
    }
    return TC_OK;
}

// Second buffer of a dataset the group reads at offsets and writes over
// [lo, hi): allocated on first use and made equal to the current buffer
// outside that box.  Returns its logical origin through *origin.
tc_status second_buffer(Ctx &c, Dataset &ds, const int lo[3], const int hi[3], void **origin) {
    const int tw = 1 - ds.cur;
    if (!ds.raw[tw] && c.noalloc)
        return fail(c, TC_ERR_STATE,
                    "the second buffer of %s does not exist yet and a call that allocates nothing cannot create "
                    "it; flush this chain once with tc_flush first", ds.name.c_str());
    if (!ds.raw[tw]) {
        ds.raw[tw] = dev_alloc(c, (size_t)(ds.bytes + ds.stagger));
        if (!ds.raw[tw]) return fail(c, TC_ERR_NOMEM, "cannot allocate the second buffer of %s", ds.name.c_str());
        ds.buf[tw] = (char *)ds.raw[tw] + ds.stagger;
        ds.twin_synced = false;
    }
    bool inside = true;
    if (ds.ever_written)
        for (int d = 0; d < 3; ++d) inside = inside && ds.wlo[d] >= lo[d] && ds.whi[d] <= hi[d];
    if (!ds.twin_synced || !inside) {
        if (hipMemcpyAsync(ds.buf[tw], ds.buf[ds.cur], (size_t)ds.bytes, hipMemcpyDeviceToDevice, c.stream) !=
            hipSuccess)
            return fail(c, TC_ERR_DEVICE, "hipMemcpyAsync (second buffer) failed");
        ds.twin_synced = true;
    }
    *origin = ds.origin(tw);
    return TC_OK;
}

tc_status euler_stage_run(Ctx &c, const std::vector<LoopRec> &chain, const FusedGroup &G) {
    const EulerStage &E = *G.estage;
    EulerStageArgs a;
    std::memset(&a, 0, sizeof a);
    auto put = [&](int k, int d) {
        const Dataset &ds = c.dats[d];
        a.ptr[k] = ds.origin(ds.cur);
        a.sy[k] = ds.sy();
        a.sz[k] = ds.sz();
    };
    for (int k = 0; k < 5; ++k) {
        put(kQ + k, E.q[k]);
        put(kQ0 + k, E.q0[k]);
    }
    for (int d = 0; d < 3; ++d) put(kU + d, E.u[d]);
    put(kP, E.p);
    for (int k = 0; k < 5; ++k) {
        Dataset &dq = c.dats[E.q[k]];
        const tc_status st = second_buffer(c, dq, E.lo, E.hi, &a.out[k]);
        if (st != TC_OK) return st;
        a.osy[k] = dq.sy();
        a.osz[k] = dq.sz();
        if (E.r_live[k]) {
            const Dataset &dr = c.dats[E.r[k]];
            a.rout[k] = dr.origin(dr.cur);
            a.rsy[k] = dr.sy();
            a.rsz[k] = dr.sz();
        }
    }
    const int c0 = E.copy0 ? 5 : 0, off = c0 + (E.prim ? 1 : 0);
    const LoopRec &rhs = chain[G.g0 + off], &rk = chain[G.g0 + off + 5];
    a.prim = E.prim ? 1 : 0;
    a.gm1 = E.prim ? chain[G.g0 + c0].params[0] : 0.0;
    a.copy0 = E.copy0 ? 1 : 0;
    if (E.copy0)
        for (int k = 0; k < 5; ++k) {
            // Q0 is read by no loop of the group but the updates at the same
            // point, which take its value from Q: written in place
            const Dataset &d0 = c.dats[E.q0[k]];
            a.q0out[k] = d0.origin(d0.cur);
            a.q0sy[k] = d0.sy();
            a.q0sz[k] = d0.sz();
        }
    a.s = rhs.params[1];
    a.a = rk.params[0];
    a.b = rk.params[1];
    a.dt = rk.params[2];
    for (int d = 0; d < 3; ++d) {
        a.lo[d] = E.lo[d];
        a.hi[d] = E.hi[d];
    }
    a.rows = c.march.rows3;
    a.tz = c.march.tz3;
    const hipError_t e = launch_euler_stage3(a, c.dats[E.q[0]].dtype, c.stream);
    if (e != hipSuccess) return fail(c, TC_ERR_DEVICE, "Runge-Kutta stage launch failed: %s", hipGetErrorString(e));
    for (int k = 0; k < 5; ++k) c.dats[E.q[k]].cur ^= 1;
    return TC_OK;
}

tc_status cheb_run(Ctx &c, const std::vector<LoopRec> &chain, const FusedGroup &G) {
    const ChebGroup &C = *G.cheb;
    if (C.steps > kChebMaxSteps) return fail(c, TC_ERR_STATE, "Chebyshev group of %d steps", C.steps);
    ChebArgs a;
    std::memset(&a, 0, sizeof a);
    const Dataset &kx = c.dats[C.kx], &ky = c.dats[C.ky];
    a.kx = kx.origin(kx.cur);
    a.skx = kx.sy();
    a.ky = ky.origin(ky.cur);
    a.sky = ky.sy();
    Dataset &sd = c.dats[C.sd], &rt = c.dats[C.rt], &z = c.dats[C.z];
    a.sd_in = sd.origin(sd.cur);
    a.ssd_in = sd.sy();
    a.rt_in = rt.origin(rt.cur);
    a.srt_in = rt.sy();
    a.z = z.origin(z.cur);
    a.sz = z.sy();
    // sd is written over the interior and its ghosts, rt over the interior
    const int slo[3] = {-C.h, -C.h, 0}, shi[3] = {C.n[0] + C.h, C.n[1] + C.h, 1};
    const int rlo[3] = {0, 0, 0}, rhi[3] = {C.n[0], C.n[1], 1};
    tc_status st = second_buffer(c, sd, slo, shi, &a.sd_out);
    if (st != TC_OK) return st;
    st = second_buffer(c, rt, rlo, rhi, &a.rt_out);
    if (st != TC_OK) return st;
    a.ssd_out = sd.sy();
    a.srt_out = rt.sy();
    for (int j = 0; j < C.steps; ++j)
        if (C.p2_loop[j] >= 0) {
            a.al[j] = chain[C.p2_loop[j]].params[0];
            a.be[j] = chain[C.p2_loop[j]].params[1];
        }
    if (C.init_loop >= 0) {
        Dataset &r = c.dats[C.r];
        a.start = 1;
        a.r = r.origin(r.cur);
        a.sr = r.sy();
        a.theta = chain[C.init_loop].params[0];
        if (C.update_loop >= 0) {
            // r is read over every workgroup's region: its new values go to
            // the second buffer; x is read and written at its own cells only
            const Dataset &p = c.dats[C.p], &w = c.dats[C.w];
            Dataset &x = c.dats[C.x];
            a.update = 1;
            a.alpha = chain[C.update_loop].params[0];
            a.p = p.origin(p.cur);
            a.sp = p.sy();
            a.w = w.origin(w.cur);
            a.sw = w.sy();
            a.x = x.origin(x.cur);
            a.sx = x.sy();
            const int ilo[3] = {0, 0, 0}, ihi[3] = {C.n[0], C.n[1], 1};
            st = second_buffer(c, r, ilo, ihi, &a.r_out);
            if (st != TC_OK) return st;
            a.sro = r.sy();
        }
    }
    a.n0 = C.n[0];
    a.n1 = C.n[1];
    a.h = C.h;
    a.steps = C.steps;
    a.last_p2 = C.last_p2 ? 1 : 0;
    const hipError_t e = launch_cheb2(a, sd.dtype, c.stream);
    if (e != hipSuccess) return fail(c, TC_ERR_DEVICE, "Chebyshev group launch failed: %s", hipGetErrorString(e));
    sd.cur ^= 1;
    rt.cur ^= 1;
    if (C.update_loop >= 0) c.dats[C.r].cur ^= 1;
    return TC_OK;
}

tc_status fused_run(Ctx &c, const std::vector<LoopRec> &chain, FusedGroup &G) {
    if (G.staged) return staged_run(c, chain, *G.staged);
    if (G.estage) return euler_stage_run(c, chain, G);
    if (G.cheb) return cheb_run(c, chain, G);
    if (G.baked) {
        // kernels with the weights compiled in serve only the weights they
        // were generated for; on a change the group falls back for good to
        // kernels that read the weights from their arguments
        size_t k = 0;
        bool same = true;
        for (int l = G.g0; l < G.g1 && same; ++l)
            for (double w : chain[l].params) same = same && k < G.wvals.size() && G.wvals[k++] == w;
        if (!same) {
            if (c.noalloc)
                return fail(c, TC_ERR_STATE,
                            "fused group [%d,%d): new weights need kernels compiled and loaded, which a call that "
                            "allocates nothing cannot do; flush once with tc_flush first", G.g0, G.g1);
            if (getenv("TC_JIT_VERBOSE"))
                std::fprintf(stderr, "fused group [%d,%d): weights changed, switching to argument weights\n", G.g0,
                             G.g1);
            G.baked = false;
            std::vector<std::shared_ptr<FusedGroup>> one{std::shared_ptr<FusedGroup>(&G, [](FusedGroup *) {})};
            const tc_status st = fused_compile(c, chain, one);
            if (st != TC_OK) return st;
        }
    }
    if ((G.nwaves_in > 0 && !G.fin) || (G.nwaves_edge > 0 && !G.fedge))
        return fail(c, TC_ERR_STATE, "fused group kernels are not loaded");
    // kernel arguments: source pointers, destination pointers, weights
    const size_t ns = std::max<size_t>(1, G.src_dat.size()), nd = std::max<size_t>(1, G.dst_dat.size());
    std::vector<unsigned char> buf(8 * (ns + nd + (size_t)std::max(1, G.nweights)), 0);
    auto put = [&](size_t slot, const void *p) { std::memcpy(&buf[8 * slot], &p, 8); };
    for (size_t i = 0; i < G.src_dat.size(); ++i) {
        const Dataset &ds = c.dats[G.src_dat[i]];
        put(i, ds.origin(ds.cur));
    }
    for (size_t i = 0; i < G.dst_dat.size(); ++i) {
        Dataset &ds = c.dats[G.dst_dat[i]];
        if (!G.dst_twin[i]) {
            put(ns + i, ds.origin(ds.cur));
            continue;
        }
        const int tw = 1 - ds.cur;
        if (!ds.raw[tw] && c.noalloc)
            return fail(c, TC_ERR_STATE,
                        "the second buffer of %s does not exist yet and a call that allocates nothing cannot create "
                        "it; flush this chain once with tc_flush first", ds.name.c_str());
        if (!ds.raw[tw]) {
            ds.raw[tw] = dev_alloc(c, (size_t)(ds.bytes + ds.stagger));
            if (!ds.raw[tw]) return fail(c, TC_ERR_NOMEM, "cannot allocate the second buffer of %s", ds.name.c_str());
            ds.buf[tw] = (char *)ds.raw[tw] + ds.stagger;
            ds.twin_synced = false;
        }
        // the second buffer must equal the current one outside the range
        // written here; it does outside the hull of earlier writes
        const bool inside = !ds.ever_written || (ds.wlo[0] >= G.xlo && ds.whi[0] <= G.xhi && ds.wlo[1] >= G.ylo &&
                                                 ds.whi[1] <= G.yhi);
        if (!ds.twin_synced || !inside) {
            if (hipMemcpyAsync(ds.buf[tw], ds.buf[ds.cur], (size_t)ds.bytes, hipMemcpyDeviceToDevice, c.stream) !=
                hipSuccess)
                return fail(c, TC_ERR_DEVICE, "hipMemcpyAsync (second buffer) failed");
            ds.twin_synced = true;
        }
        put(ns + i, ds.origin(tw));
    }
    {
        size_t k = 0;
        for (int l = G.g0; l < G.g1; ++l)
            for (double w : chain[l].params) std::memcpy(&buf[8 * (ns + nd + k++)], &w, 8);
    }
    size_t sz = buf.size();
    void *cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, buf.data(), HIP_LAUNCH_PARAM_BUFFER_SIZE, &sz, HIP_LAUNCH_PARAM_END};
    if (G.nwaves_edge > 0) {
        const unsigned nb = (unsigned)((G.nwaves_edge + 3) / 4);
        const hipError_t e = hipModuleLaunchKernel(G.fedge, nb, 1, 1, 256, 1, 1, 0, c.stream, nullptr, cfg);
        if (e != hipSuccess) return fail(c, TC_ERR_DEVICE, "fused kernel launch failed: %s", hipGetErrorString(e));
    }
    if (G.nwaves_in > 0) {
        const unsigned nb = (unsigned)((G.nwaves_in + 3) / 4);
        const hipError_t e = hipModuleLaunchKernel(G.fin, nb, 1, 1, 256, 1, 1, 0, c.stream, nullptr, cfg);
        if (e != hipSuccess) return fail(c, TC_ERR_DEVICE, "fused kernel launch failed: %s", hipGetErrorString(e));
    }
    for (size_t i = 0; i < G.dst_dat.size(); ++i)
        if (G.dst_twin[i]) {
            Dataset &ds = c.dats[G.dst_dat[i]];
            ds.cur = 1 - ds.cur;
        }
    return TC_OK;
}

tc_status fused_check_noalloc(Ctx &c, const std::vector<LoopRec> &chain, const FusedGroup &G) {
    if (G.staged) return staged_check_noalloc(c, *G.staged);
    if (G.cheb) {
        for (int d : {G.cheb->sd, G.cheb->rt, G.cheb->update_loop >= 0 ? G.cheb->r : G.cheb->sd}) {
            const Dataset &ds = c.dats[d];
            if (!ds.raw[0] || !ds.raw[1])
                return fail(c, TC_ERR_STATE,
                            "the second buffer of %s does not exist yet and a call that allocates nothing cannot "
                            "create it; flush this chain once with tc_flush first", ds.name.c_str());
        }
        return TC_OK;
    }
    if (G.estage) {
        for (int k = 0; k < 5; ++k) {
            const Dataset &ds = c.dats[G.estage->q[k]];
            if (!ds.raw[0] || !ds.raw[1])
                return fail(c, TC_ERR_STATE,
                            "the second buffer of %s does not exist yet and a call that allocates nothing cannot "
                            "create it; flush this chain once with tc_flush first", ds.name.c_str());
        }
        return TC_OK;
    }
    if (G.baked) {
        size_t k = 0;
        for (int l = G.g0; l < G.g1; ++l)
            for (double w : chain[l].params)
                if (k >= G.wvals.size() || G.wvals[k++] != w)
                    return fail(c, TC_ERR_STATE,
                                "fused group [%d,%d): new weights need kernels compiled and loaded, which a call that "
                                "allocates nothing cannot do; flush once with tc_flush first", G.g0, G.g1);
    }
    for (size_t i = 0; i < G.dst_dat.size(); ++i)
        if (G.dst_twin[i] && (!c.dats[G.dst_dat[i]].raw[0] || !c.dats[G.dst_dat[i]].raw[1]))
            return fail(c, TC_ERR_STATE,
                        "the second buffer of %s does not exist yet and a call that allocates nothing cannot create "
                        "it; flush this chain once with tc_flush first", c.dats[G.dst_dat[i]].name.c_str());
    return TC_OK;
}

void fused_release(Ctx &c) {
    for (auto &kv : c.plans)
        for (auto &g : kv.second->groups) g->fin = g->fedge = nullptr;
    for (auto &kv : c.jit_modules)
        if (kv.second) (void)hipModuleUnload(kv.second);
    c.jit_modules.clear();
}

}  // namespace tc
