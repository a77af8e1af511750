// Staged tiles: analysis (per-tile need boxes, LDS layout, second buffers),
// descriptor upload and launch.  The scheme is described in staged.hpp.
#include "staged.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include "fused.hpp"

namespace tc {

void build_desc(const Ctx &c, const LoopRec &lp, LoopDesc &d);  // api.cpp

namespace {

struct B3 {
    int lo[3], hi[3];
};

B3 none() {
    B3 b;
    for (int d = 0; d < 3; ++d) {
        b.lo[d] = INT_MAX / 2;
        b.hi[d] = INT_MIN / 2;
    }
    return b;
}

bool empty(const B3 &b) {
    for (int d = 0; d < 3; ++d)
        if (b.hi[d] <= b.lo[d]) return true;
    return false;
}

B3 hull(const B3 &a, const B3 &b) {
    if (empty(a)) return b;
    if (empty(b)) return a;
    B3 r;
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = std::min(a.lo[d], b.lo[d]);
        r.hi[d] = std::max(a.hi[d], b.hi[d]);
    }
    return r;
}

B3 isect(const B3 &a, const B3 &b) {
    B3 r;
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = std::max(a.lo[d], b.lo[d]);
        r.hi[d] = std::min(a.hi[d], b.hi[d]);
    }
    return empty(r) ? none() : r;
}

bool contains(const B3 &outer, const B3 &inner) {
    if (empty(inner)) return true;
    if (empty(outer)) return false;
    for (int d = 0; d < 3; ++d)
        if (inner.lo[d] < outer.lo[d] || inner.hi[d] > outer.hi[d]) return false;
    return true;
}

int64_t vol(const B3 &b) {
    if (empty(b)) return 0;
    return (int64_t)(b.hi[0] - b.lo[0]) * (b.hi[1] - b.lo[1]) * (b.hi[2] - b.lo[2]);
}

B3 range_of(const LoopRec &lp) {
    B3 r;
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = lp.lo[d];
        r.hi[d] = lp.hi[d];
    }
    return empty(r) ? none() : r;
}

B3 grow(const B3 &b, const Stencil &st) {
    B3 r;
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = b.lo[d] + st.lo[d];
        r.hi[d] = b.hi[d] + st.hi[d];
    }
    return r;
}

bool has_red(const LoopRec &lp) {
    for (const auto &a : lp.args)
        if (a.kind == TC_ARG_RED) return true;
    return false;
}

// Modelled cycles of one point of a loop on one lane (cost model only).  A
// staged tile reaches its data through generic (flat) addresses, and a
// point's loads cannot move above the previous point's stores, so every
// access costs about its latency: about 60 cycles for a dataset staged in
// LDS, about 500 for one read from device memory (an L2 or Infinity Cache
// hit).  Measured on MI355X with every read-only dataset in device memory:
// a PPCG chain of 63 loops took about 1.6 us per loop per tile, and a 3D
// Euler stage (primitives and five fourth-order right-hand sides) about
// 80 us per 16 x 8 x 8 tile with one workgroup per CU.
double op_cycles(const Ctx &c, const LoopRec &lp, const std::vector<int> &slot_of_arg, int base,
                 const std::vector<char> &staged) {
    double cyc = 20.0;
    if (lp.op == TC_OP_EULER_RHS) cyc = 400.0;
    if (lp.op == TC_OP_EULER_PRIM || lp.op == TC_OP_TEA_K) cyc = 120.0;
    int k = 0;
    for (const auto &a : lp.args) {
        if (a.kind != TC_ARG_DAT) continue;
        const int s = slot_of_arg[base + k++];
        const double n = c.stencils[a.stencil].npoints() + (a.writes() ? 1.0 : 0.0);
        cyc += n * (staged[s] ? 60.0 : 500.0);
    }
    return cyc;
}

// One tile's backward walk.
struct Walk {
    std::vector<B3> C;      // per group loop: computed box
    std::vector<B3> box;    // per slot: LDS box (resident) or read hull (read-only)
    std::vector<B3> load;   // per resident slot: chain-start values needed
};

struct Ana {
    const Ctx &c;
    const std::vector<LoopRec> &chain;
    int g0, g1;
    std::vector<int> slot_of_arg;  // per (loop - g0) * kMaxArgs + dataset argument
    std::vector<int> dats;
    std::vector<char> resident;
    std::vector<B3> wr;  // per slot: hull of writer ranges
    B3 U;

    Ana(const Ctx &cc, const std::vector<LoopRec> &ch, int a, int b) : c(cc), chain(ch), g0(a), g1(b) {}

    void walk(const B3 &O, Walk &w) const {
        const size_t ns = dats.size();
        std::vector<B3> need(ns, none());
        w.box.assign(ns, none());
        w.C.assign(g1 - g0, none());
        for (size_t s = 0; s < ns; ++s)
            if (resident[s]) {
                need[s] = isect(O, wr[s]);
                w.box[s] = need[s];
            }
        for (int l = g1 - 1; l >= g0; --l) {
            const LoopRec &lp = chain[l];
            B3 want = none();
            int k = 0;
            for (const auto &a : lp.args) {
                if (a.kind != TC_ARG_DAT) continue;
                if (a.writes()) want = hull(want, need[slot_of_arg[(l - g0) * kMaxArgs + k]]);
                ++k;
            }
            if (has_red(lp)) want = hull(want, O);
            const B3 C = isect(want, range_of(lp));
            w.C[l - g0] = C;
            if (empty(C)) continue;
            k = 0;
            for (const auto &a : lp.args) {
                if (a.kind != TC_ARG_DAT) continue;
                const int s = slot_of_arg[(l - g0) * kMaxArgs + k++];
                if (!a.writes()) continue;
                if (contains(C, need[s])) need[s] = none();  // every needed point is produced here
                w.box[s] = hull(w.box[s], C);
            }
            k = 0;
            for (const auto &a : lp.args) {
                if (a.kind != TC_ARG_DAT) continue;
                const int s = slot_of_arg[(l - g0) * kMaxArgs + k++];
                if (!a.reads()) continue;
                const B3 g = grow(C, c.stencils[a.stencil]);
                need[s] = hull(need[s], g);
                w.box[s] = hull(w.box[s], g);
            }
        }
        w.load.assign(ns, none());
        for (size_t s = 0; s < ns; ++s)
            if (resident[s]) w.load[s] = need[s];
    }
};

B3 tile_box(const StagedGroup &G, const int t[3]) {
    B3 O;
    for (int d = 0; d < 3; ++d) {
        O.lo[d] = G.ulo[d] + t[d] * G.tile[d];
        O.hi[d] = std::min(O.lo[d] + G.tile[d], G.uhi[d]);
    }
    return O;
}

// Sizes the LDS boxes from the walks of `tiles`, decides which datasets the
// group only reads are staged in LDS too (the most accessed first, while
// they fit), and fills the cost model; false if the written datasets do
// not fit.
bool layout(const Ctx &c, const Ana &A, StagedGroup &G, const std::vector<std::array<int, 3>> &tiles,
            std::vector<Walk> &walks) {
    const size_t ns = A.dats.size();
    const int L = A.g1 - A.g0;
    const int es = G.dtype == TC_F64 ? 8 : 4;
    std::vector<int> dim(3 * ns, 0);
    std::vector<char> twin(ns, 0);
    walks.resize(tiles.size());
    G.computed.assign(L, 0);
    for (size_t i = 0; i < tiles.size(); ++i) {
        const B3 O = tile_box(G, tiles[i].data());
        Walk &w = walks[i];
        A.walk(O, w);
        for (int l = 0; l < L; ++l)
            if (vol(w.C[l]) > 0) G.computed[l] = 1;
        for (size_t s = 0; s < ns; ++s) {
            for (int d = 0; d < 3; ++d)
                if (!empty(w.box[s])) dim[3 * s + d] = std::max(dim[3 * s + d], w.box[s].hi[d] - w.box[s].lo[d]);
            if (A.resident[s] && !contains(isect(O, A.wr[s]), w.load[s])) twin[s] = 1;
        }
    }
    auto elems = [&](size_t s) {
        return ((int64_t)std::max(1, dim[3 * s]) * std::max(1, dim[3 * s + 1]) * std::max(1, dim[3 * s + 2]) + 3) / 4 * 4;
    };
    // written datasets are always staged; read-only ones by access count
    std::vector<char> staged(ns, 0);
    int64_t used = 0;
    for (size_t s = 0; s < ns; ++s)
        if (A.resident[s]) {
            staged[s] = 1;
            used += elems(s);
        }
    if ((used * es + 15) / 16 * 16 + (int64_t)sizeof(LoopDesc) > kSLdsBudget) return false;
    {
        std::vector<std::pair<int, size_t>> order;
        std::vector<int> count(ns, 0);
        for (int l = A.g0; l < A.g1; ++l) {
            int k = 0;
            for (const auto &a : A.chain[l].args)
                if (a.kind == TC_ARG_DAT) count[A.slot_of_arg[(l - A.g0) * kMaxArgs + k++]] += c.stencils[a.stencil].npoints();
        }
        for (size_t s = 0; s < ns; ++s)
            if (!A.resident[s]) order.push_back({-count[s], s});
        std::sort(order.begin(), order.end());
        for (const auto &o : order)
            if ((((used + elems(o.second)) * es + 15) / 16 * 16) + (int64_t)sizeof(LoopDesc) <= kSLdsBudget) {
                staged[o.second] = 1;
                used += elems(o.second);
            }
    }
    double cyc_sum = 0.0, bytes_sum = 0.0;
    for (size_t i = 0; i < tiles.size(); ++i) {
        const B3 O = tile_box(G, tiles[i].data());
        const Walk &w = walks[i];
        double cyc = 0.0, bytes = 0.0;
        for (int l = 0; l < L; ++l) {
            const int64_t n = vol(w.C[l]);
            if (n == 0) continue;
            cyc += (double)((n + kSThreads - 1) / kSThreads) *
                       op_cycles(c, A.chain[A.g0 + l], A.slot_of_arg, l * kMaxArgs, staged) + 1500.0;
        }
        for (size_t s = 0; s < ns; ++s) {
            const double moved = A.resident[s] ? (double)(vol(w.load[s]) + vol(isect(O, A.wr[s]))) : (double)vol(w.box[s]);
            bytes += moved * es;
            // staging and write-back: rounds of eight loads in flight per
            // lane, each about a device-memory latency
            if (staged[s]) cyc += std::ceil(moved / (kSThreads * 8.0)) * 2000.0;
        }
        cyc_sum += cyc;
        bytes_sum += bytes;
    }
    int64_t off = 0;
    G.slots.assign(ns, SSlot());
    for (size_t s = 0; s < ns; ++s) {
        SSlot &S = G.slots[s];
        std::memset(&S, 0, sizeof S);
        S.resident = A.resident[s];
        S.staged = staged[s];
        for (int d = 0; d < 3; ++d) {
            S.wlo[d] = A.wr[s].lo[d];
            S.whi[d] = A.wr[s].hi[d];
        }
        if (!S.staged) continue;
        S.twin = twin[s];
        const int64_t bx = std::max(1, dim[3 * s]), by = std::max(1, dim[3 * s + 1]);
        S.lds_off = off;
        S.lsy = bx;
        S.lsz = bx * by;
        off += elems(s);
    }
    G.lds_bytes = off * es;
    G.desc_off = (G.lds_bytes + 15) / 16 * 16;
    // latency-bound tiles: rounds of one tile per CU; a second resident
    // workgroup per CU (if LDS allows) overlaps about half of the latency
    const double per_tile = cyc_sum / (double)tiles.size();
    const double lds = (double)(G.desc_off + sizeof(LoopDesc) + 1024);
    const double wg_per_cu = std::max(1.0, std::min(4.0, std::floor(160.0 * 1024.0 / lds)));
    const double per_cu = std::max(1.0, (double)G.ntot / 256.0);
    const double overlap = std::min(per_cu, std::min(wg_per_cu, 2.0));
    // calibration: measured staged launches took 2.4x (PPCG 256^2, 153 tiles)
    // to 3.6x (PPCG 2000^2, 2016 tiles) the cycles modelled above
    const double t_lat = 3.0 * per_cu * per_tile / ((1.0 + 0.5 * (overlap - 1.0)) * 2.4e9);
    const double t_bw = (double)G.ntot * (bytes_sum / (double)tiles.size()) / 4.0e12;
    G.cost = std::max(t_lat, t_bw) + 5e-6;
    // workgroup size: 256 threads unless asked otherwise.  On the PPCG chain
    // 256 ran faster than 1024 at both measured sizes (256^2, boxes up to
    // 52 x 36: 9.8 against 10.2 ms per solve; 700^2, boxes up to 84 x 52:
    // 14.7 against 15.2 ms); the cost above was calibrated at 1024.
    G.threads = c.staged_threads > 0 ? c.staged_threads : 256;
    return true;
}

}  // namespace

bool staged_analyse(const Ctx &c, const std::vector<LoopRec> &chain, int g0, int g1, const int tile_req[3], bool full,
                    StagedGroup &G) {
    G = StagedGroup();
    G.g0 = g0;
    G.g1 = g1;
    if (g1 - g0 < 2 || g1 - g0 > kSMaxLoops) return false;
    const LoopRec &f = chain[g0];
    G.ndim = f.ndim;
    Ana A(c, chain, g0, g1);
    A.slot_of_arg.assign((size_t)(g1 - g0) * kMaxArgs, -1);
    A.U = none();
    int dtype = -1, nprm = 0;
    for (int l = g0; l < g1; ++l) {
        const LoopRec &lp = chain[l];
        if (lp.block != f.block || lp.ndim != f.ndim) return false;
        A.U = hull(A.U, range_of(lp));
        int k = 0;
        for (const auto &a : lp.args) {
            if (a.kind != TC_ARG_DAT) continue;
            const int dt = c.dats[a.handle].dtype;
            if (dtype < 0) dtype = dt;
            if (dt != dtype) return false;
            auto it = std::find(A.dats.begin(), A.dats.end(), a.handle);
            int s = (int)(it - A.dats.begin());
            if (it == A.dats.end()) {
                A.dats.push_back(a.handle);
                A.resident.push_back(0);
                A.wr.push_back(none());
            }
            if (a.writes()) {
                A.resident[s] = 1;
                A.wr[s] = hull(A.wr[s], range_of(lp));
            }
            A.slot_of_arg[(l - g0) * kMaxArgs + k++] = s;
        }
        LoopDesc d;
        build_desc(c, lp, d);
        nprm += lp.op == TC_OP_WSUM ? d.pt0[d.nargs - 1] + d.npts[d.nargs - 1] : (int)lp.params.size();
    }
    if (dtype < 0 || empty(A.U) || (int)A.dats.size() > kSMaxDat || nprm > kSMaxPrm) return false;
    G.dtype = dtype;
    G.dats = A.dats;
    G.nprm = nprm;
    for (int d = 0; d < 3; ++d) {
        G.ulo[d] = A.U.lo[d];
        G.uhi[d] = A.U.hi[d];
    }

    // tile shapes to try: the requested one, else a list per dimension
    std::vector<std::array<int, 3>> shapes;
    if (tile_req && tile_req[0] > 0) {
        shapes.push_back({tile_req[0], G.ndim > 1 ? std::max(1, tile_req[1]) : 1, G.ndim > 2 ? std::max(1, tile_req[2]) : 1});
    } else if (!full) {
        // the split search models every candidate run with one default shape;
        // the shape is chosen for the runs that become groups
        shapes.push_back(G.ndim == 1 ? std::array<int, 3>{512, 1, 1}
                                     : (G.ndim == 2 ? std::array<int, 3>{32, 16, 1} : std::array<int, 3>{16, 8, 8}));
    } else if (G.ndim == 1) {
        shapes = {{1024, 1, 1}, {512, 1, 1}, {256, 1, 1}, {128, 1, 1}};
    } else if (G.ndim == 2) {
        shapes = {{64, 32, 1}, {32, 32, 1}, {64, 16, 1}, {32, 16, 1}, {16, 16, 1}, {16, 8, 1}, {8, 8, 1}};
    } else {
        shapes = {{32, 8, 8}, {16, 8, 8}, {16, 16, 4}, {8, 8, 8}, {16, 8, 4}, {8, 8, 4}, {8, 4, 4}};
    }
    auto tiles_of = [&](bool all) {
        std::vector<std::array<int, 3>> ts;
        std::vector<int> idx[3];
        for (int d = 0; d < 3; ++d) {
            const int n = G.nt[d];
            if (all) {
                for (int t = 0; t < n; ++t) idx[d].push_back(t);
            } else {
                for (int t : {0, n / 2, n - 1})
                    if (t >= 0 && t < n && std::find(idx[d].begin(), idx[d].end(), t) == idx[d].end())
                        idx[d].push_back(t);
            }
        }
        for (int z : idx[2])
            for (int y : idx[1])
                for (int x : idx[0]) ts.push_back({x, y, z});
        return ts;
    };
    double best = 1e300;
    std::array<int, 3> pick{0, 0, 0};
    for (const auto &sh : shapes) {
        StagedGroup T = G;
        for (int d = 0; d < 3; ++d) {
            T.tile[d] = d < G.ndim ? std::max(1, sh[d]) : 1;
            const int ext = A.U.hi[d] - A.U.lo[d];
            T.nt[d] = (ext + T.tile[d] - 1) / T.tile[d];
        }
        T.ntot = T.nt[0] * T.nt[1] * T.nt[2];
        std::vector<Walk> w;
        G.nt[0] = T.nt[0];
        G.nt[1] = T.nt[1];
        G.nt[2] = T.nt[2];
        if (!layout(c, A, T, tiles_of(false), w)) continue;
        if (T.cost < best) {
            best = T.cost;
            pick = sh;
        }
    }
    if (best >= 1e299) return false;
    for (int d = 0; d < 3; ++d) {
        G.tile[d] = d < G.ndim ? std::max(1, pick[d]) : 1;
        G.nt[d] = (A.U.hi[d] - A.U.lo[d] + G.tile[d] - 1) / G.tile[d];
    }
    G.ntot = G.nt[0] * G.nt[1] * G.nt[2];
    std::vector<Walk> walks;
    const auto tiles = tiles_of(full);
    if (!layout(c, A, G, tiles, walks)) return false;

    // per-loop extents of the most interior tile walked
    {
        size_t mid = 0;
        int bestd = -1;
        for (size_t i = 0; i < tiles.size(); ++i) {
            int dmin = INT_MAX;
            for (int d = 0; d < G.ndim; ++d) dmin = std::min(dmin, std::min(tiles[i][d], G.nt[d] - 1 - tiles[i][d]));
            if (dmin > bestd) {
                bestd = dmin;
                mid = i;
            }
        }
        const B3 O = tile_box(G, tiles[mid].data());
        G.ext.assign(g1 - g0, {-1, -1, -1, -1, -1, -1});
        for (int l = 0; l < g1 - g0; ++l) {
            const B3 &C = walks[mid].C[l];
            if (empty(C)) continue;
            for (int d = 0; d < 3; ++d) {
                G.ext[l][2 * d] = O.lo[d] - C.lo[d];
                G.ext[l][2 * d + 1] = C.hi[d] - O.hi[d];
            }
        }
    }
    // modelled algorithmic bytes: chain-start values of written datasets
    // over their write regions, read-only datasets over the union range, and
    // the write-backs
    {
        const int es = G.dtype == TC_F64 ? 8 : 4;
        int64_t b = 0;
        for (size_t s = 0; s < A.dats.size(); ++s) b += vol(A.resident[s] ? A.wr[s] : A.U) * es;
        for (size_t s = 0; s < A.dats.size(); ++s)
            if (A.resident[s]) b += vol(A.wr[s]) * es;
        G.alg_bytes = b;
    }

    // loops: slots and parameter layout
    G.loops.assign(g1 - g0, SLoop());
    int po = 0;
    G.nred_loops = 0;
    for (int l = g0; l < g1; ++l) {
        SLoop &S = G.loops[l - g0];
        std::memset(&S, 0, sizeof S);
        for (int k = 0; k < kMaxArgs; ++k) S.slot[k] = A.slot_of_arg[(l - g0) * kMaxArgs + k];
        LoopDesc d;
        build_desc(c, chain[l], d);
        S.prm_off = po;
        S.nprm = chain[l].op == TC_OP_WSUM ? d.pt0[d.nargs - 1] + d.npts[d.nargs - 1] : (int)chain[l].params.size();
        S.prm_skip = chain[l].op == TC_OP_WSUM ? d.npts[0] : 0;
        S.all_lds = 1;
        for (int a = 0; a < d.nargs; ++a) S.all_lds = S.all_lds && G.slots[S.slot[a]].staged;
        po += S.nprm;
        if (has_red(chain[l])) ++G.nred_loops;
    }

    if (full) {
        const size_t ns = A.dats.size();
        const int L = g1 - g0;
        G.rec = 6 + 9 * (int)ns + 6 * L;
        G.table.assign((size_t)G.ntot * G.rec, 0);
        for (size_t i = 0; i < tiles.size(); ++i) {
            const auto &t = tiles[i];
            const int64_t ti = t[0] + (int64_t)G.nt[0] * (t[1] + (int64_t)G.nt[1] * t[2]);
            int *r = &G.table[(size_t)ti * G.rec];
            const B3 O = tile_box(G, t.data());
            const Walk &w = walks[i];
            for (int d = 0; d < 3; ++d) {
                r[d] = O.lo[d];
                r[3 + d] = O.hi[d];
            }
            for (size_t s = 0; s < ns; ++s) {
                int *q = r + 6 + 9 * s;
                const B3 b = empty(w.box[s]) ? O : w.box[s];
                const B3 ld = A.resident[s] ? w.load[s] : (G.slots[s].staged ? w.box[s] : none());
                for (int d = 0; d < 3; ++d) {
                    q[d] = b.lo[d];
                    q[3 + d] = empty(ld) ? 0 : ld.lo[d];
                    q[6 + d] = empty(ld) ? 0 : ld.hi[d];
                }
            }
            for (int l = 0; l < L; ++l) {
                int *q = r + 6 + 9 * ns + 6 * l;
                const B3 &C = w.C[l];
                for (int d = 0; d < 3; ++d) {
                    q[d] = empty(C) ? 0 : C.lo[d];
                    q[3 + d] = empty(C) ? 0 : C.hi[d];
                }
            }
        }
    }
    return true;
}

tc_status staged_upload(Ctx &c, const std::vector<LoopRec> &chain, StagedGroup &G) {
    const int L = G.g1 - G.g0;
    std::vector<LoopDesc> descs(L);
    for (int l = 0; l < L; ++l) {
        LoopDesc &d = descs[l];
        build_desc(c, chain[G.g0 + l], d);
        // staged arguments address the LDS box with its own strides
        for (int a = 0; a < d.nargs; ++a) {
            const int s = G.loops[l].slot[a];
            const Stencil *st = nullptr;
            int k = 0;
            for (const auto &x : chain[G.g0 + l].args)
                if (x.kind == TC_ARG_DAT && k++ == a) st = &c.stencils[x.stencil];
            d.arg[a].ptr = nullptr;
            if (!G.slots[s].staged) continue;
            d.arg[a].sy = G.slots[s].lsy;
            d.arg[a].sz = G.slots[s].lsz;
            for (int p = 0; p < d.npts[a]; ++p)
                d.off[d.pt0[a] + p] = (int64_t)st->pts[3 * p] + (int64_t)st->pts[3 * p + 1] * G.slots[s].lsy +
                                      (int64_t)st->pts[3 * p + 2] * G.slots[s].lsz;
        }
        std::memset(d.prm, 0, sizeof d.prm);
        d.partials[0] = d.partials[1] = nullptr;
    }
    const size_t b_desc = sizeof(LoopDesc) * L, b_loops = sizeof(SLoop) * L, b_slots = sizeof(SSlot) * G.slots.size();
    G.off_loops = (int64_t)b_desc;
    G.off_slots = G.off_loops + (int64_t)((b_loops + 15) / 16 * 16);
    G.off_table = G.off_slots + (int64_t)((b_slots + 15) / 16 * 16);
    const size_t total = (size_t)G.off_table + G.table.size() * sizeof(int);
    std::vector<unsigned char> host(total, 0);
    std::memcpy(host.data(), descs.data(), b_desc);
    std::memcpy(host.data() + G.off_loops, G.loops.data(), b_loops);
    std::memcpy(host.data() + G.off_slots, G.slots.data(), b_slots);
    if (!G.table.empty()) std::memcpy(host.data() + G.off_table, G.table.data(), G.table.size() * sizeof(int));
    if (c.host_only) return TC_OK;
    if (c.noalloc)
        return fail(c, TC_ERR_STATE, "staged group [%d,%d) has no device tables yet; flush it once with tc_flush first",
                    G.g0, G.g1);
    void *p = dev_alloc(c, total);
    if (!p) return fail(c, TC_ERR_NOMEM, "cannot allocate the tables of staged group [%d,%d)", G.g0, G.g1);
    c.staged_allocs.push_back(p);
    if (hipMemcpy(p, host.data(), total, hipMemcpyHostToDevice) != hipSuccess)
        return fail(c, TC_ERR_DEVICE, "hipMemcpy of staged group tables failed");
    G.dev = p;
    G.dev_bytes = total;
    return TC_OK;
}

tc_status staged_check_noalloc(Ctx &c, const StagedGroup &G) {
    if (!G.dev) return fail(c, TC_ERR_STATE, "staged group [%d,%d) has no device tables yet", G.g0, G.g1);
    for (size_t s = 0; s < G.slots.size(); ++s)
        if (G.slots[s].twin && (!c.dats[G.dats[s]].raw[0] || !c.dats[G.dats[s]].raw[1]))
            return fail(c, TC_ERR_STATE,
                        "the second buffer of %s does not exist yet and a call that allocates nothing cannot create "
                        "it; flush this chain once with tc_flush first", c.dats[G.dats[s]].name.c_str());
    return TC_OK;
}

tc_status staged_run(Ctx &c, const std::vector<LoopRec> &chain, StagedGroup &G) {
    if (!G.dev) return fail(c, TC_ERR_STATE, "staged group [%d,%d) is not uploaded", G.g0, G.g1);
    SArgs a;
    std::memset(&a, 0, sizeof a);
    const unsigned char *base = (const unsigned char *)G.dev;
    a.loops = (const LoopDesc *)base;
    a.sl = (const SLoop *)(base + G.off_loops);
    a.slots = (const SSlot *)(base + G.off_slots);
    a.table = (const int *)(base + G.off_table);
    a.partials = c.partials;
    a.nloops = G.g1 - G.g0;
    a.nslots = (int)G.slots.size();
    a.rec = G.rec;
    a.ntot = G.ntot;
    a.desc_off = G.desc_off;
    for (size_t s = 0; s < G.slots.size(); ++s) {
        Dataset &ds = c.dats[G.dats[s]];
        a.src[s] = ds.origin(ds.cur);
        a.gsy[s] = ds.sy();
        a.gsz[s] = ds.sz();
        a.dst[s] = a.src[s];
        if (!G.slots[s].twin) continue;
        const int tw = 1 - ds.cur;
        if (!ds.raw[tw]) {
            if (c.noalloc)
                return fail(c, TC_ERR_STATE, "the second buffer of %s does not exist yet", ds.name.c_str());
            ds.raw[tw] = dev_alloc(c, (size_t)(ds.bytes + ds.stagger));
            if (!ds.raw[tw]) return fail(c, TC_ERR_NOMEM, "cannot allocate the second buffer of %s", ds.name.c_str());
            ds.buf[tw] = (char *)ds.raw[tw] + ds.stagger;
            ds.twin_synced = false;
        }
        // outside the group's write region of this dataset the second buffer
        // must equal the current one; it does outside the hull of earlier writes
        const SSlot &S = G.slots[s];
        bool inside = true;
        if (ds.ever_written)
            for (int d = 0; d < 3; ++d) inside = inside && ds.wlo[d] >= S.wlo[d] && ds.whi[d] <= S.whi[d];
        if (!ds.twin_synced || !inside) {
            if (hipMemcpyAsync(ds.buf[tw], ds.buf[ds.cur], (size_t)ds.bytes, hipMemcpyDeviceToDevice, c.stream) !=
                hipSuccess)
                return fail(c, TC_ERR_DEVICE, "hipMemcpyAsync (second buffer) failed");
            ds.twin_synced = true;
        }
        a.dst[s] = ds.origin(tw);
    }
    // this flush's parameters in each loop's descriptor layout (a weighted
    // sum's weights follow its output stencil points, as build_desc places them)
    for (int l = G.g0; l < G.g1; ++l) {
        const SLoop &S = G.loops[l - G.g0];
        const std::vector<double> &p = chain[l].params;
        for (size_t i = 0; i < p.size() && S.prm_skip + (int)i < S.nprm; ++i) a.prm[S.prm_off + S.prm_skip + i] = p[i];
    }
    const hipError_t e = launch_staged(a, G.dtype, (size_t)G.desc_off + sizeof(LoopDesc), G.threads, c.stream);
    if (e != hipSuccess) return fail(c, TC_ERR_DEVICE, "staged group launch failed: %s", hipGetErrorString(e));
    for (size_t s = 0; s < G.slots.size(); ++s)
        if (G.slots[s].twin) {
            Dataset &ds = c.dats[G.dats[s]];
            ds.cur = 1 - ds.cur;
        }
    return TC_OK;
}

}  // namespace tc
