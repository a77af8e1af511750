// Skewed tiling plan (Algorithm 1 of Section 4.2) and the chain-structure key
// used by the plan cache (Section 4.2: a plan is cached and reused when the
// same sequence of loops is encountered again).
//
// Readings of the printed algorithm used here (all per dimension d, ranges
// half-open):
//   * start of tile t = end of tile t-1 for the same loop (first tile: the
//     loop's start);
//   * end: the last tile takes the loop's end; otherwise the largest of the
//     read-after-write bound (what later loops of the tile read from datasets
//     this loop writes) and the write-after-read/write bound (what later loops
//     of the tile wrote, minus this loop's most negative stencil offset),
//     clipped to the loop's end; with neither, the default
//     union_start + (t+1) * tilesize clipped to the loop's end;
//   * one pass over the tiles in increasing order computes start, both
//     bounds, the default and the dependency updates of a tile;
//   * an end below its start is raised to the start (empty tile);
//   * dependencies are per dataset, per dimension and per tile index along
//     that dimension, and only grow.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>

#include "tc_internal.hpp"

namespace tc {

namespace {
constexpr int64_t kNegInf = INT64_MIN / 4;
constexpr int64_t kPosInf = INT64_MAX / 4;

// Choose a tile size per dimension when the caller left it at <= 0: every
// dimension but the slowest is left whole (long contiguous rows, as the
// paper's best tiles were much wider in x than in y); the slowest dimension
// gets the number of slices whose working set (all datasets the chain
// touches) fills about half of the 256 MB Infinity Cache.
void auto_tile(const Ctx &c, const std::vector<LoopRec> &chain, int ndim, const int64_t *ustart,
               const int64_t *uend, const int tile_in[3], int64_t ts[3]) {
    std::vector<char> used(c.dats.size(), 0);
    for (const auto &lp : chain)
        for (const auto &a : lp.args)
            if (a.kind == TC_ARG_DAT) used[a.handle] = 1;
    int64_t bytes_per_slice = 0;
    int slow = ndim - 1;
    for (size_t i = 0; i < c.dats.size(); ++i) {
        if (!used[i]) continue;
        const Dataset &d = c.dats[i];
        int64_t b = (int64_t)d.esize();
        for (int k = 0; k < ndim; ++k)
            if (k != slow) b *= (k == 0 ? d.pitch : (int64_t)d.size[k] + d.hneg[k] + d.hpos[k]);
        bytes_per_slice += b;
    }
    const int64_t budget = 128ll << 20;
    for (int d = 0; d < ndim; ++d) {
        int64_t extent = std::max<int64_t>(uend[d] - ustart[d], 1);
        if (tile_in[d] > 0) {
            ts[d] = tile_in[d];
        } else if (d == slow && ndim > 1 && bytes_per_slice > 0) {
            ts[d] = std::max<int64_t>(8, std::min<int64_t>(extent, budget / bytes_per_slice));
        } else {
            ts[d] = extent;
        }
    }
}
}  // namespace

SkewedPlan build_skewed_plan(const Ctx &c, const std::vector<LoopRec> &chain, const int tile[3]) {
    SkewedPlan P;
    const int L = (int)chain.size();
    const int D = L ? chain[0].ndim : 1;
    P.ndim = D;
    P.nloops = L;
    if (L == 0) return P;

    // union of the iteration ranges and the number of tiles per dimension
    int64_t us[3], ue[3], ts[3];
    for (int d = 0; d < D; ++d) {
        us[d] = kPosInf;
        ue[d] = kNegInf;
        for (const auto &lp : chain) {
            us[d] = std::min<int64_t>(us[d], lp.lo[d]);
            ue[d] = std::max<int64_t>(ue[d], lp.hi[d]);
        }
    }
    auto_tile(c, chain, D, us, ue, tile, ts);
    for (int d = 0; d < D; ++d) {
        int64_t ext = ue[d] - us[d];
        P.num_tiles[d] = (int)std::max<int64_t>(1, (ext - 1) / ts[d] + 1);
        P.start[d].assign((size_t)P.num_tiles[d] * L, 0);
        P.end[d].assign((size_t)P.num_tiles[d] * L, 0);
    }

    // dependency tables: [dataset][tile] -> (start, end), one per dimension
    const size_t ND = c.dats.size();
    for (int d = 0; d < D; ++d) {
        const int T = P.num_tiles[d];
        std::vector<int64_t> rdS(ND * T, kPosInf), rdE(ND * T, kNegInf);
        std::vector<int64_t> wdS(ND * T, kPosInf), wdE(ND * T, kNegInf);
        for (int l = L - 1; l >= 0; --l) {
            const LoopRec &lp = chain[l];
            for (int t = 0; t < T; ++t) {
                const int64_t s = (t == 0) ? lp.lo[d] : P.end[d][(size_t)(t - 1) * L + l];
                int64_t e = kNegInf;
                if (t == T - 1) {
                    e = lp.hi[d];
                } else {
                    for (const auto &a : lp.args) {  // read after write
                        if (!a.writes()) continue;
                        e = std::min<int64_t>(lp.hi[d], std::max(e, rdE[(size_t)a.handle * T + t]));
                    }
                    for (const auto &a : lp.args) {  // write after read / write
                        if (a.kind != TC_ARG_DAT) continue;
                        const int64_t m = c.stencils[a.stencil].lo[d];
                        const int64_t w = wdE[(size_t)a.handle * T + t];
                        if (w > kNegInf) e = std::min<int64_t>(lp.hi[d], std::max(e, w - m));
                    }
                }
                if (e == kNegInf) e = std::min<int64_t>(lp.hi[d], us[d] + (int64_t)(t + 1) * ts[d]);
                if (e < s) e = s;
                P.start[d][(size_t)t * L + l] = (int)s;
                P.end[d][(size_t)t * L + l] = (int)e;
                for (const auto &a : lp.args) {
                    if (!a.reads()) continue;
                    const Stencil &st = c.stencils[a.stencil];
                    size_t k = (size_t)a.handle * T + t;
                    rdE[k] = std::max(rdE[k], e + st.hi[d]);
                    rdS[k] = std::min(rdS[k], s + st.lo[d]);
                }
                for (const auto &a : lp.args) {
                    if (!a.writes()) continue;
                    size_t k = (size_t)a.handle * T + t;
                    wdE[k] = std::max(wdE[k], e);
                    wdS[k] = std::min(wdS[k], s);
                }
            }
        }
    }
    return P;
}

// FNV-1a over the structure of the chain: ops, blocks, ranges, dataset ids,
// stencil ids, access modes, reduction ids and the tiling request.  Scalar
// parameters are not part of the key.
uint64_t chain_key(const Ctx &c, const std::vector<LoopRec> &chain, int mode, const int tile[3], int cpl) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (uint64_t)((v >> (8 * i)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    mix(mode);
    for (int d = 0; d < 3; ++d) mix(tile[d]);
    mix(mode == TC_TILING_FUSED ? cpl : 0);
    mix((int64_t)chain.size());
    for (const auto &lp : chain) {
        mix(lp.op);
        mix(lp.block);
        mix((int64_t)lp.params.size());
        for (int d = 0; d < 3; ++d) {
            mix(lp.lo[d]);
            mix(lp.hi[d]);
        }
        mix((int64_t)lp.args.size());
        for (const auto &a : lp.args) {
            mix(a.kind);
            mix(a.handle);
            mix(a.kind == TC_ARG_DAT ? a.stencil : -1);
            mix(a.kind == TC_ARG_DAT ? a.access : -1);
        }
    }
    (void)c;
    return h;
}

}  // namespace tc
