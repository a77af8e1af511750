// Fusion-group analysis (host) and per-flush launch of fused groups.
//
// Dependency analysis follows the overlapped tiling of Section 4.4: a tile
// extends each loop's range by what the later loops of the tile read from its
// output (read dependencies only; the tiles run concurrently), so the first
// loops of a group compute a halo around the owned block that shrinks loop by
// loop.  Along the streamed dimension the same extents become lags: a loop
// runs behind the loops it reads from by their read extent plus one step, and
// a loop that overwrites a dataset runs behind the earlier readers of the old
// values (the write-after-read rule of Algorithm 1 in streaming form).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>

#include "fused.hpp"

namespace tc {

namespace {

struct Ext {
    int xlo = INT_MIN, xhi = INT_MIN, ylo = INT_MIN, yhi = INT_MIN;  // INT_MIN: not read
    void add(int a, int b, int c, int d) {
        xlo = std::max(xlo, a);
        xhi = std::max(xhi, b);
        ylo = std::max(ylo, c);
        yhi = std::max(yhi, d);
    }
    bool set() const { return xlo != INT_MIN; }
};

bool fusable(const Ctx &c, const LoopRec &lp) {
    if (lp.op != TC_OP_WSUM || lp.ndim != 2) return false;
    if (lp.args.size() > 1 + kFMaxIn) return false;
    for (const auto &a : lp.args)
        if (a.kind != TC_ARG_DAT) return false;
    // stencil reach within what a signed byte and the ring width allow
    for (const auto &a : lp.args) {
        const Stencil &st = c.stencils[a.stencil];
        if (st.lo[0] < -8 || st.hi[0] > 8 || st.lo[1] < -8 || st.hi[1] > 8) return false;
    }
    return true;
}

// Analyse loops [g0, g1); returns false if they cannot form one group.
bool analyse(const Ctx &c, const std::vector<LoopRec> &chain, int g0, int g1, const int tile[3], int lds_budget,
             FusedGroup &G) {
    const int n = g1 - g0;
    if (n < 1 || n > kFMaxLoops) return false;
    const int dtype = c.dats[chain[g0].args[0].handle].dtype;
    const int es = dtype == TC_F64 ? 8 : 4;
    std::map<int, int> ring_of;
    std::vector<int> ring_dat;
    int nent = 0, nin = 0;
    for (int l = g0; l < g1; ++l) {
        const LoopRec &lp = chain[l];
        if (!fusable(c, lp) || lp.block != chain[g0].block) return false;
        for (const auto &a : lp.args) {
            if (c.dats[a.handle].dtype != dtype) return false;
            if (!ring_of.count(a.handle)) {
                ring_of[a.handle] = (int)ring_dat.size();
                ring_dat.push_back(a.handle);
            }
            if (a.access == TC_READ) {
                nent += c.stencils[a.stencil].npoints();
                ++nin;
            }
        }
    }
    const int nr = (int)ring_dat.size();
    if (nr > kFMaxRings || nent > kFMaxEnt || nin > kFMaxLoops * 8) return false;

    FGroupD &D = G.tmpl;
    std::memset(&D, 0, sizeof D);
    D.nloops = n;
    D.nrings = nr;

    // backward pass: extents each loop must compute beyond the owned block
    std::vector<Ext> need(nr);
    std::vector<int> hlo(n), hhi(n), vlo(n), vhi(n);
    for (int i = n - 1; i >= 0; --i) {
        const LoopRec &lp = chain[g0 + i];
        const int o = ring_of[lp.args[0].handle];
        const Ext &e = need[o];
        hlo[i] = e.set() ? std::max(0, e.xlo) : 0;
        hhi[i] = e.set() ? std::max(0, e.xhi) : 0;
        vlo[i] = e.set() ? std::max(0, e.ylo) : 0;
        vhi[i] = e.set() ? std::max(0, e.yhi) : 0;
        for (size_t a = 1; a < lp.args.size(); ++a) {
            const Stencil &st = c.stencils[lp.args[a].stencil];
            need[ring_of[lp.args[a].handle]].add(hlo[i] - st.lo[0], hhi[i] + st.hi[0], vlo[i] - st.lo[1],
                                                 vhi[i] + st.hi[1]);
        }
    }
    int HR = 0;
    for (int i = 0; i < n; ++i) {
        HR = std::max({HR, hlo[i], hhi[i]});
        const LoopRec &lp = chain[g0 + i];
        for (size_t a = 1; a < lp.args.size(); ++a) {
            const Stencil &st = c.stencils[lp.args[a].stencil];
            HR = std::max({HR, hlo[i] - st.lo[0], hhi[i] + st.hi[0]});
        }
    }
    const int W = kFCols - 2 * HR;
    if (W < 32) return false;

    // forward pass: lags (rows)
    const int R = G.rows;
    std::vector<int> lag(n, 0);
    std::vector<int> lastw(nr, -1);
    std::vector<std::vector<std::pair<int, int>>> readers(nr);  // (lag, dymin) of every earlier reader
    std::vector<int> live_lag(nr, INT_MAX);   // min over live-in readers of lag - dymax
    std::vector<int> bot(nr, INT_MIN);        // max over readers of lag - dymin
    std::vector<int> wmin(nr, INT_MAX), wmax(nr, INT_MIN);
    std::vector<int> first_write(nr, -1);     // loop (group index) whose WRITE is the ring's first access
    std::vector<char> accessed(nr, 0);
    std::vector<int> ld_below(nr, 0), ld_above(nr, 0);
    for (int i = 0; i < n; ++i) {
        const LoopRec &lp = chain[g0 + i];
        int lam = 0;
        for (size_t a = 1; a < lp.args.size(); ++a) {
            const int r = ring_of[lp.args[a].handle];
            const Stencil &st = c.stencils[lp.args[a].stencil];
            if (lastw[r] >= 0) lam = std::max(lam, lag[lastw[r]] + st.hi[1] + R);
        }
        const int o = ring_of[lp.args[0].handle];
        for (auto &pr : readers[o]) lam = std::max(lam, pr.first - pr.second + R);
        if (lastw[o] >= 0) lam = std::max(lam, lag[lastw[o]] + R);
        lag[i] = lam;
        for (size_t a = 1; a < lp.args.size(); ++a) {
            const int r = ring_of[lp.args[a].handle];
            const Stencil &st = c.stencils[lp.args[a].stencil];
            readers[r].push_back({lam, st.lo[1]});
            if (lastw[r] < 0) live_lag[r] = std::min(live_lag[r], lam - st.hi[1]);
            bot[r] = std::max(bot[r], lam - st.lo[1]);
            ld_below[r] = std::max(ld_below[r], vlo[i] - st.lo[1]);
            ld_above[r] = std::max(ld_above[r], vhi[i] + st.hi[1]);
            accessed[r] = 1;
        }
        if (!accessed[o]) first_write[o] = i;
        accessed[o] = 1;
        lastw[o] = i;
        wmin[o] = std::min(wmin[o], lam);
        wmax[o] = std::max(wmax[o], lam);
        ld_below[o] = std::max(ld_below[o], vlo[i]);
        ld_above[o] = std::max(ld_above[o], vhi[i]);
    }

    // rings: loader, storer, depth, LDS offsets
    int lds = 0;
    G.ring_dat = ring_dat;
    G.ring_store.assign(nr, 0);
    for (int r = 0; r < nr; ++r) {
        FRingD &rd = D.rings[r];
        const Dataset &ds = c.dats[ring_dat[r]];
        const bool written = wmin[r] != INT_MAX;
        const bool live = live_lag[r] != INT_MAX;
        rd.load = live ? 1 : (written ? 2 : 0);
        rd.store = written ? 1 : 0;
        G.ring_store[r] = rd.store;
        int top = INT_MAX, bottom = INT_MIN;
        if (rd.load) {
            int l = INT_MAX;
            if (live) l = live_lag[r] - R;
            if (written) l = std::min(l, wmin[r] - R);
            rd.load_lag = l;
            top = std::min(top, rd.load_lag);
        }
        if (written) {
            top = std::min(top, wmin[r]);
            rd.store_lag = wmax[r] + R;
            bottom = std::max(bottom, rd.store_lag);
        }
        if (bot[r] != INT_MIN) bottom = std::max(bottom, bot[r]);
        if (top == INT_MAX || bottom == INT_MIN) {
            top = 0;
            bottom = 0;
        }
        rd.depth = bottom - top + R;
        rd.inv_depth = 1.0f / (float)rd.depth;
        rd.lds_off = lds / es;
        lds += rd.depth * kFCols * es;
        rd.ld_below = ld_below[r];
        rd.ld_above = ld_above[r];
        rd.sy = ds.sy();
        rd.ext_xlo = -ds.hneg[0];
        rd.ext_xhi = ds.size[0] + ds.hpos[0];
        rd.ext_ylo = -ds.hneg[1];
        rd.ext_yhi = ds.size[1] + ds.hpos[1];
        if (rd.load == 2) {
            const LoopRec &fw = chain[g0 + first_write[r]];
            rd.fw_xlo = fw.lo[0];
            rd.fw_xhi = fw.hi[0];
            rd.fw_ylo = fw.lo[1];
            rd.fw_yhi = fw.hi[1];
        }
    }
    if (lds > lds_budget) return false;
    D.nload = D.nstore = 0;
    for (int r = 0; r < nr; ++r) {
        if (D.rings[r].load) D.load_list[D.nload++] = r;
        if (D.rings[r].store) D.store_list[D.nstore++] = r;
    }
    if (D.nload > kFMaxLoaded) return false;

    // loops and their entries
    int e = 0, in = 0;
    for (int i = 0; i < n; ++i) {
        const LoopRec &lp = chain[g0 + i];
        FLoopD &L = D.loops[i];
        L.out_ring = ring_of[lp.args[0].handle];
        L.lag = lag[i];
        L.xlo = lp.lo[0];
        L.xhi = lp.hi[0];
        L.ylo = lp.lo[1];
        L.yhi = lp.hi[1];
        L.hlo = hlo[i];
        L.hhi = hhi[i];
        L.vlo = vlo[i];
        L.vhi = vhi[i];
        L.ent0 = e;
        L.in0 = in;
        for (size_t a = 1; a < lp.args.size(); ++a) {
            const Stencil &st = c.stencils[lp.args[a].stencil];
            FInD &I = D.ins[in++];
            I.ring = ring_of[lp.args[a].handle];
            I.ent0 = e;
            I.nent = st.npoints();
            I.star = canonical_star2(st);
            if (I.star < 0) I.star = 0;
            for (int p = 0; p < st.npoints(); ++p, ++e) {
                D.ent[e].ring = (short)I.ring;
                D.ent[e].dx = (signed char)st.pts[3 * p];
                D.ent[e].dy = (signed char)st.pts[3 * p + 1];
            }
        }
        L.nent = e - L.ent0;
        L.nin = in - L.in0;
    }
    D.nin = in;
    D.R = R;
    D.HR = HR;
    D.W = W;
    G.g0 = g0;
    G.g1 = g1;
    G.dtype = dtype;
    G.lds_bytes = lds;
    (void)tile;
    return true;
}

// Group domain: bounding box of the loops' ranges and of the store regions.
void group_domain(const Ctx &c, const std::vector<LoopRec> &chain, const FusedGroup &G, int dom[4]) {
    dom[0] = dom[2] = INT_MAX;
    dom[1] = dom[3] = INT_MIN;
    for (int l = G.g0; l < G.g1; ++l) {
        dom[0] = std::min(dom[0], chain[l].lo[0]);
        dom[1] = std::max(dom[1], chain[l].hi[0]);
        dom[2] = std::min(dom[2], chain[l].lo[1]);
        dom[3] = std::max(dom[3], chain[l].hi[1]);
    }
    for (size_t r = 0; r < G.ring_dat.size(); ++r) {
        if (!G.ring_store[r]) continue;
        const Dataset &ds = c.dats[G.ring_dat[r]];
        if (!ds.ever_written) continue;
        dom[0] = std::min(dom[0], ds.wlo[0]);
        dom[1] = std::max(dom[1], ds.whi[0]);
        dom[2] = std::min(dom[2], ds.wlo[1]);
        dom[3] = std::max(dom[3], ds.whi[1]);
    }
}

}  // namespace

std::vector<std::shared_ptr<FusedGroup>> fused_split(const Ctx &c, const std::vector<LoopRec> &chain,
                                                     const int tile[3]) {
    std::vector<std::shared_ptr<FusedGroup>> out;
    const int budget = (tile[2] > 0 ? tile[2] : 158) * 1024 - kFDescLds;
    const int rows = (tile[0] == 2 || tile[0] == 8 || tile[0] == 16) ? tile[0] : 4;
    const int L = (int)chain.size();
    int g0 = 0;
    while (g0 < L) {
        auto best = std::make_shared<FusedGroup>();
        int g1 = g0;
        for (int cand = g0 + 1; cand <= L; ++cand) {
            FusedGroup G;
            G.rows = rows;
            if (!analyse(c, chain, g0, cand, tile, budget, G)) break;
            *best = G;
            g1 = cand;
        }
        if (g1 - g0 >= 2) {
            best->hseg_req = tile[1];
            out.push_back(best);
            g0 = g1;
        } else {
            g0 += 1;  // runs as a single-loop kernel
        }
    }
    return out;
}

tc_status fused_run(Ctx &c, const std::vector<LoopRec> &chain, FusedGroup &G) {
    FGroupD &T = G.tmpl;
    int dom[4];
    // store regions after this group: hull of earlier writes and this group's writes
    std::vector<int> hull(4 * T.nrings);
    for (int r = 0; r < T.nrings; ++r) {
        const Dataset &ds = c.dats[G.ring_dat[r]];
        int h[4] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};
        if (ds.ever_written) {
            h[0] = ds.wlo[0];
            h[1] = ds.whi[0];
            h[2] = ds.wlo[1];
            h[3] = ds.whi[1];
        }
        for (int l = G.g0; l < G.g1; ++l)
            if (chain[l].args[0].handle == G.ring_dat[r]) {
                h[0] = std::min(h[0], chain[l].lo[0]);
                h[1] = std::max(h[1], chain[l].hi[0]);
                h[2] = std::min(h[2], chain[l].lo[1]);
                h[3] = std::max(h[3], chain[l].hi[1]);
            }
        for (int k = 0; k < 4; ++k) hull[4 * r + k] = h[k];
    }
    group_domain(c, chain, G, dom);
    for (int r = 0; r < T.nrings; ++r)
        if (G.ring_store[r]) {
            dom[0] = std::min(dom[0], hull[4 * r]);
            dom[1] = std::max(dom[1], hull[4 * r + 1]);
            dom[2] = std::min(dom[2], hull[4 * r + 2]);
            dom[3] = std::max(dom[3], hull[4 * r + 3]);
        }
    // the first column of every workgroup's ring rows must be even (16-byte
    // aligned row loads straight into LDS)
    if (((dom[0] - T.HR) & 1) != 0) dom[0] -= 1;
    const int width = dom[1] - dom[0], height = dom[3] - dom[2];
    const int nbx = (width + T.W - 1) / T.W;
    int Hseg = G.hseg_req;
    if (Hseg <= 0) {
        int nby = std::max(1, (int)std::lround(256.0 / nbx));
        Hseg = std::max(16, (height + nby - 1) / nby);
    }
    const int nby = (height + Hseg - 1) / Hseg;

    if (!G.host) {
        if (hipHostMalloc((void **)&G.host, sizeof(FGroupD), hipHostMallocDefault) != hipSuccess)
            return fail(c, TC_ERR_DEVICE, "hipHostMalloc of a fused descriptor failed");
        G.dev = (FGroupD *)dev_alloc(c, sizeof(FGroupD));
        if (!G.dev) return fail(c, TC_ERR_NOMEM, "cannot allocate a fused descriptor");
        if (hipEventCreateWithFlags(&G.uploaded, hipEventDisableTiming) != hipSuccess)
            return fail(c, TC_ERR_DEVICE, "hipEventCreate failed");
    } else if (hipEventSynchronize(G.uploaded) != hipSuccess) {
        return fail(c, TC_ERR_DEVICE, "hipEventSynchronize failed");
    }
    FGroupD &D = *G.host;
    std::memcpy(&D, &T, sizeof(FGroupD));
    D.Hseg = Hseg;
    D.ring_bytes = G.lds_bytes;
    D.dom_xlo = dom[0];
    D.dom_ylo = dom[2];
    D.nbx = nbx;
    D.nby = nby;
    // weights
    for (int i = 0; i < D.nloops; ++i) {
        const LoopRec &lp = chain[G.g0 + i];
        for (int k = 0; k < D.loops[i].nent; ++k) D.w[D.loops[i].ent0 + k] = lp.params[k];
    }
    // buffers: read from the current buffer, write written datasets to the twin
    for (int r = 0; r < D.nrings; ++r) {
        Dataset &ds = c.dats[G.ring_dat[r]];
        FRingD &rd = D.rings[r];
        rd.src = ds.origin(ds.cur);
        rd.dst = nullptr;
        if (rd.store) {
            const int tw = 1 - ds.cur;
            if (!ds.raw[tw]) {
                ds.raw[tw] = dev_alloc(c, (size_t)(ds.bytes + ds.stagger));
                if (!ds.raw[tw]) return fail(c, TC_ERR_NOMEM, "cannot allocate the second buffer of %s", ds.name.c_str());
                ds.buf[tw] = (char *)ds.raw[tw] + ds.stagger;
                ds.twin_synced = false;
            }
            if (!ds.twin_synced) {
                if (hipMemcpyAsync(ds.buf[tw], ds.buf[ds.cur], (size_t)ds.bytes, hipMemcpyDeviceToDevice, c.stream) !=
                    hipSuccess)
                    return fail(c, TC_ERR_DEVICE, "hipMemcpyAsync (second buffer) failed");
                ds.twin_synced = true;
            }
            rd.dst = ds.origin(tw);
            rd.hull_xlo = hull[4 * r];
            rd.hull_xhi = hull[4 * r + 1];
            rd.hull_ylo = hull[4 * r + 2];
            rd.hull_yhi = hull[4 * r + 3];
        }
    }
    // flat records for the kernel's steps
    for (int i = 0; i < D.nloops; ++i) {
        const FLoopD &L = D.loops[i];
        FLoopRec &Q = D.lrec[i];
        std::memset(&Q, 0, sizeof Q);
        Q.lag = L.lag;
        Q.ylo = L.ylo;
        Q.yhi = L.yhi;
        Q.vlo = L.vlo;
        Q.vhi = L.vhi;
        const FRingD &O = D.rings[L.out_ring];
        Q.out_off = O.lds_off;
        Q.out_depth = O.depth;
        Q.out_inv = O.inv_depth;
        Q.nin = L.nin;
        for (int k = 0; k < L.nin; ++k) {
            const FInD &I = D.ins[L.in0 + k];
            const FRingD &Rg = D.rings[I.ring];
            FInRec &J = Q.in[k];
            J.off = Rg.lds_off;
            J.depth = Rg.depth;
            J.inv = Rg.inv_depth;
            J.star = I.star;
            J.ent0 = I.ent0;
            J.nent = I.nent;
            if (I.star)
                for (int q = 0; q < I.nent; ++q) Q.w[k][q] = D.w[I.ent0 + q];
        }
    }
    for (int i = 0; i < D.nload; ++i) {
        const FRingD &Rg = D.rings[D.load_list[i]];
        FLoadRec &Q = D.ld[i];
        std::memset(&Q, 0, sizeof Q);
        Q.src = Rg.src;
        Q.sy = Rg.sy;
        Q.off = Rg.lds_off;
        Q.depth = Rg.depth;
        Q.inv = Rg.inv_depth;
        Q.lag = Rg.load_lag;
        Q.ext_ylo = Rg.ext_ylo;
        Q.ext_yhi = Rg.ext_yhi;
        Q.ld_below = Rg.ld_below;
        Q.ld_above = Rg.ld_above;
        Q.ext_xlo = Rg.ext_xlo;
        Q.ext_xhi = Rg.ext_xhi;
        Q.fw = Rg.load == 2;
        Q.fw_xlo = Rg.fw_xlo;
        Q.fw_xhi = Rg.fw_xhi;
        Q.fw_ylo = Rg.fw_ylo;
        Q.fw_yhi = Rg.fw_yhi;
        Q.alloc_xlo = -(int)c.dats[G.ring_dat[D.load_list[i]]].xorg;
    }
    for (int i = 0; i < D.nstore; ++i) {
        const FRingD &Rg = D.rings[D.store_list[i]];
        FStoreRec &Q = D.st[i];
        std::memset(&Q, 0, sizeof Q);
        Q.dst = Rg.dst;
        Q.sy = Rg.sy;
        Q.off = Rg.lds_off;
        Q.depth = Rg.depth;
        Q.inv = Rg.inv_depth;
        Q.lag = Rg.store_lag;
        Q.hxlo = Rg.hull_xlo;
        Q.hxhi = Rg.hull_xhi;
        Q.hylo = Rg.hull_ylo;
        Q.hyhi = Rg.hull_yhi;
    }
    if (hipMemcpyAsync(G.dev, G.host, sizeof(FGroupD), hipMemcpyHostToDevice, c.stream) != hipSuccess)
        return fail(c, TC_ERR_DEVICE, "hipMemcpyAsync (fused descriptor) failed");
    if (hipEventRecord(G.uploaded, c.stream) != hipSuccess) return fail(c, TC_ERR_DEVICE, "hipEventRecord failed");
    G.nblocks = nbx * nby;
    hipError_t e = launch_fused(G.dev, G.dtype, G.rows, G.nblocks, G.lds_bytes + kFDescLds, c.stream);
    if (e != hipSuccess) return fail(c, TC_ERR_DEVICE, "fused kernel launch failed: %s", hipGetErrorString(e));
    // the written datasets now live in their second buffers
    for (int r = 0; r < D.nrings; ++r)
        if (D.rings[r].store) {
            Dataset &ds = c.dats[G.ring_dat[r]];
            ds.cur = 1 - ds.cur;
        }
    return TC_OK;
}

void fused_release(Ctx &c) {
    for (auto &kv : c.plans)
        for (auto &g : kv.second->groups) {
            if (g->host) (void)hipHostFree(g->host);
            if (g->dev) dev_free(c, g->dev);
            if (g->uploaded) (void)hipEventDestroy(g->uploaded);
            g->host = nullptr;
            g->dev = nullptr;
            g->uploaded = nullptr;
        }
}

// AUTO mode (Section 4.3 chooses a tile size from the cache size; here the
// cache-based choice is one candidate and every candidate is measured): the
// first flushes of a chain structure each run one candidate schedule while
// its device time is measured; afterwards the fastest is used.  Every
// candidate computes bit-identical results, so tuning never changes answers.
namespace {
struct Cand {
    tc_tiling mode;
    int tile[3];
};
std::vector<Cand> candidates(const std::vector<LoopRec> &chain) {
    std::vector<Cand> v;
    v.push_back({TC_TILING_NONE, {0, 0, 0}});
    v.push_back({TC_TILING_SKEWED, {0, 0, 0}});
    const int nd = chain.empty() ? 2 : chain[0].ndim;
    if (nd >= 2) {
        int t[3] = {0, 0, 0};
        t[nd - 1] = 128;
        v.push_back({TC_TILING_SKEWED, {t[0], t[1], t[2]}});
    }
    bool any2d = false;
    for (const auto &lp : chain) any2d = any2d || (lp.ndim == 2 && lp.op == TC_OP_WSUM);
    if (any2d) {
        v.push_back({TC_TILING_FUSED, {4, 0, 0}});
        v.push_back({TC_TILING_FUSED, {8, 0, 0}});
    }
    return v;
}
}  // namespace

tc_tiling autotune_choose(Ctx &c, const std::vector<LoopRec> &chain, int tile[3]) {
    const int zero[3] = {0, 0, 0};
    const uint64_t key = chain_key(c, chain, TC_TILING_AUTO, zero);
    auto cands = candidates(chain);
    Ctx::Tune &T = c.tuned[key];
    int pick;
    if (T.best >= 0) {
        pick = T.best;
        c.tune_cand = -1;
    } else {
        pick = T.next;
        c.tune_cand = pick;
        c.tune_key = key;
    }
    for (int d = 0; d < 3; ++d) tile[d] = cands[pick].tile[d];
    return cands[pick].mode;
}

void autotune_record(Ctx &c, double seconds) {
    if (c.tune_cand < 0) return;
    Ctx::Tune &T = c.tuned[c.tune_key];
    T.seconds.push_back(seconds);
    T.next = c.tune_cand + 1;
    // the candidate list depends only on the chain structure, so its length
    // is recovered from the number of candidates of any chain with this key
    c.tune_cand = -1;
}

void autotune_finish(Ctx &c, size_t ncand) {
    Ctx::Tune &T = c.tuned[c.tune_key];
    if (T.best < 0 && T.seconds.size() >= ncand) {
        int b = 0;
        for (size_t i = 1; i < T.seconds.size(); ++i)
            if (T.seconds[i] < T.seconds[b]) b = (int)i;
        T.best = b;
    }
}

size_t autotune_candidates(const std::vector<LoopRec> &chain) { return candidates(chain).size(); }

}  // namespace tc
