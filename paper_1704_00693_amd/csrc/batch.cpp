// Host side of the batched heat-conduction solves (kernels in batch.hip):
// slots, admission by HBM footprint, the tile list, graph capture and replay,
// retirement of finished solves.
#include "batch.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <unordered_map>
#include <vector>

#include "fused.hpp"
#include "tc_internal.hpp"

namespace tc {
hipError_t batch_enqueue_iteration(BInst *insts, int ninst, const BTileList &all, const BTileList &three,
                                   const BTileList &fused, double *part, int grid, int cheb_steps, bool mixed, int fh,
                                   int fty, int f3, bool with3d, bool setup, hipStream_t s);
}

using namespace tc;

struct tc_batch {
    tc_ctx *ctx = nullptr;
    tc_batch_opts o{};
    BInst *d_inst = nullptr, *h_inst = nullptr;
    // every resident solve's tiles (kBTX x kBTY), the 3D solves' tiles (their
    // kBTX x kBTY tiles, or kF3X x kF3Y x kF3Z segments when their Chebyshev
    // steps are fused), and the 2D solves' fused Chebyshev tiles (kFTX x kFTY)
    BTileList all, three, fused;
    int fh = kFH, fty = kFTY;  // fused Chebyshev steps per launch (0: one launch per step) and tile height
    int f3 = 3;                // 3D: fused Chebyshev steps per launch (0: one launch per step)
    bool graphs = true;        // replay the captured iteration (else enqueue its launches directly)
    double *stage = nullptr;   // pinned staging memory of kept solutions
    int64_t stage_cap = 0;     // its size in doubles
    double *d_part = nullptr;
    int64_t tile_cap = 0;
    int grid = 0;
    // the captured iteration, gx[setup][with3d]: without set-up kernels
    // (replayed except right after an admission), without the 3D instances'
    // per-step Chebyshev launches (replayed while no 3D solve is resident)
    hipGraphExec_t gx[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    bool has3d = false;
    bool replayed = false;  // replays are in flight on the stream

    struct Slot {
        int64_t ticket = -1;
        int64_t bytes = 0;
        int64_t tiles = 0;
        void *mem = nullptr;
        double t_submit = 0.0, t_admit = 0.0;
        tc_solve_desc d{};
    };
    std::vector<Slot> slots;
    struct Req {
        int64_t ticket;
        tc_solve_desc d;
        double t_submit;
    };
    std::deque<Req> pending;
    struct Done {
        tc_solve_result r{};
        std::vector<double> x;
    };
    std::unordered_map<int64_t, Done> done;
    std::unordered_map<int64_t, int> running;  // ticket -> slot
    int64_t next_ticket = 0;
    int64_t resident_bytes = 0, resident_tiles = 0;
};

namespace {

Ctx &C(tc_batch *b) { return b->ctx->c; }

Ctx *batch_ctx(tc_batch *b) { return b && b->ctx ? &b->ctx->c : nullptr; }

int64_t padded_cells(const tc_solve_desc &d) {
    const int64_t p = d.n + 2;
    return d.ndim == 3 ? p * p * p : p * p;
}

int64_t tiles_of(const tc_solve_desc &d) {
    const int64_t tx = (d.n + kBTX - 1) / kBTX, ty = (d.n + kBTY - 1) / kBTY;
    return tx * ty * (d.ndim == 3 ? d.n : 1);
}

int64_t round256(int64_t v) { return (v + 255) / 256 * 256; }

// Bytes of one solve's fields (each field padded by one ghost layer and
// aligned to 256 bytes): FP64 mode 10 + ndim double fields; mixed mode
// 3 + ndim double fields and 9 + ndim float fields (the sweep fields include
// the second rt buffer of the fused Chebyshev steps).
int64_t footprint(const tc_solve_desc &d, bool mixed) {
    const int64_t cells = padded_cells(d);
    const int64_t f8 = round256(cells * 8), f4 = round256(cells * 4);
    if (!mixed) return (10 + d.ndim) * f8;
    return (3 + d.ndim) * f8 + (9 + d.ndim) * f4;
}

tc_status admit(tc_batch *b, int slot, const tc_batch::Req &q) {
    Ctx &c = C(b);
    const tc_solve_desc &d = q.d;
    const bool mixed = b->o.mixed != 0;
    const int64_t bytes = footprint(d, mixed);
    void *mem = dev_alloc(c, (size_t)bytes);
    if (!mem) return fail(c, TC_ERR_NOMEM, "tc_batch: cannot allocate %lld bytes for a solve", (long long)bytes);
    tc_batch::Slot &S = b->slots[slot];
    S.ticket = q.ticket;
    S.bytes = bytes;
    S.tiles = tiles_of(d);
    S.mem = mem;
    S.t_submit = q.t_submit;
    S.t_admit = now_s();
    S.d = d;
    BInst &I = b->h_inst[slot];
    std::memset(&I, 0, sizeof I);
    I.ndim = d.ndim;
    I.n = d.n;
    I.state = B_INIT;
    I.mixed = mixed ? 1 : 0;
    I.max_iter = d.max_iter;
    I.max_outer = d.max_outer;
    I.cheb_steps = b->o.cheb_steps;
    I.seed = d.seed;
    I.tol = d.tol;
    I.inner_tol = b->o.inner_tol;
    I.rx = d.dt * (double)d.n * (double)d.n;
    const int64_t p = d.n + 2;
    I.sy = p;
    I.sz = d.ndim == 3 ? p * p : 0;
    I.org = 1 + I.sy + (d.ndim == 3 ? I.sz : 0);
    const int64_t cells = padded_cells(d);
    const int64_t f8 = round256(cells * 8), f4 = round256(cells * 4);
    char *m = (char *)mem;
    auto take = [&](int64_t sz) {
        void *r = m;
        m += sz;
        return r;
    };
    I.u = (double *)take(f8);
    I.u0 = (double *)take(f8);
    I.r = (double *)take(f8);
    I.kx = (double *)take(f8);
    I.ky = (double *)take(f8);
    I.kz = d.ndim == 3 ? (double *)take(f8) : nullptr;
    if (!mixed) {
        I.xi = I.u;
        I.ri = I.r;
        I.kxi = I.kx;
        I.kyi = I.ky;
        I.kzi = I.kz;
        I.p = take(f8);
        I.w = take(f8);
        I.z = take(f8);
        I.rt = take(f8);
        I.sd0 = take(f8);
        I.sd1 = take(f8);
        I.rt2 = take(f8);
    } else {
        I.xi = take(f4);
        I.ri = take(f4);
        I.kxi = take(f4);
        I.kyi = take(f4);
        I.kzi = d.ndim == 3 ? take(f4) : nullptr;
        I.p = take(f4);
        I.w = take(f4);
        I.z = take(f4);
        I.rt = take(f4);
        I.sd0 = take(f4);
        I.sd1 = take(f4);
        I.rt2 = take(f4);
    }
    b->resident_bytes += bytes;
    b->resident_tiles += S.tiles;
    b->running[q.ticket] = slot;
    return TC_OK;
}

// Copy the interior of x (n^ndim values) of a resident solve to host memory:
// the padded field in one copy into pinned staging memory, then its rows.
tc_status copy_x(tc_batch *b, int slot, std::vector<double> &out) {
    Ctx &c = C(b);
    const BInst &I = b->h_inst[slot];
    const int64_t n = I.n, nz = I.ndim == 3 ? n : 1;
    const int64_t cells = padded_cells(b->slots[slot].d);
    if (b->stage_cap < cells) {
        if (b->stage) (void)hipHostFree(b->stage);
        b->stage = nullptr;
        b->stage_cap = 0;
        if (hipHostMalloc((void **)&b->stage, (size_t)cells * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return fail(c, TC_ERR_NOMEM, "tc_batch: cannot allocate %lld bytes of pinned staging memory",
                        (long long)(cells * 8));
        b->stage_cap = cells;
    }
    if (hipMemcpyAsync(b->stage, I.u, (size_t)cells * sizeof(double), hipMemcpyDeviceToHost, c.stream) !=
            hipSuccess ||
        hipStreamSynchronize(c.stream) != hipSuccess)
        return fail(c, TC_ERR_DEVICE, "tc_batch: copy of a solution failed");
    out.assign((size_t)(n * n * nz), 0.0);
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < n; ++y)
            std::memcpy(out.data() + (z * n + y) * n, b->stage + I.org + y * I.sy + z * I.sz, (size_t)n * sizeof(double));
    return TC_OK;
}

void retire(tc_batch *b, int slot) {
    Ctx &c = C(b);
    tc_batch::Slot &S = b->slots[slot];
    const BInst &I = b->h_inst[slot];
    tc_batch::Done D;
    D.r.state = TC_SOLVE_DONE;
    D.r.iterations = I.iters;
    D.r.outer = I.outer;
    D.r.bnorm = I.bnorm;
    D.r.lmax = I.lmax;
    D.r.rel_residual = std::sqrt(I.true_rr) / I.bnorm;
    D.r.converged = D.r.rel_residual <= I.tol ? 1 : 0;
    const double t = now_s();
    D.r.seconds = t - S.t_submit;
    D.r.queue_seconds = S.t_admit - S.t_submit;
    if (S.d.keep_x) (void)copy_x(b, slot, D.x);
    b->done[S.ticket] = std::move(D);
    b->running.erase(S.ticket);
    dev_free(c, S.mem);
    b->resident_bytes -= S.bytes;
    b->resident_tiles -= S.tiles;
    S = tc_batch::Slot();
    b->h_inst[slot].state = B_FREE;
}

// Tile list of the resident solves, slot order, tiles row-major (x fastest)
// within a solve; every resident record is uploaded with its tile range.
tc_status rebuild_tiles(tc_batch *b) {
    Ctx &c = C(b);
    int64_t nt = 0, n3 = 0, nf = 0;
    for (size_t s = 0; s < b->slots.size(); ++s) {
        BInst &I = b->h_inst[s];
        if (I.state == B_FREE) {
            I.tile0 = 0;
            I.ntile = 0;
            continue;
        }
        const int tx = (I.n + kBTX - 1) / kBTX, ty = (I.n + kBTY - 1) / kBTY, tz = I.ndim == 3 ? I.n : 1;
        I.tile0 = nt;
        const bool march3 = I.ndim == 3 && b->fh > 0 && b->f3 > 0;
        for (int z = 0; z < tz; ++z)
            for (int y = 0; y < ty; ++y)
                for (int x = 0; x < tx; ++x) {
                    b->all.h[nt++] = BTile{(int32_t)s, x, y, z};
                    if (I.ndim == 3 && !march3) b->three.h[n3++] = BTile{(int32_t)s, x, y, z};
                }
        if (march3) {
            const int mx = (I.n + kF3X - 1) / kF3X, my = (I.n + kF3Y - 1) / kF3Y, mz = (I.n + kF3Z - 1) / kF3Z;
            for (int z = 0; z < mz; ++z)
                for (int y = 0; y < my; ++y)
                    for (int x = 0; x < mx; ++x) b->three.h[n3++] = BTile{(int32_t)s, x, y, z};
        }
        I.ntile = nt - I.tile0;
        if (I.ndim == 2) {
            const int fx = (I.n + kFTX - 1) / kFTX, fy = (I.n + b->fty - 1) / b->fty;
            for (int y = 0; y < fy; ++y)
                for (int x = 0; x < fx; ++x) b->fused.h[nf++] = BTile{(int32_t)s, x, y, 0};
        }
    }
    *b->all.hn = nt;
    *b->three.hn = n3;
    b->has3d = n3 > 0;
    *b->fused.hn = nf;
    auto up = [&](BTileList &L) {
        return hipMemcpyAsync(L.d, L.h, (size_t)std::max<int64_t>(*L.hn, 1) * sizeof(BTile), hipMemcpyHostToDevice,
                              c.stream) == hipSuccess &&
               hipMemcpyAsync(L.dn, L.hn, sizeof(int64_t), hipMemcpyHostToDevice, c.stream) == hipSuccess;
    };
    if (!up(b->all) || !up(b->three) || !up(b->fused) ||
        hipMemcpyAsync(b->d_inst, b->h_inst, b->slots.size() * sizeof(BInst), hipMemcpyHostToDevice, c.stream) !=
            hipSuccess)
        return fail(c, TC_ERR_DEVICE, "tc_batch: upload of the tile lists failed");
    return TC_OK;
}

tc_status capture(tc_batch *b) {
    Ctx &c = C(b);
    if (!c.cap_stream && hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(c, TC_ERR_DEVICE, "tc_batch: cannot create the capture stream");
    for (int setup = 0; setup < 2; ++setup)
        for (int with3d = 0; with3d < 2; ++with3d) {
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return fail(c, TC_ERR_DEVICE, "tc_batch: graph capture failed to start");
            const hipError_t e = batch_enqueue_iteration(b->d_inst, (int)b->slots.size(), b->all, b->three, b->fused,
                                                         b->d_part, b->grid, b->o.cheb_steps, b->o.mixed != 0, b->fh,
                                                         b->fty, b->f3, with3d != 0, setup != 0, c.cap_stream);
            const hipError_t e2 = hipStreamEndCapture(c.cap_stream, &g);
            if (e != hipSuccess || e2 != hipSuccess || !g)
                return fail(c, TC_ERR_DEVICE, "tc_batch: graph capture failed");
            const hipError_t e3 = hipGraphInstantiate(&b->gx[setup][with3d], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e3 != hipSuccess) return fail(c, TC_ERR_DEVICE, "tc_batch: graph instantiation failed");
        }
    return TC_OK;
}

}  // namespace

// Bodies of the C ABI calls; the exported wrappers below turn any C++
// exception into a status code.

static tc_status impl_tc_batch_create(tc_ctx *ctx, const tc_batch_opts *opts, tc_batch **out) {
    if (!ctx || !opts || !out) return TC_ERR_ARG;
    Ctx &c = ctx->c;
    if (c.poisoned) return TC_ERR_DEVICE;
    if (c.host_only) return fail(c, TC_ERR_STATE, "tc_batch_create: host-only context");
    if (opts->max_instances < 1 || opts->max_cells < 1 || opts->hbm_budget < 1)
        return fail(c, TC_ERR_ARG, "tc_batch_create: capacities must be positive");
    if (opts->cheb_steps < 0 || opts->cheb_steps > kBMaxCheb)
        return fail(c, TC_ERR_ARG, "tc_batch_create: cheb_steps must be 0..%d", kBMaxCheb);
    tc_batch *b = new tc_batch();
    b->ctx = ctx;
    b->o = *opts;
    if (b->o.cheb_steps == 0) b->o.cheb_steps = 10;
    if (b->o.replays_per_step <= 0) b->o.replays_per_step = 4;
    if (b->o.inner_tol <= 0.0) b->o.inner_tol = 1e-4;
    b->slots.resize((size_t)opts->max_instances);
    // every solve needs at most ceil(n/64) ceil(n/4) n_z tiles for n^2 or n^3
    // cells; bound the list by the cell budget plus one partial tile row per slot
    b->tile_cap = opts->max_cells / (kBTX * kBTY) * 2 + 64 * (int64_t)opts->max_instances + 64;
    b->grid = (int)std::min<int64_t>(b->tile_cap, 2048);
    const size_t ib = b->slots.size() * sizeof(BInst);
    b->d_inst = (BInst *)dev_alloc(c, ib);
    b->d_part = (double *)dev_alloc(c, (size_t)b->tile_cap * 4 * sizeof(double));
    bool ok = b->d_inst && b->d_part;
    ok = ok && hipHostMalloc((void **)&b->h_inst, ib, hipHostMallocDefault) == hipSuccess;
    // a solve's fused tiles and 3D tiles are never more than its kBTX x kBTY tiles
    for (BTileList *L : {&b->all, &b->three, &b->fused}) {
        L->d = (BTile *)dev_alloc(c, (size_t)b->tile_cap * sizeof(BTile));
        L->dn = (int64_t *)dev_alloc(c, sizeof(int64_t));
        ok = ok && L->d && L->dn;
        ok = ok && hipHostMalloc((void **)&L->h, (size_t)b->tile_cap * sizeof(BTile), hipHostMallocDefault) == hipSuccess;
        ok = ok && hipHostMalloc((void **)&L->hn, sizeof(int64_t), hipHostMallocDefault) == hipSuccess;
    }
    if (!ok) {
        tc_batch_destroy(b);
        return fail(c, TC_ERR_NOMEM, "tc_batch_create: cannot allocate the engine's arrays");
    }
    std::memset(b->h_inst, 0, ib);
    // TC_BATCH_FUSED=FH[,FTY]: Chebyshev steps per fused launch (0: none), tile height
    if (const char *e = getenv("TC_BATCH_FUSED")) {
        int fh = kFH, fty = kFTY;
        if (std::sscanf(e, "%d,%d", &fh, &fty) < 1) fh = kFH;
        const bool shape = (fh == 3 && (fty == 16 || fty == 32)) || (fh == 5 && (fty == 16 || fty == 32)) ||
                           (fh == 9 && fty == 16);
        b->fh = fh <= 0 ? 0 : (shape ? fh : kFH);
        b->fty = shape ? fty : kFTY;
    }
    // TC_BATCH_FUSED3=0: the 3D solves' Chebyshev steps one launch each
    if (const char *e = getenv("TC_BATCH_FUSED3")) b->f3 = atoi(e) > 0 ? 3 : 0;
    // TC_BATCH_GRAPHS=0: enqueue each iteration's launches instead of replaying the graph
    if (const char *e = getenv("TC_BATCH_GRAPHS")) b->graphs = atoi(e) != 0;
    if (rebuild_tiles(b) != TC_OK || capture(b) != TC_OK) {
        tc_batch_destroy(b);
        return TC_ERR_DEVICE;
    }
    *out = b;
    return TC_OK;
}

static tc_status impl_tc_batch_submit(tc_batch *b, const tc_solve_desc *d, int64_t *ticket) {
    if (!b || !d || !ticket) return TC_ERR_ARG;
    Ctx &c = C(b);
    if (c.poisoned) return TC_ERR_DEVICE;
    if ((d->ndim != 2 && d->ndim != 3) || d->n < 2 || !(d->tol > 0.0) || d->max_iter < 1 || d->max_outer < 0 ||
        !(d->dt > 0.0))
        return fail(c, TC_ERR_ARG, "tc_batch_submit: bad solve description");
    *ticket = b->next_ticket++;
    b->pending.push_back(tc_batch::Req{*ticket, *d, now_s()});
    return TC_OK;
}

static tc_status impl_tc_batch_step(tc_batch *b, int32_t *unfinished) {
    if (!b) return TC_ERR_ARG;
    Ctx &c = C(b);
    if (c.poisoned) return TC_ERR_DEVICE;
    // the previous replays, then the device records
    if (b->replayed) {
        if (hipMemcpyAsync(b->h_inst, b->d_inst, b->slots.size() * sizeof(BInst), hipMemcpyDeviceToHost, c.stream) !=
                hipSuccess ||
            hipStreamSynchronize(c.stream) != hipSuccess)
            return fail(c, TC_ERR_DEVICE, "tc_batch_step: device sync failed");
        b->replayed = false;
    }
    bool dirty = false, admitted = false;
    for (size_t s = 0; s < b->slots.size(); ++s)
        if (b->slots[s].ticket >= 0 && b->h_inst[s].state == B_DONE) {
            retire(b, (int)s);
            dirty = true;
        }
    // admission in arrival order while slots, cells and the HBM budget allow
    while (!b->pending.empty()) {
        const tc_batch::Req &q = b->pending.front();
        const int64_t bytes = footprint(q.d, b->o.mixed != 0), tl = tiles_of(q.d);
        if (bytes > b->o.hbm_budget || tl > b->tile_cap) {
            tc_batch::Done D;
            D.r.state = TC_SOLVE_REJECTED;
            b->done[q.ticket] = D;
            b->pending.pop_front();
            continue;
        }
        if (b->resident_bytes + bytes > b->o.hbm_budget || b->resident_tiles + tl > b->tile_cap) break;
        int slot = -1;
        for (size_t s = 0; s < b->slots.size(); ++s)
            if (b->slots[s].ticket < 0) {
                slot = (int)s;
                break;
            }
        if (slot < 0) break;
        const tc_status st = admit(b, slot, q);
        if (st != TC_OK) return st;
        b->pending.pop_front();
        dirty = true;
        admitted = true;
    }
    if (dirty) {
        const tc_status st = rebuild_tiles(b);
        if (st != TC_OK) return st;
    }
    if (!b->running.empty()) {
        // instances are in the set-up state only from their admission to the
        // end of the next iteration
        const int with3d = b->has3d || b->fh == 0 ? 1 : 0;
        for (int k = 0; k < b->o.replays_per_step; ++k) {
            const bool setup = admitted && k == 0;
            if (!b->graphs) {
                // the same launches as the captured iteration, enqueued directly
                if (batch_enqueue_iteration(b->d_inst, (int)b->slots.size(), b->all, b->three, b->fused, b->d_part,
                                            b->grid, b->o.cheb_steps, b->o.mixed != 0, b->fh, b->fty, b->f3,
                                            with3d != 0, setup, c.stream) != hipSuccess)
                    return fail(c, TC_ERR_DEVICE, "tc_batch_step: launch failed");
            } else if (hipGraphLaunch(b->gx[setup ? 1 : 0][with3d], c.stream) != hipSuccess) {
                return fail(c, TC_ERR_DEVICE, "tc_batch_step: graph launch failed");
            }
        }
        b->replayed = true;
    }
    if (unfinished) *unfinished = (int32_t)(b->running.size() + b->pending.size());
    return TC_OK;
}

static tc_status impl_tc_batch_poll(tc_batch *b, int64_t ticket, tc_solve_result *out) {
    if (!b || !out) return TC_ERR_ARG;
    auto it = b->done.find(ticket);
    std::memset(out, 0, sizeof *out);
    if (it != b->done.end()) {
        *out = it->second.r;
        return TC_OK;
    }
    if (ticket < 0 || ticket >= b->next_ticket) return fail(C(b), TC_ERR_ARG, "tc_batch_poll: unknown ticket");
    out->state = b->running.count(ticket) ? TC_SOLVE_RUNNING : TC_SOLVE_PENDING;
    return TC_OK;
}

static tc_status impl_tc_batch_wait(tc_batch *b) {
    if (!b) return TC_ERR_ARG;
    int32_t left = 1;
    while (left > 0) {
        const tc_status st = tc_batch_step(b, &left);
        if (st != TC_OK) return st;
    }
    // a last round retires what the final replays finished
    return tc_batch_step(b, &left);
}

static tc_status impl_tc_batch_read_x(tc_batch *b, int64_t ticket, double *host, int64_t cap) {
    if (!b || !host) return TC_ERR_ARG;
    auto it = b->done.find(ticket);
    if (it == b->done.end() || it->second.x.empty())
        return fail(C(b), TC_ERR_STATE, "tc_batch_read_x: no kept solution for this ticket");
    if (cap < (int64_t)it->second.x.size()) return fail(C(b), TC_ERR_ARG, "tc_batch_read_x: buffer too small");
    std::memcpy(host, it->second.x.data(), it->second.x.size() * sizeof(double));
    return TC_OK;
}

static tc_status impl_tc_batch_destroy(tc_batch *b) {
    if (!b) return TC_OK;
    Ctx &c = C(b);
    (void)hipStreamSynchronize(c.stream);
    for (auto &S : b->slots)
        if (S.mem) dev_free(c, S.mem);
    for (auto &row : b->gx)
        for (hipGraphExec_t ge : row)
            if (ge) (void)hipGraphExecDestroy(ge);
    if (b->d_inst) dev_free(c, b->d_inst);
    for (BTileList *L : {&b->all, &b->three, &b->fused}) {
        if (L->d) dev_free(c, L->d);
        if (L->dn) dev_free(c, L->dn);
        if (L->h) (void)hipHostFree(L->h);
        if (L->hn) (void)hipHostFree(L->hn);
    }
    if (b->d_part) dev_free(c, b->d_part);
    if (b->h_inst) (void)hipHostFree(b->h_inst);
    if (b->stage) (void)hipHostFree(b->stage);
    delete b;
    return TC_OK;
}

extern "C" {

tc_status tc_batch_create(tc_ctx *ctx, const tc_batch_opts *opts, tc_batch **out) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_batch_create(ctx, opts, out); });
}

tc_status tc_batch_submit(tc_batch *b, const tc_solve_desc *d, int64_t *ticket) {
    return tc::guard_abi(batch_ctx(b), [&] { return impl_tc_batch_submit(b, d, ticket); });
}

tc_status tc_batch_step(tc_batch *b, int32_t *unfinished) {
    return tc::guard_abi(batch_ctx(b), [&] { return impl_tc_batch_step(b, unfinished); });
}

tc_status tc_batch_poll(tc_batch *b, int64_t ticket, tc_solve_result *out) {
    return tc::guard_abi(batch_ctx(b), [&] { return impl_tc_batch_poll(b, ticket, out); });
}

tc_status tc_batch_wait(tc_batch *b) {
    return tc::guard_abi(batch_ctx(b), [&] { return impl_tc_batch_wait(b); });
}

tc_status tc_batch_read_x(tc_batch *b, int64_t ticket, double *host, int64_t cap) {
    return tc::guard_abi(batch_ctx(b), [&] { return impl_tc_batch_read_x(b, ticket, host, cap); });
}

tc_status tc_batch_destroy(tc_batch *b) {
    return tc::guard_abi(batch_ctx(b), [&] { return impl_tc_batch_destroy(b); });
}

}  // extern "C"
