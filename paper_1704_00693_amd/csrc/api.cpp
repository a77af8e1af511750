// C ABI of tilechain: declarations, the delayed-execution recorder (Section
// 4.1), validation, flush (plan lookup, execution, reductions) and data
// access.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "fused.hpp"
#include "kernels.hpp"
#include "tc_internal.hpp"

using namespace tc;

namespace tc {

// Device scratch of the calls that allocate nothing (tc_reduction_result_static):
// reduction partials followed by the finalised (hi, lo) pairs.  One copy per
// device, held until the process ends; its device address is looked up once
// per device (hipGetSymbolAddress) when a context is created on that device.
constexpr int64_t kScratchDoubles = 1 << 17;  // 1 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double *g_scratch_ptr[kMaxDevices];

// Called with the context's device current.
tc_status bind_scratch(Ctx &c) {
    if (c.device < 0 || c.device >= kMaxDevices) return fail(c, TC_ERR_UNSUPPORTED, "device ordinal above %d", kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[c.device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(c, TC_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[c.device] = (double *)ptr;
    }
    c.scratch = g_scratch_ptr[c.device];
    return TC_OK;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

tc_status fail(Ctx &c, tc_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c.last_error = buf;
    if (s == TC_ERR_DEVICE) c.poisoned = true;
    return s;
}

#define HIPCHK(c, expr)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail((c), TC_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

#define CHECK_CTX(ctx)                                   \
    do {                                                 \
        if (!(ctx)) return TC_ERR_ARG;                   \
        if ((ctx)->c.poisoned) return TC_ERR_DEVICE;     \
    } while (0)

void *dev_alloc(Ctx &c, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (c.alloc) return c.alloc(bytes, c.alloc_user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(Ctx &c, void *p) {
    if (!p) return;
    if (c.free)
        c.free(p, c.alloc_user);
    else
        (void)hipFree(p);
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// op signatures
// ---------------------------------------------------------------------------
struct Sig {
    int ndat_min, ndat_max;  // dataset arguments
    int nred;                // reduction arguments
    int red_op;              // required reduction op (-1: any)
    int nparams;             // -1: computed (WSUM)
};

bool op_sig(int op, int ndim, Sig &s) {
    switch (op) {
    case TC_OP_WSUM: s = {2, kMaxArgs, 0, -1, -1}; return true;
    case TC_OP_COPY: s = {2, 2, 0, -1, 0}; return true;
    case TC_OP_AXPBY: s = {2, 2, 0, -1, 2}; return true;
    case TC_OP_DOT: s = {2, 2, 1, TC_RED_SUM, 0}; return true;
    case TC_OP_SUM: s = {1, 1, 1, TC_RED_SUM, 0}; return true;
    case TC_OP_HALO_REFLECT: s = {1, 1, 0, -1, 3}; return true;
    case TC_OP_TEA_INIT: s = {4, 4, 0, -1, 0}; return true;
    case TC_OP_TEA_K: s = {1 + ndim, 1 + ndim, 0, -1, 1}; return true;
    case TC_OP_TEA_RESID: s = {ndim + 3, ndim + 3, 0, -1, 0}; return true;
    case TC_OP_TEA_MATVEC_DOT: s = {ndim + 2, ndim + 2, 1, TC_RED_SUM, 0}; return true;
    case TC_OP_TEA_P1: s = {ndim + 3, ndim + 3, 0, -1, 0}; return true;
    case TC_OP_TEA_P2: s = {2, 2, 0, -1, 2}; return true;
    case TC_OP_TEA_PRECON_INIT: s = {4, 4, 0, -1, 1}; return true;
    case TC_OP_TEA_CG_UPDATE: s = {4, 4, 0, -1, 1}; return true;
    case TC_OP_TEA_CG_P: s = {2, 2, 0, -1, 1}; return true;
    case TC_OP_TEA_GERSH: s = {ndim, ndim, 1, TC_RED_MAX, 0}; return true;
    case TC_OP_EULER_PRIM: s = {2 * ndim + 3, 2 * ndim + 3, 0, -1, 1}; return true;
    case TC_OP_EULER_RHS: s = {ndim + 3, ndim + 3, 0, -1, 2}; return true;
    case TC_OP_RK_STAGE: s = {3, 3, 0, -1, 3}; return true;
    default: return false;
    }
}

// Required access of dataset argument i of an op (-1: any read-only).
int op_access(int op, int ndim, int i) {
    const int R = TC_READ, W = TC_WRITE, RW = TC_RW;
    switch (op) {
    case TC_OP_WSUM: return i == 0 ? W : R;
    case TC_OP_COPY: return i == 0 ? W : R;
    case TC_OP_AXPBY: return i == 0 ? RW : R;
    case TC_OP_DOT:
    case TC_OP_SUM: return R;
    case TC_OP_HALO_REFLECT: return RW;
    case TC_OP_TEA_INIT: return i < 2 ? R : W;
    case TC_OP_TEA_K: return i == 0 ? R : W;
    case TC_OP_TEA_RESID: return i < ndim + 2 ? R : W;
    case TC_OP_TEA_MATVEC_DOT: return i <= ndim ? R : W;
    case TC_OP_TEA_P1: return i <= ndim ? R : RW;
    case TC_OP_TEA_P2: return i == 0 ? RW : R;
    case TC_OP_TEA_PRECON_INIT: return i == 0 ? R : W;
    case TC_OP_TEA_CG_UPDATE: return i < 2 ? RW : R;
    case TC_OP_TEA_CG_P: return i == 0 ? RW : R;
    case TC_OP_TEA_GERSH: return R;
    case TC_OP_EULER_PRIM: return i < ndim + 2 ? R : W;
    case TC_OP_EULER_RHS: return i == 0 ? W : R;
    case TC_OP_RK_STAGE: return i == 1 ? RW : R;
    default: return -2;
    }
}

// Points the op's kernel reads from dataset argument i, as a box of offsets
// per dimension; the declared stencil must cover it (so the range check on
// the declared stencil bounds every access).  Returns false for "exactly the
// declared points" (WSUM) and the reflect op (checked separately).
bool op_footprint(int op, int ndim, int i, int lo[3], int hi[3]) {
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = 0;
    switch (op) {
    case TC_OP_WSUM:
    case TC_OP_HALO_REFLECT: return false;
    case TC_OP_TEA_K:
        if (i == 0)
            for (int d = 0; d < ndim; ++d) lo[d] = -1;
        return true;
    case TC_OP_TEA_RESID:
    case TC_OP_TEA_MATVEC_DOT:
    case TC_OP_TEA_P1:
    case TC_OP_TEA_GERSH:
        if (i < ndim) {
            hi[i] = 1;
        } else if (i == ndim && op != TC_OP_TEA_GERSH) {
            for (int d = 0; d < ndim; ++d) {
                lo[d] = -1;
                hi[d] = 1;
            }
        }
        return true;
    case TC_OP_EULER_RHS:
        if (i > 0)
            for (int d = 0; d < ndim; ++d) {
                lo[d] = -2;
                hi[d] = 2;
            }
        return true;
    default: return true;
    }
}

bool access_ok(int want, int got) {
    if (want == TC_RW) return got == TC_RW || got == TC_INC;
    return want == got;
}

// ---------------------------------------------------------------------------
// device resources for reductions
// ---------------------------------------------------------------------------
tc_status ensure_partials(Ctx &c, int64_t pairs, int nslots) {
    if (c.noalloc) {
        // partials at the start of the scratch array, the outputs after them;
        // laid out by the flush's first call (its plan's partial count), kept
        // by later calls that only ask for the outputs
        if (pairs == 0 && c.red_out && c.red_out_cap >= 2 * (int64_t)nslots) return TC_OK;
        const int64_t need = 2 * pairs + 2 * (int64_t)nslots;
        if (need > kScratchDoubles)
            return fail(c, TC_ERR_ARG,
                        "this chain's reductions need %lld doubles of scratch (%lld partials, %d results); the static "
                        "scratch holds %lld",
                        (long long)need, (long long)pairs, nslots, (long long)kScratchDoubles);
        c.partials = c.scratch;
        c.partials_cap = 2 * pairs;
        c.red_out = c.scratch + 2 * pairs;
        c.red_out_cap = 2 * (int64_t)nslots;
        return TC_OK;
    }
    if (pairs * 2 > c.partials_cap) {
        dev_free(c, c.partials);
        int64_t cap = std::max<int64_t>(pairs * 2, 1 << 16);
        c.partials = (double *)dev_alloc(c, cap * sizeof(double));
        if (!c.partials) {
            c.partials_cap = 0;
            return fail(c, TC_ERR_NOMEM, "cannot allocate %lld reduction partials", (long long)cap);
        }
        c.partials_cap = cap;
    }
    if (nslots * 2 > c.red_out_cap) {
        dev_free(c, c.red_out);
        if (c.red_host) (void)hipHostFree(c.red_host);
        int64_t cap = std::max<int64_t>(nslots * 2, 64);
        c.red_out = (double *)dev_alloc(c, cap * sizeof(double));
        if (!c.red_out) return fail(c, TC_ERR_NOMEM, "cannot allocate reduction outputs");
        // coherent: the combining kernel's stores reach host memory, not
        // the GPU's caches, and are visible once the stream is synchronised
        HIPCHK(c, hipHostMalloc((void **)&c.red_host, cap * sizeof(double), hipHostMallocCoherent));
        HIPCHK(c, hipHostGetDevicePointer((void **)&c.red_host_dev, c.red_host, 0));
        c.red_out_cap = cap;
    }
    return TC_OK;
}

// ---------------------------------------------------------------------------
// descriptors
// ---------------------------------------------------------------------------
void build_desc(const Ctx &c, const LoopRec &lp, LoopDesc &d) {
    std::memset(&d, 0, sizeof d);
    d.op = lp.op;
    d.ndim = lp.ndim;
    int na = 0, q = 0, nr = 0;
    for (const auto &a : lp.args) {
        if (a.kind == TC_ARG_RED) {
            d.red_op[nr++] = c.reds[a.handle].op;
            continue;
        }
        const Dataset &ds = c.dats[a.handle];
        const Stencil &st = c.stencils[a.stencil];
        d.arg[na].ptr = ds.origin(ds.cur);
        d.arg[na].sy = ds.sy();
        d.arg[na].sz = ds.sz();
        d.npts[na] = st.npoints();
        d.pt0[na] = q;
        for (int k = 0; k < st.npoints(); ++k) d.qarg[q + k] = (unsigned char)na;
        for (int k = 0; k < st.npoints(); ++k, ++q)
            d.off[q] = (int64_t)st.pts[3 * k] + (int64_t)st.pts[3 * k + 1] * ds.sy() +
                       (int64_t)st.pts[3 * k + 2] * ds.sz();
        ++na;
    }
    d.nargs = na;
    d.nred = nr;
    if (lp.op == TC_OP_WSUM) {
        // weights aligned with the stencil points of the inputs
        int w = 0;
        for (int a = 1; a < na; ++a)
            for (int k = 0; k < d.npts[a]; ++k) d.prm[d.pt0[a] + k] = lp.params[w++];
    } else {
        for (size_t i = 0; i < lp.params.size(); ++i) d.prm[i] = lp.params[i];
    }
}

// Radius of a 2D star stencil listed in the canonical order (centre, -x, +x,
// [-2x, +2x,] -y, +y, [-2y, +2y]), or -1.
int canonical_star2(const Stencil &st) {
    static const int r1[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};
    static const int r2[9][2] = {{0, 0}, {-1, 0}, {1, 0}, {-2, 0}, {2, 0}, {0, -1}, {0, 1}, {0, -2}, {0, 2}};
    if (st.ndim != 2) return -1;
    const int n = st.npoints();
    if (n != 5 && n != 9) return -1;
    for (int p = 0; p < n; ++p) {
        const int *w = n == 5 ? r1[p] : r2[p];
        if (st.pts[3 * p] != w[0] || st.pts[3 * p + 1] != w[1]) return -1;
    }
    return n == 5 ? 1 : 2;
}

// Radius mask for the register-window weighted-sum kernel, or -1.
// Radius of a 3D star stencil listed in the canonical order (centre, then
// per axis x, y, z the offsets -1, +1[, -2, +2]), or -1.
int canonical_star3(const Stencil &st) {
    if (st.ndim != 3) return -1;
    const int n = st.npoints();
    if (n != 7 && n != 13) return -1;
    const int r = n == 7 ? 1 : 2;
    int q = 0;
    if (st.pts[0] != 0 || st.pts[1] != 0 || st.pts[2] != 0) return -1;
    ++q;
    for (int ax = 0; ax < 3; ++ax)
        for (int d = 1; d <= r; ++d)
            for (int sgn : {-1, 1}) {
                for (int k = 0; k < 3; ++k)
                    if (st.pts[3 * q + k] != (k == ax ? sgn * d : 0)) return -1;
                ++q;
            }
    return r;
}

int march_mask_of(const Ctx &c, const LoopRec &lp) {
    if (lp.op == TC_OP_EULER_RHS) return lp.ndim == 3 ? 0 : -1;  // the z-marching 3D kernel
    if (lp.op != TC_OP_WSUM || (lp.ndim != 2 && lp.ndim != 3) || lp.args.size() > 5) return -1;
    if (!c.stencils[lp.args[0].stencil].centre_only() || c.stencils[lp.args[0].stencil].npoints() != 1) return -1;
    int mask = 0;
    for (size_t a = 1; a < lp.args.size(); ++a) {
        const Stencil &st = c.stencils[lp.args[a].stencil];
        const int r = lp.ndim == 2 ? canonical_star2(st) : canonical_star3(st);
        if (r < 0) return -1;
        if (r == 2) mask |= 1 << (a - 1);
    }
    return mask;
}

int dat_dtype(const Ctx &c, const LoopRec &lp, int which) {
    int k = 0;
    for (const auto &a : lp.args)
        if (a.kind == TC_ARG_DAT) {
            if (k == which) return c.dats[a.handle].dtype;
            ++k;
        }
    return TC_F64;
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
void add_launch(const Ctx &c, const LoopRec &lp, int l, const int lo[3], const int hi[3],
                std::shared_ptr<CachedPlan> &P, std::vector<int64_t> &slot_used) {
    for (int d = 0; d < 3; ++d)
        if (hi[d] <= lo[d]) return;
    Launch L;
    L.loop = l;
    for (int d = 0; d < 3; ++d) {
        L.lo[d] = lo[d];
        L.hi[d] = hi[d];
    }
    Box b = make_box(lp.ndim, lo, hi);
    L.nb = b.nb;
    int j = 0;
    L.part_off[0] = L.part_off[1] = 0;
    for (const auto &a : lp.args) {
        if (a.kind != TC_ARG_RED) continue;
        int slot = (int)(std::find(P->red_handles.begin(), P->red_handles.end(), a.handle) - P->red_handles.begin());
        L.part_off[j++] = slot;  // temporarily the slot; fixed up below
        slot_used[slot] += b.nb;
    }
    P->steps.push_back({0, (int)P->launches.size()});
    P->launches.push_back(L);
}

void finish_partials(const Ctx &c, const std::vector<LoopRec> &chain, std::shared_ptr<CachedPlan> &P,
                     const std::vector<int64_t> &slot_used) {
    const size_t ns = P->red_handles.size();
    P->red_base.assign(ns, 0);
    P->red_count.assign(ns, 0);
    int64_t tot = 0;
    for (size_t s = 0; s < ns; ++s) {
        P->red_base[s] = tot;
        tot += slot_used[s];
    }
    P->partials_total = tot;
    std::vector<int64_t> fill(ns, 0);
    for (const Step &st : P->steps) {
        if (st.kind == 0) {
            Launch &L = P->launches[st.index];
            const LoopRec &lp = chain[L.loop];
            int j = 0;
            for (const auto &a : lp.args) {
                if (a.kind != TC_ARG_RED) continue;
                int slot = (int)L.part_off[j];
                L.part_off[j] = P->red_base[slot] + fill[slot];
                fill[slot] += L.nb;
                ++j;
            }
        } else if (auto S = P->groups[st.index]->staged) {
            for (int k = S->g0; k < S->g1; ++k) {
                int j = 0;
                for (const auto &a : chain[k].args) {
                    if (a.kind != TC_ARG_RED) continue;
                    const int slot = (int)S->loops[k - S->g0].part[j];
                    S->loops[k - S->g0].part[j++] = P->red_base[slot] + fill[slot];
                    fill[slot] += S->ntot;
                }
            }
        }
    }
    for (size_t s = 0; s < ns; ++s) P->red_count[s] = fill[s];
    (void)c;
}

std::shared_ptr<CachedPlan> build_plan(Ctx &c, const std::vector<LoopRec> &chain, tc_tiling mode,
                                       const int tile[3], int cpl) {
    auto P = std::make_shared<CachedPlan>();
    P->mode = mode;
    for (const auto &lp : chain)
        for (const auto &a : lp.args)
            if (a.kind == TC_ARG_RED &&
                std::find(P->red_handles.begin(), P->red_handles.end(), a.handle) == P->red_handles.end())
                P->red_handles.push_back(a.handle);
    std::vector<int64_t> used(P->red_handles.size(), 0);
    if (mode == TC_TILING_SKEWED) {
        P->skewed = build_skewed_plan(c, chain, tile);
        const SkewedPlan &S = P->skewed;
        const int L = (int)chain.size();
        for (int d = 0; d < S.ndim; ++d) {
            int best = 0;
            for (int t = 0; t + 1 < S.num_tiles[d]; ++t) {
                int mn = INT32_MAX, mx = INT32_MIN;
                for (int l = 0; l < L; ++l) {
                    mn = std::min(mn, S.e(d, t, l));
                    mx = std::max(mx, S.e(d, t, l));
                }
                best = std::max(best, mx - mn);
            }
            P->max_skew[d] = best;
        }
        // tiles in lexicographic order, slowest dimension outermost
        const int T0 = S.num_tiles[0], T1 = S.ndim > 1 ? S.num_tiles[1] : 1, T2 = S.ndim > 2 ? S.num_tiles[2] : 1;
        for (int t2 = 0; t2 < T2; ++t2)
            for (int t1 = 0; t1 < T1; ++t1)
                for (int t0 = 0; t0 < T0; ++t0)
                    for (int l = 0; l < L; ++l) {
                        int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
                        int tt[3] = {t0, t1, t2};
                        for (int d = 0; d < S.ndim; ++d) {
                            lo[d] = S.s(d, tt[d], l);
                            hi[d] = S.e(d, tt[d], l);
                        }
                        add_launch(c, chain[l], l, lo, hi, P, used);
                    }
    } else if (mode == TC_TILING_FUSED) {
        P->groups = fused_split(c, chain, tile, cpl);
        size_t gi = 0;
        for (int l = 0; l < (int)chain.size();) {
            if (gi < P->groups.size() && P->groups[gi]->g0 == l) {
                P->steps.push_back({1, (int)gi});
                if (auto S = P->groups[gi]->staged) {
                    // one partial per tile for every reduction argument (the
                    // slot for now; finish_partials turns it into an offset)
                    for (int k = S->g0; k < S->g1; ++k) {
                        int j = 0;
                        for (const auto &a : chain[k].args) {
                            if (a.kind != TC_ARG_RED) continue;
                            const int slot = (int)(std::find(P->red_handles.begin(), P->red_handles.end(), a.handle) -
                                                   P->red_handles.begin());
                            S->loops[k - S->g0].part[j++] = slot;
                            used[slot] += S->ntot;
                        }
                    }
                }
                l = P->groups[gi]->g1;
                ++gi;
            } else {
                add_launch(c, chain[l], l, chain[l].lo, chain[l].hi, P, used);
                ++l;
            }
        }
    } else {
        for (int l = 0; l < (int)chain.size(); ++l) add_launch(c, chain[l], l, chain[l].lo, chain[l].hi, P, used);
    }
    finish_partials(c, chain, P, used);
    return P;
}

// ---------------------------------------------------------------------------
// flush
// ---------------------------------------------------------------------------
// Extend the hull of points ever written of every dataset the loop writes.
void note_loop_writes(Ctx &c, const LoopRec &lp) {
    if (lp.points() == 0) return;
    for (const auto &a : lp.args) {
        if (!a.writes()) continue;
        Dataset &ds = c.dats[a.handle];
        for (int d = 0; d < 3; ++d) {
            ds.wlo[d] = ds.ever_written ? std::min(ds.wlo[d], lp.lo[d]) : lp.lo[d];
            ds.whi[d] = ds.ever_written ? std::max(ds.whi[d], lp.hi[d]) : lp.hi[d];
        }
        ds.ever_written = true;
    }
}

tc_status ensure_events(Ctx &c, size_t n) {
    while (c.events.size() < n) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c.events.push_back(e);
    }
    return TC_OK;
}

uint64_t fnv(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Per-loop schedules (no fused groups): launch directly, or capture the
// launches into a graph and replay it when the arguments repeat.
tc_status run_per_loop_graph(Ctx &c, const std::vector<LoopRec> &chain, CachedPlan &P, bool &done) {
    done = false;
    std::vector<LoopDesc> descs(chain.size());
    std::vector<int> march(chain.size());
    for (size_t l = 0; l < chain.size(); ++l) {
        build_desc(c, chain[l], descs[l]);
        march[l] = c.march_enabled ? march_mask_of(c, chain[l]) : -1;
    }
    struct Item {
        LoopDesc d;
        Box b;
        int t0, t1, mm;
    };
    std::vector<Item> items;
    items.reserve(P.launches.size());
    uint64_t h = 1469598103934665603ull;
    for (const auto &L : P.launches) {
        Item it;
        it.d = descs[L.loop];
        for (int j = 0; j < it.d.nred; ++j) it.d.partials[j] = c.partials + 2 * L.part_off[j];
        it.b = make_box(chain[L.loop].ndim, L.lo, L.hi);
        it.t0 = dat_dtype(c, chain[L.loop], 0);
        it.t1 = dat_dtype(c, chain[L.loop], 1);
        it.mm = march[L.loop];
        h = fnv(h, &it.d, sizeof(LoopDesc));
        h = fnv(h, &it.b, sizeof(Box));
        h = fnv(h, &it.t0, 3 * sizeof(int));
        items.push_back(it);
    }
    h = fnv(h, &c.march, sizeof(MarchShape));
    if (P.gexec && P.ghash == h) {
        HIPCHK(c, hipGraphLaunch(P.gexec, c.stream));
        done = true;
        return TC_OK;
    }
    hipStream_t s = c.stream;
    const bool capture = P.ghash_prev == h;
    P.ghash_prev = h;
    if (capture) {
        if (!c.cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
        HIPCHK(c, hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal));
        s = c.cap_stream;
    }
    hipError_t err = hipSuccess;
    for (const auto &it : items) {
        err = launch_loop(it.d, it.b, it.t0, it.t1, it.mm, c.march, s);
        if (err != hipSuccess) break;
    }
    if (capture) {
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(c.cap_stream, &graph);
        if (err == hipSuccess) err = e2;
        if (err == hipSuccess) {
            if (P.gexec) (void)hipGraphExecDestroy(P.gexec);
            P.gexec = nullptr;
            err = hipGraphInstantiate(&P.gexec, graph, nullptr, nullptr, 0);
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (err == hipSuccess) {
            P.ghash = h;
            err = hipGraphLaunch(P.gexec, c.stream);
        }
    }
    if (err != hipSuccess) return fail(c, TC_ERR_DEVICE, "per-loop launch failed: %s", hipGetErrorString(err));
    done = true;
    return TC_OK;
}

tc_status run_launches(Ctx &c, const std::vector<LoopRec> &chain, CachedPlan &P) {
    if (c.use_graphs && !c.profiling && P.groups.empty() && P.launches.size() >= 2) {
        bool done = false;
        tc_status st = run_per_loop_graph(c, chain, P, done);
        if (st != TC_OK) return st;
        if (done) {
            for (const auto &L : P.launches) note_loop_writes(c, chain[L.loop]);
            return TC_OK;
        }
    }
    std::vector<LoopDesc> descs(chain.size());
    std::vector<char> built(chain.size(), 0);
    std::vector<int> march(chain.size());
    for (size_t l = 0; l < chain.size(); ++l) march[l] = c.march_enabled ? march_mask_of(c, chain[l]) : -1;
    if (c.profiling) {
        tc_status st = ensure_events(c, 2 * P.steps.size());
        if (st != TC_OK) return st;
    }
    size_t i = 0;
    for (const auto &S : P.steps) {
        if (c.profiling) HIPCHK(c, hipEventRecord(c.events[2 * i], c.stream));
        if (S.kind == 0) {
            const Launch &L = P.launches[S.index];
            if (!built[L.loop]) {  // descriptors see the buffers current at this point
                build_desc(c, chain[L.loop], descs[L.loop]);
                built[L.loop] = 1;
            }
            LoopDesc d = descs[L.loop];
            for (int j = 0; j < d.nred; ++j) d.partials[j] = c.partials + 2 * L.part_off[j];
            Box b = make_box(chain[L.loop].ndim, L.lo, L.hi);
            HIPCHK(c, launch_loop(d, b, dat_dtype(c, chain[L.loop], 0), dat_dtype(c, chain[L.loop], 1),
                                  march[L.loop], c.march, c.stream));
            note_loop_writes(c, chain[L.loop]);
        } else {
            const FusedGroup &G = *P.groups[S.index];
            tc_status st = fused_run(c, chain, *P.groups[S.index]);
            if (st != TC_OK) return st;
            for (int l = G.g0; l < G.g1; ++l) note_loop_writes(c, chain[l]);
            std::fill(built.begin(), built.end(), 0);  // buffers were swapped
        }
        if (c.profiling) HIPCHK(c, hipEventRecord(c.events[2 * i + 1], c.stream));
        ++i;
    }
    if (c.profiling) {
        HIPCHK(c, hipStreamSynchronize(c.stream));
        double tot = 0.0, fused = 0.0;
        for (size_t k = 0; k < i; ++k) {
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, c.events[2 * k], c.events[2 * k + 1]));
            tot += ms * 1e-3;
            if (P.steps[k].kind == 1) fused += ms * 1e-3;
        }
        c.stats.prof_kernel_seconds = tot;
        c.stats.prof_fused_seconds = fused;
        c.stats.prof_launches = (int64_t)i;
    }
    return TC_OK;
}

tc_status flush(Ctx &c) {
    if (c.poisoned) return TC_ERR_DEVICE;
    if (c.chain.empty()) return TC_OK;
    if (c.host_only) return fail(c, TC_ERR_STATE, "host-only context cannot execute loops");
    const double t0 = now_s();
    std::vector<LoopRec> chain;
    chain.swap(c.chain);

    tc_tiling mode = c.mode;
    int tile[3] = {c.tile[0], c.tile[1], c.tile[2]};
    int cpl = c.jit_cpl;
    const bool tuning_flush = mode == TC_TILING_AUTO && !c.noalloc;
    if (mode == TC_TILING_AUTO && c.noalloc) {
        TuneCand k;
        if (!autotune_lookup(c, chain, k)) {
            c.chain.swap(chain);
            return fail(c, TC_ERR_STATE,
                        "the autotuner has not chosen a schedule for this chain yet (its measurement flushes "
                        "allocate); flush it with tc_flush until it has");
        }
        mode = k.mode;
        for (int d = 0; d < 3; ++d) tile[d] = k.tile[d];
        cpl = k.cpl;
    }
    if (tuning_flush) {
        const TuneCand k = autotune_choose(c, chain);
        mode = k.mode;
        for (int d = 0; d < 3; ++d) tile[d] = k.tile[d];
        cpl = k.cpl;
    }

    tc_status st = TC_OK;
    int64_t bytes = 0, cells = 0;
    for (const auto &lp : chain) {
        cells += lp.points();
        for (const auto &a : lp.args)
            if (a.kind == TC_ARG_DAT)
                bytes += lp.points() * (int64_t)c.dats[a.handle].esize() *
                         ((a.access == TC_RW || a.access == TC_INC) ? 2 : 1);
    }

    std::vector<int> red_handles;
    std::vector<int64_t> red_base, red_count;
    int launches = 0, tiles = 0, groups = 0;
    {
        const uint64_t key = chain_key(c, chain, mode, tile, cpl);
        std::shared_ptr<CachedPlan> P;
        auto it = c.plans.find(key);
        if (it != c.plans.end()) {
            P = it->second;
            c.stats.plan_hits++;
        } else if (c.noalloc && mode == TC_TILING_FUSED) {
            c.chain.swap(chain);
            return fail(c, TC_ERR_STATE,
                        "no cached fused plan for this chain: its kernels must be compiled and loaded, which a call "
                        "that allocates nothing cannot do; flush it once with tc_flush first");
        } else {
            const double pb = now_s();
            P = build_plan(c, chain, mode, tile, cpl);
            if (mode == TC_TILING_FUSED) {
                st = fused_compile(c, chain, P->groups);
                if (st != TC_OK) return st;
            }
            P->build_seconds = now_s() - pb;
            c.stats.plan_seconds += P->build_seconds;
            c.stats.plan_misses++;
            c.plans[key] = P;
        }
        st = ensure_partials(c, P->partials_total, (int)P->red_handles.size());
        if (st == TC_OK && c.noalloc)
            for (const auto &g : P->groups)
                if ((st = fused_check_noalloc(c, chain, *g)) != TC_OK) break;
        if (st != TC_OK) {
            if (c.noalloc) c.chain.swap(chain);  // nothing ran: the chain stays pending
            return st;
        }
        if (tuning_flush && c.tune_cand >= 0) {  // the candidate's device time, plan work excluded
            for (auto &e : c.tune_ev)
                if (!e) HIPCHK(c, hipEventCreate(&e));
            HIPCHK(c, hipEventRecord(c.tune_ev[0], c.stream));
        }
        st = run_launches(c, chain, *P);
        if (st != TC_OK) return st;
        red_handles = P->red_handles;
        red_base = P->red_base;
        red_count = P->red_count;
        launches = (int)P->steps.size();
        tiles = P->skewed.num_tiles[0] * P->skewed.num_tiles[1] * P->skewed.num_tiles[2];
        groups = (int)P->groups.size();
        c.stats.fused_bytes = 0;
        if (mode == TC_TILING_FUSED) {
            tiles = 0;
            for (auto &g : P->groups) {
                tiles += g->nblocks;
                c.stats.fused_bytes += g->alg_bytes;
            }
        }
        for (int d = 0; d < 3; ++d) c.stats.max_skew[d] = P->max_skew[d];
    }

    if (!red_handles.empty()) {
        st = ensure_partials(c, 0, (int)red_handles.size());
        if (st != TC_OK) return st;
        std::vector<double> host_out(c.noalloc ? 2 * red_handles.size() : 0);
        double *dst = c.noalloc ? host_out.data() : c.red_host;
        std::vector<int> ops(red_handles.size());
        for (size_t s = 0; s < red_handles.size(); ++s) ops[s] = c.reds[red_handles[s]].op;
        if (c.noalloc) {
            // the results go to the scratch array and are copied from there
            HIPCHK(c, launch_finalize_many(c.partials, red_base.data(), red_count.data(), ops.data(),
                                           (int)red_handles.size(), c.red_out, c.stream));
            HIPCHK(c, hipMemcpyAsync(dst, c.red_out, red_handles.size() * 2 * sizeof(double),
                                     hipMemcpyDeviceToHost, c.stream));
        } else {
            // one launch combines every reduction's partials straight into
            // the pinned host results: no copy
            HIPCHK(c, launch_finalize_many(c.partials, red_base.data(), red_count.data(), ops.data(),
                                           (int)red_handles.size(), c.red_host_dev, c.stream));
        }
        HIPCHK(c, hipStreamSynchronize(c.stream));
        for (size_t s = 0; s < red_handles.size(); ++s) {
            Reduction &r = c.reds[red_handles[s]];
            const double hi = dst[2 * s], lo = dst[2 * s + 1];
            if (r.op == TC_RED_SUM) {
                double sum = r.hi + hi;
                double bb = sum - r.hi;
                double e = (r.hi - (sum - bb)) + (hi - bb);
                r.hi = sum;
                r.lo += lo + e;
            } else if (!r.touched) {
                r.hi = hi;
            } else {
                r.hi = r.op == TC_RED_MIN ? std::min(r.hi, hi) : std::max(r.hi, hi);
            }
            r.touched = true;
        }
    }
    if (tuning_flush && c.tune_cand >= 0) {
        HIPCHK(c, hipEventRecord(c.tune_ev[1], c.stream));
        HIPCHK(c, hipEventSynchronize(c.tune_ev[1]));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c.tune_ev[0], c.tune_ev[1]));
        autotune_record(c, ms * 1e-3);
        autotune_finish(c, chain);
    }
    c.stats.flushes++;
    c.stats.last_launches = launches;
    c.stats.last_tiles = tiles;
    c.stats.last_groups = groups;
    c.stats.last_mode = mode;
    for (int d = 0; d < 3; ++d) c.stats.last_tile[d] = tile[d];
    c.stats.last_cpl = cpl;
    c.stats.tuning = tuning_flush && c.tuned[autotune_key(c, chain)].best < 0 ? 1 : 0;
    c.stats.modelled_bytes = bytes;
    c.stats.cell_updates = cells;
    c.stats.last_flush_seconds = now_s() - t0;
    return TC_OK;
}

tc_status copy_host(Ctx &c, Dataset &ds, void *host, const void *src, int which, bool to_device) {
    const int64_t nxa = (int64_t)ds.size[0] + ds.hneg[0] + ds.hpos[0];
    const size_t es = ds.esize();
    const size_t width = nxa * es;
    const size_t dpitch = ds.pitch * es;
    char *dev = (char *)ds.buf[which] + (ds.xorg - ds.hneg[0]) * (int64_t)es;
    for (int64_t z = 0; z < ds.nz_alloc; ++z) {
        char *dplane = dev + z * ds.ny_alloc * dpitch;
        const int64_t hoff = z * ds.ny_alloc * width;
        if (to_device)
            HIPCHK(c, hipMemcpy2DAsync(dplane, dpitch, (const char *)src + hoff, width, width, ds.ny_alloc,
                                       hipMemcpyHostToDevice, c.stream));
        else
            HIPCHK(c, hipMemcpy2DAsync((char *)host + hoff, width, dplane, dpitch, width, ds.ny_alloc,
                                       hipMemcpyDeviceToHost, c.stream));
    }
    HIPCHK(c, hipStreamSynchronize(c.stream));
    return TC_OK;
}

}  // namespace tc

// ===========================================================================
// C ABI
// ===========================================================================
// Bodies of the C ABI calls; the exported wrappers below turn any C++
// exception into a status code.

static tc_status impl_tc_init(const tc_init_opts *opts, tc_ctx **out) {
    if (!out) return TC_ERR_ARG;
    *out = nullptr;
    tc_ctx *ctx = new (std::nothrow) tc_ctx();
    if (!ctx) return TC_ERR_NOMEM;
    Ctx &c = ctx->c;
    if (opts) {
        c.device = opts->device;
        c.host_only = (opts->flags & TC_INIT_HOST_ONLY) != 0;
        c.stream = (hipStream_t)opts->stream;
        c.alloc = opts->alloc;
        c.free = opts->free;
        c.alloc_user = opts->alloc_user;
        if ((c.alloc == nullptr) != (c.free == nullptr)) {
            delete ctx;
            return TC_ERR_ARG;
        }
    }
    if (const char *e = getenv("TC_WSUM_MARCH")) c.march_enabled = atoi(e) != 0;
    if (const char *e = getenv("TC_MARCH_TY")) c.march.ty = std::max(1, atoi(e));
    if (const char *e = getenv("TC_MARCH3_ROWS")) {
        const int v = atoi(e);
        if (v == 4 || v == 8) c.march.rows3 = v;
    }
    if (const char *e = getenv("TC_MARCH3_TZ")) c.march.tz3 = std::min(512, std::max(0, atoi(e) / 4 * 4));
    if (const char *e = getenv("TC_GRAPHS")) c.use_graphs = atoi(e) != 0;
    if (const char *e = getenv("TC_STAGGER")) c.stagger_unit = std::max(0ll, atoll(e)) / 256 * 256;
    if (const char *e = getenv("TC_JIT_UNROLL")) c.jit_unroll = std::min(16, std::max(1, atoi(e)));
    if (const char *e = getenv("TC_JIT_PREFETCH")) c.jit_prefetch = std::min(8, std::max(1, atoi(e)));
    if (const char *e = getenv("TC_JIT_BAKE")) c.jit_bake = atoi(e) != 0;
    if (const char *e = getenv("TC_JIT_TEST_SHORT_WINDOWS")) c.jit_test_short_windows = atoi(e) != 0;
    if (const char *e = getenv("TC_JIT_CPL")) c.jit_cpl = atoi(e) == 2 ? 2 : 1;
    if (const char *e = getenv("TC_JIT_EDGE_DIV")) c.jit_edge_div = std::min(16, std::max(1, atoi(e)));
    if (const char *e = getenv("TC_JIT_WPE")) c.jit_wpe = std::min(8, std::max(0, atoi(e)));
    if (const char *e = getenv("TC_JIT_MAXWIN")) c.jit_max_window = std::max(0, atoi(e));
    if (const char *e = getenv("TC_JIT_CSE")) c.jit_cse_steps = atoi(e) != 0;
    if (const char *e = getenv("TC_JIT_FENCE")) c.jit_sched_fence = atoi(e) != 0;
    if (const char *e = getenv("TC_JIT_ALIGN")) c.jit_align_store = atoi(e) != 0;
    if (const char *e = getenv("TC_STAGED")) c.staged_mode = std::min(2, std::max(0, atoi(e)));
    if (const char *e = getenv("TC_CHEB")) c.cheb_enabled = atoi(e) != 0;
    if (const char *e = getenv("TC_CHEB_STEPS")) c.cheb_steps = std::min(kChebMaxSteps, std::max(1, atoi(e)));
    if (const char *e = getenv("TC_STAGED_THREADS")) {
        const int v = atoi(e);
        if (v == 256 || v == 1024) c.staged_threads = v;
    }
    if (const char *e = getenv("TC_STAGED_TILE")) {
        int v[3] = {0, 0, 0};
        if (std::sscanf(e, "%d,%d,%d", &v[0], &v[1], &v[2]) >= 1)
            for (int d = 0; d < 3; ++d) c.staged_tile[d] = std::max(0, v[d]);
    }
    if (!c.host_only) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || n <= 0 || c.device < 0 || c.device >= n) {
            delete ctx;
            return TC_ERR_DEVICE;
        }
        if (hipSetDevice(c.device) != hipSuccess) {
            delete ctx;
            return TC_ERR_DEVICE;
        }
        if (bind_scratch(c) != TC_OK) {
            delete ctx;
            return TC_ERR_DEVICE;
        }
        if (!c.stream && !(opts && (opts->flags & TC_INIT_BORROW_STREAM))) {
            if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess) {
                delete ctx;
                return TC_ERR_DEVICE;
            }
            c.own_stream = true;
        }
    }
    *out = ctx;
    return TC_OK;
}

static tc_status impl_tc_finalize(tc_ctx *ctx) {
    if (!ctx) return TC_OK;
    Ctx &c = ctx->c;
    tc_status st = TC_OK;
    if (!c.poisoned && !c.host_only) {
        st = flush(c);
        (void)hipStreamSynchronize(c.stream);
    }
    if (!c.host_only) {
        for (auto &d : c.dats) {
            dev_free(c, d.raw[0]);
            dev_free(c, d.raw[1]);
        }
        fused_release(c);
        for (auto &kv : c.plans)
            if (kv.second->gexec) (void)hipGraphExecDestroy(kv.second->gexec);
        if (c.cap_stream) (void)hipStreamDestroy(c.cap_stream);
        for (auto e : c.events) (void)hipEventDestroy(e);
        for (auto e : c.tune_ev)
            if (e) (void)hipEventDestroy(e);
        for (void *p : c.staged_allocs) dev_free(c, p);
        dev_free(c, c.partials);
        dev_free(c, c.red_out);
        if (c.red_host) (void)hipHostFree(c.red_host);
        if (c.own_stream) (void)hipStreamDestroy(c.stream);
    }
    delete ctx;
    return st;
}

static tc_status impl_tc_decl_block(tc_ctx *ctx, int ndim, const char *name, tc_block *out) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (ndim < 1 || ndim > 3 || !out) return fail(c, TC_ERR_ARG, "block dimension must be 1..3");
    c.blocks.push_back({ndim, name ? name : ""});
    *out = (tc_block)c.blocks.size() - 1;
    return TC_OK;
}

static tc_status impl_tc_decl_dat(tc_ctx *ctx, tc_block blk, tc_dtype dtype, const int32_t *size, const int32_t *halo_neg,
                      const int32_t *halo_pos, const void *host_init, const char *name, tc_dat *out) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (blk < 0 || blk >= (int)c.blocks.size() || !size || !out)
        return fail(c, TC_ERR_ARG, "tc_decl_dat: bad block or null argument");
    if (dtype != TC_F64 && dtype != TC_F32) return fail(c, TC_ERR_ARG, "tc_decl_dat: bad dtype");
    Dataset ds;
    ds.block = blk;
    ds.dtype = dtype;
    ds.ndim = c.blocks[blk].ndim;
    ds.name = name ? name : "";
    for (int d = 0; d < 3; ++d) {
        const bool used = d < ds.ndim;
        ds.size[d] = used ? size[d] : 1;
        ds.hneg[d] = used && halo_neg ? halo_neg[d] : 0;
        ds.hpos[d] = used && halo_pos ? halo_pos[d] : 0;
        if (ds.size[d] < 1 || ds.hneg[d] < 0 || ds.hpos[d] < 0 || ds.hneg[d] > kMaxHalo || ds.hpos[d] > kMaxHalo)
            return fail(c, TC_ERR_ARG, "tc_decl_dat: size must be >= 1 and halos 0..%d", kMaxHalo);
        ds.wlo[d] = 0;
        ds.whi[d] = 0;
    }
    ds.xorg = round_up(ds.hneg[0], kXAlign);
    ds.pitch = round_up(ds.xorg + ds.size[0] + ds.hpos[0], kXAlign);
    ds.ny_alloc = (int64_t)ds.size[1] + ds.hneg[1] + ds.hpos[1];
    ds.nz_alloc = (int64_t)ds.size[2] + ds.hneg[2] + ds.hpos[2];
    ds.bytes = ds.pitch * ds.ny_alloc * ds.nz_alloc * (int64_t)ds.esize();
    ds.stagger = c.stagger_unit * (int64_t)(c.dats.size() % 16);
    if (!c.host_only) {
        ds.raw[0] = dev_alloc(c, (size_t)(ds.bytes + ds.stagger));
        if (!ds.raw[0]) return fail(c, TC_ERR_NOMEM, "tc_decl_dat: cannot allocate %lld bytes", (long long)ds.bytes);
        ds.buf[0] = (char *)ds.raw[0] + ds.stagger;
        hipError_t e = hipMemsetAsync(ds.buf[0], 0, (size_t)ds.bytes, c.stream);
        if (e != hipSuccess) {
            dev_free(c, ds.raw[0]);
            return fail(c, TC_ERR_DEVICE, "hipMemsetAsync failed: %s", hipGetErrorString(e));
        }
    }
    c.dats.push_back(ds);
    *out = (tc_dat)c.dats.size() - 1;
    if (host_init && !c.host_only) {
        tc_status st = copy_host(c, c.dats.back(), nullptr, host_init, 0, true);
        if (st != TC_OK) return st;
    } else if (!c.host_only) {
        HIPCHK(c, hipStreamSynchronize(c.stream));
    }
    return TC_OK;
}

static tc_status impl_tc_decl_stencil(tc_ctx *ctx, int ndim, int npoints, const int32_t *offsets, const char *name,
                          tc_stencil *out) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (ndim < 1 || ndim > 3 || npoints < 1 || npoints > kMaxPts || !offsets || !out)
        return fail(c, TC_ERR_ARG, "tc_decl_stencil: ndim 1..3, 1..%d points", kMaxPts);
    Stencil s;
    s.ndim = ndim;
    s.name = name ? name : "";
    s.pts.assign(3 * npoints, 0);
    for (int d = 0; d < 3; ++d) {
        s.lo[d] = 0;
        s.hi[d] = 0;
    }
    for (int p = 0; p < npoints; ++p)
        for (int d = 0; d < ndim; ++d) {
            int v = offsets[p * ndim + d];
            if (v < -kMaxHalo || v > kMaxHalo) return fail(c, TC_ERR_ARG, "stencil offset out of range");
            s.pts[3 * p + d] = v;
        }
    for (int d = 0; d < 3; ++d) {
        s.lo[d] = s.hi[d] = s.pts[d];
        for (int p = 1; p < npoints; ++p) {
            s.lo[d] = std::min(s.lo[d], s.pts[3 * p + d]);
            s.hi[d] = std::max(s.hi[d], s.pts[3 * p + d]);
        }
    }
    c.stencils.push_back(s);
    *out = (tc_stencil)c.stencils.size() - 1;
    return TC_OK;
}

static tc_status impl_tc_decl_reduction(tc_ctx *ctx, tc_redop op, const char *name, tc_red *out) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if ((op != TC_RED_SUM && op != TC_RED_MIN && op != TC_RED_MAX) || !out)
        return fail(c, TC_ERR_ARG, "tc_decl_reduction: bad op");
    Reduction r;
    r.op = op;
    r.name = name ? name : "";
    if (op == TC_RED_MIN) r.hi = INFINITY;
    if (op == TC_RED_MAX) r.hi = -INFINITY;
    c.reds.push_back(r);
    *out = (tc_red)c.reds.size() - 1;
    return TC_OK;
}

static tc_status impl_tc_par_loop(tc_ctx *ctx, const char *name, tc_op op, tc_block blk, const int32_t *range, const tc_arg *args,
                      int nargs, const double *params, int nparams) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (blk < 0 || blk >= (int)c.blocks.size() || !range || (nargs > 0 && !args) || nargs < 0 ||
        nargs > kMaxArgs || nparams < 0 || nparams > kMaxParams || (nparams > 0 && !params))
        return fail(c, TC_ERR_ARG, "tc_par_loop: bad block, range, argument or parameter list");
    const int ndim = c.blocks[blk].ndim;
    Sig sig;
    if (!op_sig(op, ndim, sig)) return fail(c, TC_ERR_ARG, "tc_par_loop: unknown op %d", (int)op);
    LoopRec lp;
    lp.op = op;
    lp.block = blk;
    lp.ndim = ndim;
    lp.name = name ? name : "";
    lp.args.reserve((size_t)nargs);
    for (int d = 0; d < 3; ++d) {
        lp.lo[d] = d < ndim ? range[2 * d] : 0;
        lp.hi[d] = d < ndim ? range[2 * d + 1] : 1;
        if (lp.hi[d] < lp.lo[d]) return fail(c, TC_ERR_ARG, "tc_par_loop %s: range end below start", lp.name.c_str());
    }
    int ndat = 0, nred = 0, npts = 0;
    int dtype0 = -1;
    for (int i = 0; i < nargs; ++i) {
        ArgRec a{args[i].kind, args[i].handle, args[i].stencil, args[i].access};
        if (a.kind == TC_ARG_RED) {
            if (a.handle < 0 || a.handle >= (int)c.reds.size())
                return fail(c, TC_ERR_ARG, "tc_par_loop %s: bad reduction handle", lp.name.c_str());
            if (sig.red_op >= 0 && c.reds[a.handle].op != sig.red_op)
                return fail(c, TC_ERR_ARG, "tc_par_loop %s: reduction op does not match", lp.name.c_str());
            ++nred;
            lp.args.push_back(a);
            continue;
        }
        if (a.kind != TC_ARG_DAT) return fail(c, TC_ERR_ARG, "tc_par_loop: bad argument kind");
        if (a.handle < 0 || a.handle >= (int)c.dats.size() || a.stencil < 0 || a.stencil >= (int)c.stencils.size())
            return fail(c, TC_ERR_ARG, "tc_par_loop %s: bad dataset or stencil handle", lp.name.c_str());
        const Dataset &ds = c.dats[a.handle];
        const Stencil &st = c.stencils[a.stencil];
        if (ds.block != blk || st.ndim != ndim)
            return fail(c, TC_ERR_ARG, "tc_par_loop %s: dataset/stencil not on this block", lp.name.c_str());
        const int want = op_access(op, ndim, ndat);
        if (!access_ok(want, a.access))
            return fail(c, TC_ERR_ARG, "tc_par_loop %s: argument %d has the wrong access mode", lp.name.c_str(), i);
        {
            int flo[3], fhi[3];
            if (op_footprint(op, ndim, ndat, flo, fhi))
                for (int d = 0; d < 3; ++d)
                    if (flo[d] < st.lo[d] || fhi[d] > st.hi[d])
                        return fail(c, TC_ERR_ARG, "tc_par_loop %s: stencil of argument %d does not cover the op's reads",
                                    lp.name.c_str(), i);
        }
        if (a.writes() && !st.centre_only() && op != TC_OP_HALO_REFLECT)
            return fail(c, TC_ERR_ARG, "tc_par_loop %s: a write must use the centre stencil", lp.name.c_str());
        if (op != TC_OP_COPY) {
            if (dtype0 < 0) dtype0 = ds.dtype;
            if (ds.dtype != dtype0)
                return fail(c, TC_ERR_ARG, "tc_par_loop %s: mixed dataset types", lp.name.c_str());
        }
        if (lp.points() > 0)
            for (int d = 0; d < ndim; ++d)
                if (lp.lo[d] + st.lo[d] < -ds.hneg[d] || lp.hi[d] - 1 + st.hi[d] >= ds.size[d] + ds.hpos[d])
                    return fail(c, TC_ERR_RANGE, "tc_par_loop %s: range plus stencil leaves dataset %s's halo",
                                lp.name.c_str(), ds.name.c_str());
        npts += st.npoints();
        ++ndat;
        lp.args.push_back(a);
    }
    if (ndat < sig.ndat_min || ndat > sig.ndat_max || nred != sig.nred)
        return fail(c, TC_ERR_ARG, "tc_par_loop %s: wrong number of arguments for op %d", lp.name.c_str(), (int)op);
    if (npts > kMaxPts) return fail(c, TC_ERR_ARG, "tc_par_loop %s: more than %d stencil points", lp.name.c_str(), kMaxPts);
    // one dataset may not be written twice, or written and read at an offset
    for (size_t i = 0; i < lp.args.size(); ++i) {
        const ArgRec &a = lp.args[i];
        if (!a.writes()) continue;
        for (size_t j = 0; j < lp.args.size(); ++j) {
            if (i == j || lp.args[j].kind != TC_ARG_DAT || lp.args[j].handle != a.handle) continue;
            if (lp.args[j].writes() || !c.stencils[lp.args[j].stencil].centre_only())
                return fail(c, TC_ERR_ARG, "tc_par_loop %s: dataset written and accessed again in one loop",
                            lp.name.c_str());
        }
    }
    int want_params = sig.nparams;
    if (op == TC_OP_WSUM) {
        want_params = npts - c.stencils[lp.args[0].stencil].npoints();
    }
    if (nparams != want_params)
        return fail(c, TC_ERR_ARG, "tc_par_loop %s: expected %d parameters, got %d", lp.name.c_str(), want_params,
                    nparams);
    if (op == TC_OP_HALO_REFLECT) {
        const int axis = (int)params[0], side = (int)params[1], n = (int)params[2];
        if (axis < 0 || axis >= ndim || (side != 0 && side != 1) || n < 1)
            return fail(c, TC_ERR_ARG, "tc_par_loop %s: bad reflect parameters", lp.name.c_str());
        if (lp.points() > 0) {
            const Stencil &st = c.stencils[lp.args[0].stencil];
            for (int ci : {lp.lo[axis], lp.hi[axis] - 1}) {
                if (ci >= 0 && ci < n)
                    return fail(c, TC_ERR_ARG, "tc_par_loop %s: reflect range must be ghost points", lp.name.c_str());
                int off = (side == 0 ? -1 - ci : 2 * n - 1 - ci) - ci;
                if (off < st.lo[axis] || off > st.hi[axis])
                    return fail(c, TC_ERR_ARG, "tc_par_loop %s: reflect source outside the stencil", lp.name.c_str());
            }
            for (int d = 0; d < ndim; ++d)
                if (d != axis && (st.lo[d] != 0 || st.hi[d] != 0))
                    return fail(c, TC_ERR_ARG, "tc_par_loop %s: reflect stencil must lie on the axis", lp.name.c_str());
        }
    }
    lp.params.assign(params, params + nparams);
    if (c.chain.capacity() == c.chain.size()) c.chain.reserve(std::max<size_t>(128, 2 * c.chain.size()));
    c.chain.push_back(std::move(lp));
    c.stats.loops_recorded++;
    return TC_OK;
}

static tc_status impl_tc_par_loops(tc_ctx *ctx, int32_t n, const tc_loop *loops, const tc_arg *args,
                                   const double *params, int32_t *recorded) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (recorded) *recorded = 0;
    if (n < 0 || (n > 0 && !loops)) return fail(c, TC_ERR_ARG, "tc_par_loops: bad loop list");
    for (int32_t i = 0; i < n; ++i) {
        const tc_loop &L = loops[i];
        if (L.nargs < 0 || L.nparams < 0 || L.first_arg < 0 || L.first_param < 0 || (L.nargs > 0 && !args) ||
            (L.nparams > 0 && !params))
            return fail(c, TC_ERR_ARG, "tc_par_loops: loop %d has a bad argument or parameter slice", (int)i);
        const tc_status st = impl_tc_par_loop(ctx, "", (tc_op)L.op, L.block, L.range, args + L.first_arg, L.nargs,
                                              params + L.first_param, L.nparams);
        if (st != TC_OK) return st;
        if (recorded) *recorded = i + 1;
    }
    return TC_OK;
}

static tc_status impl_tc_flush(tc_ctx *ctx) {
    CHECK_CTX(ctx);
    return flush(ctx->c);
}

static tc_status impl_tc_reduction_result(tc_ctx *ctx, tc_red red, double *out) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (red < 0 || red >= (int)c.reds.size() || !out) return fail(c, TC_ERR_ARG, "bad reduction handle");
    tc_status st = flush(c);
    if (st != TC_OK) return st;
    Reduction &r = c.reds[red];
    *out = r.op == TC_RED_SUM ? r.hi + r.lo : r.hi;
    r.hi = r.op == TC_RED_SUM ? 0.0 : (r.op == TC_RED_MIN ? INFINITY : -INFINITY);
    r.lo = 0.0;
    r.touched = false;
    return TC_OK;
}

// tc_reduction_result without any device allocation: the context's
// partials, outputs, graph use and profiling are swapped out for the call.
static tc_status impl_tc_reduction_result_static(tc_ctx *ctx, tc_red red, double *out) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (red < 0 || red >= (int)c.reds.size() || !out) return fail(c, TC_ERR_ARG, "bad reduction handle");
    if (c.host_only) return fail(c, TC_ERR_STATE, "host-only context cannot execute loops");
    if (!c.scratch) return fail(c, TC_ERR_STATE, "no static scratch on this context's device");
    struct Saved {
        Ctx &c;
        double *partials, *red_out;
        int64_t partials_cap, red_out_cap;
        bool graphs, profiling;
        explicit Saved(Ctx &cc)
            : c(cc), partials(cc.partials), red_out(cc.red_out), partials_cap(cc.partials_cap),
              red_out_cap(cc.red_out_cap), graphs(cc.use_graphs), profiling(cc.profiling) {
            c.noalloc = true;
            c.use_graphs = false;
            c.profiling = false;
            c.partials = c.red_out = nullptr;  // laid out in the scratch by the flush
            c.partials_cap = c.red_out_cap = 0;
        }
        ~Saved() {
            c.partials = partials;
            c.red_out = red_out;
            c.partials_cap = partials_cap;
            c.red_out_cap = red_out_cap;
            c.use_graphs = graphs;
            c.profiling = profiling;
            c.noalloc = false;
        }
    } saved(c);
    tc_status st = flush(c);
    if (st != TC_OK) return st;
    Reduction &r = c.reds[red];
    *out = r.op == TC_RED_SUM ? r.hi + r.lo : r.hi;
    r.hi = r.op == TC_RED_SUM ? 0.0 : (r.op == TC_RED_MIN ? INFINITY : -INFINITY);
    r.lo = 0.0;
    r.touched = false;
    return TC_OK;
}

static tc_status impl_tc_dat_read(tc_ctx *ctx, tc_dat dat, void *host) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (dat < 0 || dat >= (int)c.dats.size() || !host) return fail(c, TC_ERR_ARG, "bad dataset handle");
    if (c.host_only) return fail(c, TC_ERR_STATE, "host-only context has no data");
    tc_status st = flush(c);
    if (st != TC_OK) return st;
    Dataset &ds = c.dats[dat];
    return copy_host(c, ds, host, nullptr, ds.cur, false);
}

static tc_status impl_tc_dat_write(tc_ctx *ctx, tc_dat dat, const void *host) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (dat < 0 || dat >= (int)c.dats.size() || !host) return fail(c, TC_ERR_ARG, "bad dataset handle");
    if (c.host_only) return fail(c, TC_ERR_STATE, "host-only context has no data");
    tc_status st = flush(c);
    if (st != TC_OK) return st;
    Dataset &ds = c.dats[dat];
    ds.twin_synced = false;
    return copy_host(c, ds, nullptr, host, ds.cur, true);
}

static tc_status impl_tc_dat_device_view(tc_ctx *ctx, tc_dat dat, void **origin, int64_t strides[3]) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (dat < 0 || dat >= (int)c.dats.size() || !origin || !strides) return fail(c, TC_ERR_ARG, "bad argument");
    if (c.host_only) return fail(c, TC_ERR_STATE, "host-only context has no data");
    tc_status st = flush(c);
    if (st != TC_OK) return st;
    Dataset &ds = c.dats[dat];
    *origin = ds.origin(ds.cur);
    strides[0] = 1;
    strides[1] = ds.sy();
    strides[2] = ds.sz();
    ds.twin_synced = false;  // the caller may write through the view
    return TC_OK;
}

static tc_status impl_tc_set_tiling(tc_ctx *ctx, tc_tiling mode, const int32_t *tile) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (mode < TC_TILING_NONE || mode > TC_TILING_AUTO) return fail(c, TC_ERR_ARG, "bad tiling mode");
    tc_status st = flush(c);  // the new mode applies to loops recorded from now on
    if (st != TC_OK) return st;
    c.mode = mode;
    for (int d = 0; d < 3; ++d) c.tile[d] = tile ? tile[d] : 0;
    return TC_OK;
}

static tc_status impl_tc_set_profiling(tc_ctx *ctx, int on) {
    CHECK_CTX(ctx);
    if (ctx->c.host_only && on) return fail(ctx->c, TC_ERR_STATE, "host-only context cannot time kernels");
    ctx->c.profiling = on != 0;
    return TC_OK;
}

static tc_status impl_tc_get_stats(tc_ctx *ctx, tc_stats *out) {
    CHECK_CTX(ctx);
    if (!out) return TC_ERR_ARG;
    *out = ctx->c.stats;
    out->jit_compile_seconds = ctx->c.jit_compile_seconds;
    return TC_OK;
}

static tc_status impl_tc_chain_plan(tc_ctx *ctx, tc_tiling mode, const int32_t *tile, int32_t *num_tiles, int32_t *ranges,
                        int64_t cap) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if ((mode != TC_TILING_SKEWED && mode != TC_TILING_FUSED) || !num_tiles)
        return fail(c, TC_ERR_UNSUPPORTED, "tc_chain_plan: skewed or fused mode only");
    int t3[3] = {tile ? tile[0] : 0, tile ? tile[1] : 0, tile ? tile[2] : 0};
    if (mode == TC_TILING_FUSED) {
        auto groups = fused_split(c, c.chain, t3, c.jit_cpl);
        const int L = (int)c.chain.size();
        num_tiles[0] = (int32_t)groups.size();
        num_tiles[1] = L;
        num_tiles[2] = 0;
        const int64_t need = 2 * (int64_t)groups.size() + 7 * (int64_t)L;
        if (!ranges || cap < need) return fail(c, TC_ERR_ARG, "tc_chain_plan: need %lld slots", (long long)need);
        for (size_t g = 0; g < groups.size(); ++g) {
            ranges[2 * g] = groups[g]->g0;
            ranges[2 * g + 1] = groups[g]->g1;
        }
        int32_t *per = ranges + 2 * groups.size();
        for (int l = 0; l < L; ++l) {
            per[7 * l] = -1;
            for (int k = 1; k < 7; ++k) per[7 * l + k] = 0;
        }
        for (const auto &g : groups) {
            if (g->estage || g->cheb) {
                for (int l = g->g0; l < g->g1; ++l) per[7 * l] = g->estage ? 3 : 4;
                continue;
            }
            if (g->staged) {
                const StagedGroup &S = *g->staged;
                for (int l = S.g0; l < S.g1; ++l) {
                    int32_t *e = per + 7 * l;
                    const auto &x = S.ext[l - S.g0];
                    e[0] = S.computed[l - S.g0] ? 2 : 0;
                    if (x[0] < 0) continue;
                    for (int k = 0; k < 6; ++k) e[1 + k] = x[k];
                }
                continue;
            }
            for (const auto &J : g->loops) {
                int32_t *e = per + 7 * J.loop;
                e[0] = J.needed ? 1 : 0;
                if (!J.needed) continue;
                e[1] = J.extL;
                e[2] = J.extR;
                e[3] = J.extB;
                e[4] = J.extT;
            }
        }
        return fused_compile(c, c.chain, groups);
    }
    SkewedPlan P = build_skewed_plan(c, c.chain, t3);
    int maxT = 1;
    for (int d = 0; d < 3; ++d) {
        num_tiles[d] = d < P.ndim ? P.num_tiles[d] : 1;
        maxT = std::max(maxT, num_tiles[d]);
    }
    const int L = P.nloops;
    const int64_t need = (int64_t)P.ndim * maxT * L * 2;
    if (!ranges || cap < need) return fail(c, TC_ERR_ARG, "tc_chain_plan: need %lld slots", (long long)need);
    for (int d = 0; d < P.ndim; ++d)
        for (int t = 0; t < P.num_tiles[d]; ++t)
            for (int l = 0; l < L; ++l) {
                ranges[((int64_t)(d * maxT + t) * L + l) * 2] = P.s(d, t, l);
                ranges[((int64_t)(d * maxT + t) * L + l) * 2 + 1] = P.e(d, t, l);
            }
    return TC_OK;
}

static tc_status impl_tc_staged_tiles(tc_ctx *ctx, const int32_t *tile, int32_t group, int32_t *info, int32_t *boxes,
                                      int64_t cap) {
    CHECK_CTX(ctx);
    Ctx &c = ctx->c;
    if (!info) return fail(c, TC_ERR_ARG, "tc_staged_tiles: info is NULL");
    int t3[3] = {tile ? tile[0] : 0, tile ? tile[1] : 0, tile ? tile[2] : 0};
    auto groups = fused_split(c, c.chain, t3, c.jit_cpl);
    if (group < 0 || group >= (int)groups.size()) return fail(c, TC_ERR_ARG, "tc_staged_tiles: no group %d", group);
    const FusedGroup &g = *groups[group];
    info[0] = g.g0;
    info[1] = g.g1;
    if (!g.staged) {
        info[2] = 0;
        return TC_OK;
    }
    const StagedGroup &S = *g.staged;
    info[2] = S.ntot;
    for (int d = 0; d < 3; ++d) info[3 + d] = S.tile[d];
    const int L = S.g1 - S.g0, ns = (int)S.slots.size();
    const int64_t per = 6 + 6 * (int64_t)L, need = per * S.ntot;
    if (!boxes) return TC_OK;
    if (cap < need) return fail(c, TC_ERR_ARG, "tc_staged_tiles: need %lld slots", (long long)need);
    for (int t = 0; t < S.ntot; ++t) {
        const int *r = &S.table[(size_t)t * S.rec];
        int32_t *o = boxes + per * t;
        for (int k = 0; k < 6; ++k) o[k] = r[k];
        for (int l = 0; l < L; ++l)
            for (int k = 0; k < 6; ++k) o[6 + 6 * l + k] = r[6 + 9 * ns + 6 * l + k];
    }
    return TC_OK;
}

static tc_status impl_tc_pending(tc_ctx *ctx, int32_t *nloops) {
    CHECK_CTX(ctx);
    if (!nloops) return TC_ERR_ARG;
    *nloops = (int32_t)ctx->c.chain.size();
    return TC_OK;
}

extern "C" {

tc_status tc_init(const tc_init_opts *opts, tc_ctx **out) {
    return tc::guard_abi(nullptr, [&] { return impl_tc_init(opts, out); });
}

tc_status tc_finalize(tc_ctx *ctx) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_finalize(ctx); });
}

tc_status tc_decl_block(tc_ctx *ctx, int ndim, const char *name, tc_block *out) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_decl_block(ctx, ndim, name, out); });
}

tc_status tc_decl_dat(tc_ctx *ctx, tc_block blk, tc_dtype dtype, const int32_t *size, const int32_t *halo_neg,
                      const int32_t *halo_pos, const void *host_init, const char *name, tc_dat *out) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] {
        return impl_tc_decl_dat(ctx, blk, dtype, size, halo_neg, halo_pos, host_init, name, out);
    });
}

tc_status tc_decl_stencil(tc_ctx *ctx, int ndim, int npoints, const int32_t *offsets, const char *name,
                          tc_stencil *out) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] {
        return impl_tc_decl_stencil(ctx, ndim, npoints, offsets, name, out);
    });
}

tc_status tc_decl_reduction(tc_ctx *ctx, tc_redop op, const char *name, tc_red *out) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_decl_reduction(ctx, op, name, out); });
}

tc_status tc_par_loop(tc_ctx *ctx, const char *name, tc_op op, tc_block blk, const int32_t *range, const tc_arg *args,
                      int nargs, const double *params, int nparams) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] {
        return impl_tc_par_loop(ctx, name, op, blk, range, args, nargs, params, nparams);
    });
}

tc_status tc_par_loops(tc_ctx *ctx, int32_t n, const tc_loop *loops, const tc_arg *args, const double *params,
                       int32_t *recorded) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_par_loops(ctx, n, loops, args, params, recorded); });
}

tc_status tc_flush(tc_ctx *ctx) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_flush(ctx); });
}

tc_status tc_reduction_result(tc_ctx *ctx, tc_red red, double *out) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_reduction_result(ctx, red, out); });
}

tc_status tc_reduction_result_static(tc_ctx *ctx, tc_red red, double *out) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_reduction_result_static(ctx, red, out); });
}

tc_status tc_dat_read(tc_ctx *ctx, tc_dat dat, void *host) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_dat_read(ctx, dat, host); });
}

tc_status tc_dat_write(tc_ctx *ctx, tc_dat dat, const void *host) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_dat_write(ctx, dat, host); });
}

tc_status tc_dat_device_view(tc_ctx *ctx, tc_dat dat, void **origin, int64_t strides[3]) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_dat_device_view(ctx, dat, origin, strides); });
}

tc_status tc_set_tiling(tc_ctx *ctx, tc_tiling mode, const int32_t *tile) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_set_tiling(ctx, mode, tile); });
}

tc_status tc_set_profiling(tc_ctx *ctx, int on) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_set_profiling(ctx, on); });
}

tc_status tc_get_stats(tc_ctx *ctx, tc_stats *out) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_get_stats(ctx, out); });
}

tc_status tc_chain_plan(tc_ctx *ctx, tc_tiling mode, const int32_t *tile, int32_t *num_tiles, int32_t *ranges,
                        int64_t cap) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] {
        return impl_tc_chain_plan(ctx, mode, tile, num_tiles, ranges, cap);
    });
}

tc_status tc_staged_tiles(tc_ctx *ctx, const int32_t *tile, int32_t group, int32_t *info, int32_t *boxes, int64_t cap) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_staged_tiles(ctx, tile, group, info, boxes, cap); });
}

tc_status tc_pending(tc_ctx *ctx, int32_t *nloops) {
    return tc::guard_abi(ctx ? &ctx->c : nullptr, [&] { return impl_tc_pending(ctx, nloops); });
}

const char *tc_status_string(tc_status s) {
    switch (s) {
    case TC_OK: return "ok";
    case TC_ERR_ARG: return "invalid argument";
    case TC_ERR_STATE: return "invalid state";
    case TC_ERR_DEVICE: return "device error";
    case TC_ERR_NOMEM: return "out of memory";
    case TC_ERR_UNSUPPORTED: return "unsupported";
    case TC_ERR_RANGE: return "range outside halo";
    default: return "unknown status";
    }
}

const char *tc_last_error(tc_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->c.last_error.c_str();
}

}  // extern "C"
