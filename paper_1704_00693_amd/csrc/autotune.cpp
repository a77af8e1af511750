// AUTO mode: per chain structure, time each candidate schedule and keep the
// fastest.
#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "fused.hpp"

namespace tc {

// AUTO mode (Section 4.3 chooses a tile size from the cache size and reports
// that the automatic choice lands within a few percent of the best measured
// tile; here the cache-based choice is one candidate and every candidate is
// measured): the first flushes of a chain structure run the candidate
// schedules in turn.  Each candidate gets kTuneWarm untimed flushes (they
// build the plan, compile fused kernels, capture the launch graph and
// allocate second buffers) and then kTuneReps timed ones; its score is the
// median device time.  Afterwards the fastest is used.  Every candidate
// computes bit-identical results, so tuning never changes answers.
//
// Choices persist per chain key: in the context, and, when TC_TUNE_CACHE
// names a file, across processes (one line per chain key: key, mode, tile,
// columns per lane, median seconds).
namespace {
constexpr int kTuneWarm = 2;  // untimed flushes of a candidate before the timed ones
constexpr int kTuneReps = 3;  // timed flushes per candidate (the median is kept)

std::vector<TuneCand> candidates(const std::vector<LoopRec> &chain) {
    std::vector<TuneCand> v;
    v.push_back({TC_TILING_NONE, {0, 0, 0}, 1});
    v.push_back({TC_TILING_SKEWED, {0, 0, 0}, 1});
    const int nd = chain.empty() ? 2 : chain[0].ndim;
    if (nd >= 2) {
        int t[3] = {0, 0, 0};
        t[nd - 1] = 128;
        v.push_back({TC_TILING_SKEWED, {t[0], t[1], t[2]}, 1});
    }
    bool fusable = false;
    for (const auto &lp : chain) fusable = fusable || fused_op_supported(lp);
    if (!fusable && chain.size() >= 2) {
        // no weighted sums for register windows: the fused mode's staged
        // groups (any ops and ranges) are the one fused candidate
        v.push_back({TC_TILING_FUSED, {0, 0, 0}, 1});
    } else if (fusable) {
        // fused layouts: one or two columns per lane, and register budgets
        // that trade group depth (fewer, deeper groups) against the
        // recomputed overlap and occupancy
        v.push_back({TC_TILING_FUSED, {0, 0, 0}, 1});
        v.push_back({TC_TILING_FUSED, {0, 96, 0}, 1});
        v.push_back({TC_TILING_FUSED, {0, 0, 0}, 2});
        v.push_back({TC_TILING_FUSED, {0, 240, 0}, 2});
    }
    return v;
}

double median(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    return n % 2 ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

bool same(const TuneCand &a, const TuneCand &b) {
    return a.mode == b.mode && a.cpl == b.cpl && a.tile[0] == b.tile[0] && a.tile[1] == b.tile[1] &&
           a.tile[2] == b.tile[2];
}

void load_cache(Ctx &c) {
    if (c.tune_cache_loaded) return;
    c.tune_cache_loaded = true;
    const char *path = getenv("TC_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *fp = std::fopen(path, "r");
    if (!fp) return;
    unsigned long long key;
    TuneCand k;
    int mode;
    double sec;
    while (std::fscanf(fp, "%llx %d %d %d %d %d %lf", &key, &mode, &k.tile[0], &k.tile[1], &k.tile[2], &k.cpl,
                       &sec) == 7) {
        k.mode = (tc_tiling)mode;
        c.tune_saved[(uint64_t)key] = k;
    }
    std::fclose(fp);
}

void save_choice(Ctx &c, uint64_t key, const TuneCand &k, double sec) {
    c.tune_saved[key] = k;
    const char *path = getenv("TC_TUNE_CACHE");
    if (!path || !*path) return;
    if (FILE *fp = std::fopen(path, "a")) {
        std::fprintf(fp, "%016llx %d %d %d %d %d %.9g\n", (unsigned long long)key, (int)k.mode, k.tile[0], k.tile[1],
                     k.tile[2], k.cpl, sec);
        std::fclose(fp);
    }
}
}  // namespace

uint64_t autotune_key(const Ctx &c, const std::vector<LoopRec> &chain) {
    const int zero[3] = {0, 0, 0};
    return chain_key(c, chain, TC_TILING_AUTO, zero, 0);
}

TuneCand autotune_choose(Ctx &c, const std::vector<LoopRec> &chain) {
    const uint64_t key = autotune_key(c, chain);
    const auto cands = candidates(chain);
    load_cache(c);
    Ctx::Tune &T = c.tuned[key];
    c.tune_cand = -1;
    if (T.best < 0) {
        auto it = c.tune_saved.find(key);
        if (it != c.tune_saved.end())
            for (size_t i = 0; i < cands.size(); ++i)
                if (same(cands[i], it->second)) T.best = (int)i;
    }
    if (T.best >= 0) return cands[T.best];
    c.tune_key = key;
    if (T.warm < kTuneWarm)
        ++T.warm;  // warming up: not timed
    else
        c.tune_cand = T.next;
    return cands[T.next];
}

bool autotune_lookup(Ctx &c, const std::vector<LoopRec> &chain, TuneCand &out) {
    const uint64_t key = autotune_key(c, chain);
    const auto cands = candidates(chain);
    load_cache(c);
    auto t = c.tuned.find(key);
    if (t != c.tuned.end() && t->second.best >= 0) {
        out = cands[t->second.best];
        return true;
    }
    auto it = c.tune_saved.find(key);
    if (it == c.tune_saved.end()) return false;
    for (const auto &k : cands)
        if (same(k, it->second)) {
            out = k;
            return true;
        }
    return false;
}

void autotune_record(Ctx &c, double seconds) {
    if (c.tune_cand < 0) return;
    Ctx::Tune &T = c.tuned[c.tune_key];
    if (T.samples.size() <= (size_t)c.tune_cand) T.samples.resize(c.tune_cand + 1);
    T.samples[c.tune_cand].push_back(seconds);
    if ((int)T.samples[c.tune_cand].size() >= kTuneReps) {
        T.seconds.push_back(median(T.samples[c.tune_cand]));
        T.next = c.tune_cand + 1;
        T.warm = 0;
    }
    c.tune_cand = -1;
}

void autotune_finish(Ctx &c, const std::vector<LoopRec> &chain) {
    Ctx::Tune &T = c.tuned[c.tune_key];
    const auto cands = candidates(chain);
    if (T.best < 0 && T.seconds.size() >= cands.size()) {
        int b = 0;
        for (size_t i = 1; i < T.seconds.size(); ++i)
            if (T.seconds[i] < T.seconds[b]) b = (int)i;
        T.best = b;
        save_choice(c, c.tune_key, cands[b], T.seconds[b]);
        if (getenv("TC_TUNE_VERBOSE"))
            for (size_t i = 0; i < cands.size(); ++i)
                std::fprintf(stderr, "autotune %016llx: mode %d tile (%d,%d,%d) cpl %d: %.3f ms%s\n",
                             (unsigned long long)c.tune_key, (int)cands[i].mode, cands[i].tile[0], cands[i].tile[1],
                             cands[i].tile[2], cands[i].cpl, T.seconds[i] * 1e3, (int)i == b ? "  <- chosen" : "");
    }
}

}  // namespace tc
