// AUTO mode: per chain structure, time each candidate schedule and keep the
// fastest.
#include "fused.hpp"

namespace tc {

// AUTO mode (Section 4.3 chooses a tile size from the cache size; here the
// cache-based choice is one candidate and every candidate is measured): the
// first flushes of a chain structure run the candidate schedules in turn,
// three flushes each; the first two build the plan (and compile fused
// kernels, capture the launch graph, allocate second buffers) and are not
// timed, the device time of the third is recorded.  Afterwards the fastest
// is used.  Every candidate computes bit-identical results, so tuning never
// changes answers.
namespace {
constexpr int kTuneWarm = 2;  // untimed flushes of a candidate before the timed one
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
        v.push_back({TC_TILING_FUSED, {0, 0, 0}});
        v.push_back({TC_TILING_FUSED, {0, 96, 0}});
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
        c.tune_key = key;
        if (T.warm < kTuneWarm) {
            ++T.warm;
            c.tune_cand = -1;  // warming up: not timed
        } else {
            c.tune_cand = pick;
        }
    }
    for (int d = 0; d < 3; ++d) tile[d] = cands[pick].tile[d];
    return cands[pick].mode;
}

void autotune_record(Ctx &c, double seconds) {
    if (c.tune_cand < 0) return;
    Ctx::Tune &T = c.tuned[c.tune_key];
    T.seconds.push_back(seconds);
    T.next = c.tune_cand + 1;
    T.warm = 0;
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
