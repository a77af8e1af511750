// Placeholder implementations until the fused executor lands.
#include "fused.hpp"

namespace tc {

tc_status fused_flush(Ctx &c, const std::vector<LoopRec> &, const int *, std::vector<int> &, std::vector<int64_t> &,
                      std::vector<int64_t> &, int &, int &, int &) {
    c.last_error = "fused tiling is not available";
    return TC_ERR_UNSUPPORTED;
}

void fused_release(Ctx &) {}

tc_tiling autotune_choose(Ctx &, const std::vector<LoopRec> &, int *) { return TC_TILING_NONE; }

}  // namespace tc
