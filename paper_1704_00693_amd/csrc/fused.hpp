// Fused (overlapped, LDS-streamed) execution of a loop chain and the
// autotuner's choice between execution modes.
#pragma once

#include "tc_internal.hpp"

namespace tc {

// Execute `chain` in fused mode.  Fills the reductions it used (slot order),
// their partial ranges, and launch / tile / group counts for the statistics.
tc_status fused_flush(Ctx &c, const std::vector<LoopRec> &chain, const int tile[3], std::vector<int> &red_handles,
                      std::vector<int64_t> &red_base, std::vector<int64_t> &red_count, int &launches, int &tiles,
                      int &groups);

// Release device memory held for fused execution.
void fused_release(Ctx &c);

// AUTO mode: the execution mode (and tile, written back) to use for this chain.
tc_tiling autotune_choose(Ctx &c, const std::vector<LoopRec> &chain, int tile[3]);

}  // namespace tc
