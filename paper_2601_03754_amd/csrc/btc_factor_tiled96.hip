// Tile-parallel factorization level step, padded block size 96.
#include "btc_tiled.h"

namespace btc {

hipError_t launch_factor_tiled96(const Launch<FactorDesc>& p, int mode, int part, bool deferred, int64_t items,
                                  hipStream_t st) {
    if (mode == 2) return launch_tiled_np<96, true, true>(p, part, deferred, items, st);
    if (mode == 1) return launch_tiled_np<96, true, false>(p, part, deferred, items, st);
    return launch_tiled_np<96, false, false>(p, part, deferred, items, st);
}

}  // namespace btc
