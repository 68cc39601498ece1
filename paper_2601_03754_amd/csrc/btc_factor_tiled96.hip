// Tile-parallel factorization level step, padded block size 96.
#include "btc_tiled.h"

namespace btc {

hipError_t launch_factor_tiled96(const Launch<FactorDesc>& p, int mode, int part, int level_hint, int64_t items,
                                  hipStream_t st) {
    if (mode == 2) return launch_tiled_np<96, true, true>(p, part, level_hint, items, st);
    if (mode == 1) return launch_tiled_np<96, true, false>(p, part, level_hint, items, st);
    return launch_tiled_np<96, false, false>(p, part, level_hint, items, st);
}

}  // namespace btc
