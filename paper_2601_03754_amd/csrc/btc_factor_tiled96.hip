// Tile-parallel factorization level step, padded block size 96.
#include "btc_tiled.h"

namespace btc {

hipError_t launch_factor_tiled96(const Launch<FactorDesc>& p, bool mixed, int level_hint, int64_t items,
                                 hipStream_t st) {
    return mixed ? launch_tiled_np<96, true>(p, level_hint, items, st)
                 : launch_tiled_np<96, false>(p, level_hint, items, st);
}

}  // namespace btc
