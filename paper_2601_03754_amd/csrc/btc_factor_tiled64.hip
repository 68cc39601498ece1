// Tile-parallel factorization level step at padded block size 64 (a variant
// of the single-kernel path that the autotuner may choose: smaller LDS per
// workgroup, so several nodes share a compute unit).
#include "btc_tiled.h"

namespace btc {

hipError_t launch_factor_tiled64(const Launch<FactorDesc>& p, int mode, int part, bool deferred, int64_t items,
                                 hipStream_t st) {
    if (mode == 2) return launch_tiled_np<64, true, true>(p, part, deferred, items, st);
    if (mode == 1) return launch_tiled_np<64, true, false>(p, part, deferred, items, st);
    return launch_tiled_np<64, false, false>(p, part, deferred, items, st);
}

}  // namespace btc
