// Tile-parallel factorization level step, padded block size 128, and the
// dispatcher over the padded sizes.
#include "btc_tiled.h"

namespace btc {

hipError_t launch_factor_tiled128(const Launch<FactorDesc>& p, int mode, int part, bool deferred, int64_t items,
                                  hipStream_t st) {
    if (mode == 2) return launch_tiled_np<128, true, true>(p, part, deferred, items, st);
    if (mode == 1) return launch_tiled_np<128, true, false>(p, part, deferred, items, st);
    return launch_tiled_np<128, false, false>(p, part, deferred, items, st);
}

hipError_t launch_factor_tiled(const Launch<FactorDesc>& p, int np, int mode, int part, bool deferred,
                               int64_t items, hipStream_t st) {
    switch (np) {
        case 32: return launch_factor_tiled32(p, mode, part, deferred, items, st);
        case 64: return launch_factor_tiled64(p, mode, part, deferred, items, st);
        case 96: return launch_factor_tiled96(p, mode, part, deferred, items, st);
        case 128: return launch_factor_tiled128(p, mode, part, deferred, items, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace btc
