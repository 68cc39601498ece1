// Tile-parallel factorization level step at padded block size 32 (a variant
// the autotuner may choose over the one-workgroup-per-node kernels: its
// pivot kernel needs a fraction of their LDS, so many more nodes share a
// compute unit).
#include "btc_tiled.h"

namespace btc {

hipError_t launch_factor_tiled32(const Launch<FactorDesc>& p, int mode, int part, bool deferred, int64_t items,
                                 hipStream_t st) {
    if (mode == 2) return launch_tiled_np<32, true, true>(p, part, deferred, items, st);
    if (mode == 1) return launch_tiled_np<32, true, false>(p, part, deferred, items, st);
    return launch_tiled_np<32, false, false>(p, part, deferred, items, st);
}

}  // namespace btc
