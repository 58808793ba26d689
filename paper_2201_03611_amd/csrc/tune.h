// Tune cache lookups (tune.hip): the tile / schedule recorded by the autotuner
// for these sizes on the current device's architecture, if any.
#pragma once

#include "common.h"

namespace rise {
bool tune_lookup_gemm(int64_t M, int64_t N, int64_t K, int mode, rise_tile* out);
bool tune_lookup_stencil(int64_t H, int64_t W, int k, rise_stencil_schedule* out);
}  // namespace rise
