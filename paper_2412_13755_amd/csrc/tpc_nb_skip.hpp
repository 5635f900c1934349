#pragma once
#include "tpc_internal.hpp"

// Adjacent-row neighbours, then partners across one missing row for the
// clusters left unlinked (same workspace as the adjacent-row search).
hipError_t launch_neighbours_skip(const tpc_context *ctx, const tpc_frames *fr, int32_t *up, int32_t *dn,
                                  const NbWs &ws, hipStream_t st);
