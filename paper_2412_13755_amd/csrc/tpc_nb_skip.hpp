#pragma once
#include "tpc_internal.hpp"

// Workspace of the search across a missing row: the adjacent-row search's,
// then the list of queried clusters (id, segment) and its counter.
struct SkipWs {
    NbWs nb;
    int2 *list;         // [N]
    int32_t *count;     // device scalar
};
size_t skip_ws_layout(void *ws, int64_t N, int64_t NR, SkipWs *out);

// Adjacent-row neighbours, then partners across one missing row for the
// clusters left unlinked.
hipError_t launch_neighbours_skip(const tpc_context *ctx, const tpc_frames *fr, int32_t *up, int32_t *dn,
                                  const SkipWs &ws, hipStream_t st);
