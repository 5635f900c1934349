#pragma once
#include "tpc_internal.hpp"

// Track ids, chain refits and joint looper circles from the merging links.
hipError_t launch_refit(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd, const tpc_tracks *seg,
                        const int32_t *next, const int32_t *prev, const int32_t *leg, const float *map,
                        int32_t *track_id, const tpc_tracks *out, float *loop_par, float *loop_cov,
                        float *loop_chi2, hipStream_t st);
