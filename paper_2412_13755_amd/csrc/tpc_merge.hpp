#pragma once
#include "tpc_internal.hpp"

// Mutual-best links between fitted segments of neighbouring sectors.
hipError_t launch_merge(const tpc_context *ctx, const tpc_seeds *sd, const tpc_tracks *tr, double cut,
                        int32_t *next, int32_t *prev, float *chi2, float *mpar, float *mcov, int32_t *leg,
                        float *leg_chi2, hipStream_t st);
