// Launchers of the fit with material and of the fit over any rows (tpc_fit_ms.hip).
#pragma once

#include "tpc_internal.hpp"

hipError_t launch_fit_material(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                               const tpc_material *mat, const tpc_tracks *tr, uint8_t *rejected,
                               void *ws, hipStream_t st);

// Seeds whose hits may skip pad rows (rows looked up in the cluster layout),
// per-cluster errors err[N][2] (sigma_y, sigma_z) or null, material or null.
hipError_t launch_fit_rows(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd, const float *err,
                           const tpc_material *mat, const tpc_tracks *tr, uint8_t *rejected, void *ws,
                           hipStream_t st);
