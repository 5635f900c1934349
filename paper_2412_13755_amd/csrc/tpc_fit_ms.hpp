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

// The fit over rows, then the smoother: the state at every seed hit's plane
// (hit_par [cap_hits][5], hit_cov [cap_hits][15]); rejected is required.
// Workspace: smooth_ws_layout bytes (the fit's, then per-seed final states,
// per-hit filtered deviations and rows).
struct SmWs {
    double *pfin;      // [cap_seeds][5] final states of the fit
    double *wd;        // [cap_hits][38] filtered deviation, covariance, reference, arriving step
    int16_t *wrow;     // [cap_hits] pad row of each hit
};
size_t smooth_ws_layout(void *ws, int64_t cap_seeds, int64_t cap_hits, SmWs *out);
hipError_t launch_smooth(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd, const float *err,
                         const tpc_material *mat, const tpc_tracks *tr, uint8_t *rejected, float *hit_par,
                         float *hit_cov, void *ws, hipStream_t st);
