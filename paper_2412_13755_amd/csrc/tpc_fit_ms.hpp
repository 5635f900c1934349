// Launcher of the fit with material (tpc_fit_ms.hip).
#pragma once

#include "tpc_internal.hpp"

hipError_t launch_fit_material(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                               const tpc_material *mat, const tpc_tracks *tr, uint8_t *rejected,
                               void *ws, hipStream_t st);
