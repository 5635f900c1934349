// Launcher of the rANS decoder (tpc_rans.hip).
#pragma once

#include "tpc_internal.hpp"

size_t rans_decode_ws_bytes();
hipError_t launch_rans_decode(const void *in, uint64_t size, int32_t *out, int64_t cap, int64_t *n_out,
                              int32_t *dev_status, void *ws, hipStream_t st);
