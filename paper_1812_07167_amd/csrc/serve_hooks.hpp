// Library-internal entry points shared by the C ABI and the request loop: the solve of
// one factor on an explicit stream, the size of its workspace, and the workspace pool.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "../../include/hps.h"

namespace hps {

// Device bytes one solve call of f with nrhs right-hand sides allocates for its
// workspace (with or without a body load s); host arithmetic only.
size_t solve_workspace_bytes(hps_factor* f, int nrhs, bool with_s);

// hps_solve on stream st; the residual-correction record goes to *info.  Throws
// hps::Error on failure.
void solve_on(hps_factor* f, int nrhs, const double* s, const double* t, double* u,
              hipStream_t st, hps_solve_info* info);

// Device memory for one call's workspace or staging, from the library's cache of
// buffers on the current device: ws_alloc orders stream st after the buffer's previous
// use, ws_free marks the buffer idle once st's queued work reaches that point, ws_trim
// frees the idle buffers of the current device.  ws_alloc throws hps::Error.
void* ws_alloc(size_t bytes, hipStream_t st);
void ws_free(void* p, hipStream_t st);
void ws_trim();
// The same cache for long-lived buffers that several streams may use: ws_free_idle
// synchronizes the device before the buffer becomes reusable, so reuse needs no event.
void* ws_alloc_idle(size_t bytes);
void ws_free_idle(void* p);

// Message hps_last_error() returns on the calling thread.
void set_last_error(const std::string& msg);

}  // namespace hps
