// Library-internal entry points the request loop uses beside the public C ABI: the
// solve of one factor on an explicit stream, and the size of its workspace.
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

// Message hps_last_error() returns on the calling thread.
void set_last_error(const std::string& msg);

}  // namespace hps
