// Library-internal entry points shared by the C ABI and the request loop: the solve of
// one factor, or of several factors' problems together, on an explicit stream, the size
// of its workspace, and the workspace pool.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <vector>

#include "../../include/hps.h"

namespace hps {

// Device bytes one solve call of f with nrhs right-hand sides allocates for its
// workspace (with or without a body load s); host arithmetic only.
size_t solve_workspace_bytes(hps_factor* f, int nrhs, bool with_s);

// hps_solve on stream st; the residual-correction record goes to *info.  Throws
// hps::Error on failure.
void solve_on(hps_factor* f, int nrhs, const double* s, const double* t, double* u,
              hipStream_t st, hps_solve_info* info);

// One request's share of a solve over several problems: nrhs right-hand sides of factor
// f's problem (s may be NULL), solution into u; pointers as for hps_solve.
struct SolvePart {
  hps_factor* f = nullptr;
  int nrhs = 0;
  const double* s = nullptr;
  const double* t = nullptr;
  double* u = nullptr;
};
// Whether the problems of a and b can share one solve's launches (same leaf grid, p and
// level precisions, no residual correction).
bool solve_shareable(const hps_factor* a, const hps_factor* b);
// Most distinct problems one shared solve takes.
int solve_share_max();
// Solve the parts (pairwise shareable problems, at most solve_share_max() distinct; parts
// of one problem take consecutive right-hand-side columns) with one launch per level
// step on stream st.  With bytes set, only returns the device bytes the call allocates.
// Throws hps::Error.
void solve_parts(const std::vector<SolvePart>& parts, hipStream_t st, size_t* bytes = nullptr);

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

// The caller's allocator hook (hps_set_allocator).  hook_alloc returns nullptr when no
// hook is installed and throws hps::Error when the hook has no memory; hook_free hands p
// back to the hook that provided it (after synchronizing the device when sync_device is
// set) and returns false for memory no hook provided.
void set_hook(hps_alloc_fn alloc, hps_free_fn free, void* ctx);
void* hook_alloc(size_t bytes, hipStream_t st);
bool hook_free(void* p, hipStream_t st, bool sync_device = false);
// Device memory from the hook when one is installed, else hipMalloc; dev_free returns it
// (hipFree waits for the device; hooked memory is handed back after a device
// synchronization).  dev_alloc throws hps::Error.
void* dev_alloc(size_t bytes);
void dev_free(void* p);

// Message hps_last_error() returns on the calling thread.
void set_last_error(const std::string& msg);

}  // namespace hps
