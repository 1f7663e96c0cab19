// Device construction of the graph (build.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "internal.h"

namespace dbbc {

// Device arrays a build hands to its graph handle (hipMalloc'ed; the handle
// frees them): per side, the packed CSR entries (m words plus kAdjPad zero
// words) and the row offsets (n + 1 words).
struct DeviceCsr {
  void* adj[2] = {nullptr, nullptr};
  size_t adj_bytes[2] = {0, 0};
  void* off[2] = {nullptr, nullptr};
  size_t off_bytes[2] = {0, 0};
};

// Build the relabelled CSR pair on the device from an edge list (host
// memory, or device memory with DBBC_INPUT_DEVICE), stream-ordered on st,
// and fill the host copy g that the planner reads.  Returns a DBBC status
// and fills err on failure (nothing is handed over then).
int build_device_graph(int32_t n_u, int32_t n_v, int64_t m, const int32_t* u, const int32_t* v,
                       const int8_t* sign, uint32_t flags, hipStream_t st, HostGraph& g, DeviceCsr& out,
                       std::string& err);

}  // namespace dbbc
