// Device construction of the graph (build.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "devmem.h"
#include "internal.h"
#include "plan_dev.h"

namespace dbbc {

// Device arrays a build hands to its graph handle (from the current
// allocator; the handle takes them over): per side, the packed CSR entries
// (m words plus kAdjPad zero words), the row offsets (n + 1 words), each
// entry's position in the other side's row (rev, m words), each row's
// higher-priority prefix (cut, n), the global ranks and the input ids by
// side rank (grank, ord: n each); and the input record of every U-side
// entry (rec, m).
struct DeviceCsr {
  DevBuf adj[2];
  DevBuf off[2];
  DevBuf rev[2], cut[2], grank[2], ord[2];
  DevBuf rec;
};

// Build the relabelled CSR pair on the device from an edge list (host
// memory, or device memory with DBBC_INPUT_DEVICE), stream-ordered on st,
// and fill the sizes of g (its arrays stay empty: fetch_host_arrays).
// Returns a DBBC status and fills err on failure (nothing is handed over
// then).
int build_device_graph(int32_t n_u, int32_t n_v, int64_t m, const int32_t* u, const int32_t* v,
                       const int8_t* sign, uint32_t flags, hipStream_t st, HostGraph& g, DeviceCsr& out,
                       std::string& err);

// What a text ingestion hands to its graph handle besides the CSR: the
// per-side compact -> raw id maps (int64 arrays of ascending raw ids, from
// the current allocator; the handle takes them over) and the line and record
// counts.
struct IngestOut {
  int64_t lines = 0, records = 0;
  DevBuf raw[2];
};

// Parse an edge list in text form on the device (host text, or device text
// with DBBC_INPUT_DEVICE), compact each side's ids and build the graph as
// build_device_graph does.  Returns a DBBC status and fills err on failure
// (nothing is handed over then).
int ingest_text(const char* text, int64_t len, uint32_t flags, hipStream_t st, HostGraph& g, DeviceCsr& csr,
                IngestOut& out, std::string& err);

// Copy a built graph's arrays from the device into g.side[] (the host
// planner's input; a no-op when g already holds them).  Returns a DBBC
// status and fills err on failure.
int fetch_host_arrays(const DevGraphView& d, HostGraph& g, hipStream_t st, std::string& err);

}  // namespace dbbc
