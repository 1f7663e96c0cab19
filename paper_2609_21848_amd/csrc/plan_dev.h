// Counting plan built on the device (plan_dev.hip): the same work split as
// make_plan (plan.cpp) for count plans, from the device CSR, with kernels,
// scans and sorts instead of host loops.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "devmem.h"
#include "internal.h"

namespace dbbc {

// The device arrays of a built graph (per side: row offsets, packed
// entries, reverse positions, higher-priority prefix lengths, global ranks,
// input ids; the U side's input records).
struct DevGraphView {
  int32_t n[2] = {0, 0};
  int64_t m = 0;
  const uint32_t* off[2] = {nullptr, nullptr};
  const uint32_t* adj[2] = {nullptr, nullptr};
  const int32_t* rev[2] = {nullptr, nullptr};
  const int32_t* cut[2] = {nullptr, nullptr};
  const int32_t* grank[2] = {nullptr, nullptr};
  const int32_t* ord[2] = {nullptr, nullptr};  // side rank -> input id
  const uint32_t* rec = nullptr;                // U-side entry -> input record
};

// The device lists of a count plan (the layout the count kernels read) and
// the dense block's sign matrices, padded to K columns.
struct DevPlanLists {
  DevBuf segs, small_segs, small_groups, direct_items, hash_items, reverse_items, reduces, acc;
  DevBuf hub_B[2], hub_Bm[2];
  int32_t hub_K[2] = {0, 0};
};

// Build the count plan of g for p (p.per_vertex must be false) on stream st.
// Fills hp's scalars (windows, list sizes, per-kernel wedge and run totals;
// its vectors stay empty) and the device lists, from the current allocator.
// Returns a DBBC status and fills err on failure.
int make_plan_device(const DevGraphView& g, const PlanParams& p, hipStream_t st, HostPlan& hp, DevPlanLists& out,
                     std::string& err);

}  // namespace dbbc
