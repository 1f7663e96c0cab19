// Plans built on the device (plan_dev.hip): the same work split as make_plan
// (plan.cpp), count and per-vertex plans, from the device CSR, with kernels,
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
  int64_t max_deg[2] = {0, 0};
  const uint32_t* off[2] = {nullptr, nullptr};
  const uint32_t* adj[2] = {nullptr, nullptr};
  const int32_t* rev[2] = {nullptr, nullptr};
  const int32_t* cut[2] = {nullptr, nullptr};
  const int32_t* grank[2] = {nullptr, nullptr};
  const int32_t* ord[2] = {nullptr, nullptr};  // side rank -> input id
  const uint32_t* rec = nullptr;                // U-side entry -> input record
};

// The device lists of a plan (the layout the counting kernels read) and the
// dense block's sign matrices, padded to K columns.  Per-vertex plans add
// each run's mid and first-edge position, the small items' owners, the hub
// pivots' tally runs and items, and the constants of the block's credit
// products: B and Bm transposed (K x T), Zc[x][y] = #{w > x : B[w][y] != 0},
// Zc'[w][y] = #{x < w : Bm[x][y] != 0} and the CSR position of every hub
// edge (-1 where none), each T x K.
struct DevPlanLists {
  DevBuf segs, small_segs, small_groups, direct_items, hash_items, reverse_items, reduces, acc;
  DevBuf hub_B[2], hub_Bm[2];
  int32_t hub_K[2] = {0, 0};
  DevBuf seg_mid, seg_edge, small_seg_mid, small_seg_edge, small_owner, hub_items, hub_segs;
  DevBuf hub_Bt[2], hub_Bmt[2], hub_Zc[2], hub_Zcp[2], hub_pos[2];
  bool any_wide = false;  // some run keeps two-word edge credits (kMidWide)
};

// Build the plan of g for p on stream st.  Fills hp's scalars (windows,
// list sizes, per-kernel wedge and run totals, per-side list splits; its
// vectors stay empty) and the device lists, from the current allocator.
// Returns a DBBC status and fills err on failure.
int make_plan_device(const DevGraphView& g, const PlanParams& p, hipStream_t st, HostPlan& hp, DevPlanLists& out,
                     std::string& err);

// U-CSR position k -> the V-CSR position of the same edge (m entries).
int edge_positions_device(const DevGraphView& g, uint32_t* out, hipStream_t st, std::string& err);

}  // namespace dbbc
