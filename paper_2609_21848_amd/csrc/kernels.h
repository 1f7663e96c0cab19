// Kernel argument blocks and launchers shared by the host code and the HIP
// kernels of libdbbc.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace dbbc {

// Zero words appended to every CSR entry array: a 16-byte load may start at
// the last entry of a run.
constexpr size_t kAdjPad = 64;

// Layout of a graph's int64 result slot (res + graph * kResStride).
enum : int {
  kResBalanced = 0,
  kResUnbalanced = 1,
  kResTotal = 2,
  kResDenseWedges = 3,
  kResStride = 4,
};
enum : unsigned long long {
  kErrHashFull = 1ull,
  kErrLdsLayout = 2ull,  // an LDS array lacks the alignment its addressing assumes
};

// Per graph and side s (the side of an item's keys): where the item's
// segments point and where hub-pair partial counts go.  Kernels read them
// from a table indexed 2 * item.graph + item.side.
struct DevSideConst {
  const uint32_t* other_adj;     // CSR entries of the other side (entries are side-s ranks)
  const Segment* segs;           // the graph's runs (direct, reverse and hash items)
  const Segment* small_segs;     // the graph's tagged runs (small-item groups)
  int32_t* hub_xy;               // [2 x T x T]: p + n, then p - n, of each hub pair's
                                 // sparse wedges (w > x), or null
  uint32_t* acc;                 // the graph's multi-part accumulators
  int32_t T;                     // hub rows of side s (0 = no dense path)
  int32_t R;                     // reverse window of side s
  int32_t key_bits;              // bits of a side-s rank in a small-group hash key
  int32_t acc_width;             // words per accumulator slot
  // per-vertex pass only
  const uint32_t* seg_mid;        // mid (other-side rank) of every run of segs
  const uint32_t* small_seg_mid;  // ... of every run of small_segs
  const int32_t* small_owner;     // owners of the items of the groups (from acc_slot)
  const int32_t* orig;            // side-s rank -> input id
  const int32_t* orig_mid;        // other-side rank -> input id
  unsigned long long* bal;        // per-vertex outputs of side s (input id order)
  unsigned long long* unb;
  unsigned long long* bal_mid;    // ... of the other side
  unsigned long long* unb_mid;
  // key credits of the direct items by side-s rank (their keys are below
  // the window, kPVKeyRanks), added to bal / unb after the direct launches
  unsigned long long* key_bal;
  unsigned long long* key_unb;
  // per-edge credits (per-edge pass only): every wedge credits its two
  // edges, the run's first edge (a position in side s's CSR) and the walked
  // entry (a position in the other side's CSR).  Credits of runs without the
  // kMidWide flag go to one word per edge, balanced in the low and
  // unbalanced in the high 32 bits; those of wide runs to two words.  (The
  // dense block splits its edges the same way, by row.)
  const uint32_t* seg_edge;       // position of every run's first edge in side s's CSR
  const uint32_t* small_seg_edge; // ... of every run of small_segs
  unsigned long long* epack;      // [m] by position in side s's CSR
  unsigned long long* ewb;        // [m] wide balanced
  unsigned long long* ewu;        // [m] wide unbalanced
  unsigned long long* epack_o;    // ... by position in the other side's CSR
  unsigned long long* ewb_o;
  unsigned long long* ewu_o;
};

struct DirectArgs {
  const Item* items;
  const DevSideConst* sides;
  uint32_t* queue;
  unsigned long long* res;   // per-graph result slots
  unsigned long long* err;   // kErr* bits
  int32_t n_items;
  uint32_t long_len;  // runs at least this long are streamed by the whole wavefront
};

// Reverse items (items) or small-item groups (items = groups, segs tagged).
struct SmallArgs {
  const Item* items;
  const DevSideConst* sides;
  unsigned long long* res;   // per-graph result slots
  unsigned long long* err;   // kErr* bits
  int32_t n_items;
  uint32_t long_len;
};

struct HashArgs {
  const Item* items;
  const DevSideConst* sides;
  uint32_t* queue;
  unsigned long long* res;   // per-graph result slots
  unsigned long long* err;   // kErr* bits
  int32_t n_items;
  uint32_t long_len;
};

struct ReduceArgs {
  const Reduce* reduces;
  const DevSideConst* sides;
  unsigned long long* res;   // per-graph result slots
  unsigned long long* err;   // kErr* bits
  int32_t n_reduces;
};

// Source of one graph's item (or reduce) list for the batch assembly copy.
struct AssembleSrc {
  const void* src;
  uint32_t n;
  uint32_t dst_off;  // first destination index
  uint32_t graph;    // index of the graph in the batch
};

// Dense hub block of one side: X = |Bm| |B|^T and Y = Bm B^T over the T_other
// mids, combined with the sparse hub-pair partials, reduced to res.  The
// contraction length is padded with zero columns to a multiple of kHubKPad.
constexpr int32_t kHubKPad = 64;
struct HubArgs {
  const int8_t* Bm = nullptr;    // [T x K] row-major, K = padded mid count
  const int8_t* B = nullptr;     // [T x K]
  int32_t* hub_xy = nullptr;     // [2 x T x T] sparse partials: p + n, then p - n
  unsigned long long* res = nullptr;  // res[0..2] sums, res[3] dense wedges
  int32_t T = 0;                 // rows (pairs side)
  int32_t K = 0;                 // padded contraction length (multiple of kHubKPad)
  // per-vertex pass only (bal != null): the completed counts X = P + N and
  // Y = P - N of every hub pair (x, w), w below x, are stored back into
  // hub_xy (zeros at w not below x), and each pair's C(P,2) + C(N,2) and
  // P N are credited to both its vertices; null in the count pass
  const int32_t* orig = nullptr;      // side rank -> input id
  unsigned long long* bal = nullptr;  // per-vertex outputs of the side (input id order)
  unsigned long long* unb = nullptr;
};

hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t st);
// Write the two side-table entries src2[0..2) (host values) to device
// memory dst by a kernel (no copy from host memory).
hipError_t launch_store_sides(const DevSideConst* src2, DevSideConst* dst, hipStream_t st);
hipError_t launch_direct(const DirectArgs& a, int grid, hipStream_t st);
hipError_t launch_small(const SmallArgs& a, int grid, hipStream_t st);
hipError_t launch_reverse(const SmallArgs& a, int grid, hipStream_t st);
hipError_t launch_hash(const HashArgs& a, int grid, hipStream_t st);
hipError_t launch_reduce(const ReduceArgs& a, int max_grid, hipStream_t st);
// The dense block of up to two sides (n <= 2) in one launch; sides with
// T = 0 are skipped.
hipError_t launch_hub(const HubArgs* sides, int n, hipStream_t st);
// Dense block of the per-vertex pass.
//  - launch_pv_hub_tally: the hub pairs' sparse counts, from the plan's hub
//    runs (one item per hub pivot x, keys (x, T)), stored as p + n and p - n
//    into row x of hub_xy (which starts at zero).
//  - launch_hub with bal set: completes and stores them (see HubArgs).
//  - launch_hub_digits: the completed X and Y (upper triangle) as kHubDigits
//    signed 7-bit digits, row-major and transposed, for the credit products.
//  - launch_hub_credit: the credits of the block's wedges (x - y - w, y a hub
//    mid), as products of the completed counts with the sign matrices:
//    for the pivot-mid edge (x, y), with ZX = X B+ and ZY = Y B (B+ = |B|),
//      2 bal = |Bm| (ZX - 2 Zc) + Bm ZY,   2 unb = |Bm| ZX - Bm ZY,
//    Zc[x][y] = #{w > x : B[w][y] != 0}; the mid y takes the column sums;
//    for the end-mid edge (w, y), with ZX' = X^T Bm+ and ZY' = Y^T Bm,
//      2 bal = |B| (ZX' - 2 Zc') + B ZY',   2 unb = |B| ZX' - B ZY',
//    Zc'[w][y] = #{x < w : Bm[x][y] != 0}.
constexpr int kHubDigitBits = 7;  // signed digits: v = sum_k d_k 2^(7 k)
struct HubTallyArgs {
  const Item* items;             // hub items (keys (owner, T))
  const Segment* segs;           // their runs
  const uint32_t* other_adj;     // CSR entries of the other side
  int32_t* hub_xy;               // [2 x T x T]
  int32_t n_items;
  int32_t T;
  uint32_t long_len;
};
struct HubDigitArgs {
  const int32_t* hub_xy;         // [2 x T x T] completed X, Y (upper triangle)
  int8_t* rows;                  // [2 (X, Y) x D x T x T] digits, row-major (row x)
  int8_t* cols;                  // [2 x D x T x T] digits, transposed (row w)
  int32_t T;
  int32_t D;                     // digits per value
};
struct HubCreditArgs {
  const int8_t* A;               // [2 (X, Y) x D x T x T] digits of the left operand
  const int8_t* Bt;              // [K x T] signs of the right operand, transposed (row y)
  const int8_t* E;               // [T x K] signs multiplying the products: Bm (pivot-mid) or B (end-mid)
  const int32_t* Zc;             // [T x K] the counts Zc or Zc'
  const int32_t* pos;            // [T x K] position of edge (row, y) in the side's CSR (or -1); null: no edges
  const int32_t* orig_mid;       // other-side rank -> input id (mid credits; null: none)
  unsigned long long* bal_mid;   // per-vertex outputs of the other side
  unsigned long long* unb_mid;
  unsigned long long* ewb;       // per-edge wide credits by position in the side's CSR
  unsigned long long* ewu;
  unsigned long long* epack;     // per-edge packed credits (balanced | unbalanced << 32)
  // rows whose degree d has d * max_deg_other < 2^32 keep their edges'
  // credits in the packed words, the others (all with wide_all) in ewb and ewu
  const uint32_t* off;           // [n + 1] the side's CSR row offsets
  int32_t n;
  unsigned long long max_deg_other;
  int32_t wide_all;
  int32_t T, K, D;
  int32_t upper;                 // 1: row r contracts over t > r (pivot-mid); 0: over t < r (end-mid)
};
hipError_t launch_pv_hub_tally(const HubTallyArgs* sides, int n, int grid, hipStream_t st);
hipError_t launch_hub_digits(const HubDigitArgs& a, hipStream_t st);
hipError_t launch_hub_credit(const HubCreditArgs& a, hipStream_t st);

// Per-vertex pass (plans made with per_vertex): direct items, reverse items,
// small-item groups and hash items.
hipError_t launch_pv_direct(const DirectArgs& a, int grid, hipStream_t st);
// Largest rank a per-vertex direct item's key may have (the widest window),
// and the adding of the rank-indexed key credits of side s (ranks below n)
// into its per-vertex outputs.
constexpr int32_t kPVKeyRanks = 32768;
hipError_t launch_pv_key_flush(const DevSideConst* sides, int32_t s, int32_t n, hipStream_t st);
hipError_t launch_pv_reverse(const SmallArgs& a, int grid, hipStream_t st);
hipError_t launch_pv_small(const SmallArgs& a, int grid, hipStream_t st);
hipError_t launch_pv_hash(const HashArgs& a, int grid, hipStream_t st);
// Per-edge outputs by input record: out[rec[k]] = e[0][k] + e[1][pos_v[k]]
// over the U-CSR positions k (e[s] holds the credits by position in side s's
// CSR, packed and wide words; records dropped as duplicates are not
// written).
struct EdgeCombineArgs {
  const unsigned long long* e_pack[2];
  const unsigned long long* e_wb[2];
  const unsigned long long* e_wu[2];
  const uint32_t* rec;    // [m] input record of U-CSR entry k
  const uint32_t* pos_v;  // [m] position of the same edge in the V CSR
  long long* out_bal;     // [m_in] by input record
  long long* out_unb;
  int64_t m;
  int32_t wide;           // 0: no run kept two-word credits (e_wb, e_wu are all zero)
  // Which edges can hold two-word credits (all with wide_all): those whose U
  // or V end has degree d with d * (the other side's largest degree) >= 2^32
  // (the runs of such mids are flagged wide, and the dense block keeps such
  // rows' credits in two words).  Side ranks are in non-increasing degree
  // order, so both sets are rank prefixes, found from the row offsets.
  const uint32_t* off_u;  // [n_u + 1] U-CSR row offsets
  const uint32_t* off_v;  // [n_v + 1]
  const uint32_t* adj_u;  // [m] U-CSR entries (V rank << 1 | negative)
  int32_t n_u, n_v;
  unsigned long long max_deg_u, max_deg_v;
  int32_t wide_all;
};

// The per-vertex pass with per-edge credits as well (the same plans).
hipError_t launch_pe_direct(const DirectArgs& a, int grid, hipStream_t st);
hipError_t launch_pe_reverse(const SmallArgs& a, int grid, hipStream_t st);
hipError_t launch_pe_small(const SmallArgs& a, int grid, hipStream_t st);
hipError_t launch_pe_hash(const HashArgs& a, int grid, hipStream_t st);
hipError_t launch_edge_combine(const EdgeCombineArgs& a, int grid, hipStream_t st);

// Explicit-verification count of one side's pivots (the wedge-separation
// baseline): per-workgroup scratch of 4 x n_s words and list_cap bytes.
struct ExplicitArgs {
  const uint32_t* off_s;    // side s CSR offsets [n_s + 1]
  const uint32_t* adj_s;    // side s entries
  const int32_t* rev_s;     // per side-s entry: index of its row vertex inside the other row
  const int32_t* cut_s;     // per side-s row: neighbours of higher priority
  const uint32_t* off_o;    // other side's CSR
  const uint32_t* adj_o;
  int32_t n_s;
  uint32_t* scratch;
  uint8_t* lists;
  int64_t list_cap;         // at least the wedges of any pivot
  uint32_t* queue;
  unsigned long long* res;  // result slot
  unsigned long long* err;
};
hipError_t launch_explicit(const ExplicitArgs& a, int grid, hipStream_t st);

// Copy k graphs' item lists (or reduce lists) into one list, setting each
// entry's graph field.
hipError_t launch_assemble_items(const AssembleSrc* srcs, int k, Item* dst, hipStream_t st);
hipError_t launch_assemble_reduces(const AssembleSrc* srcs, int k, Reduce* dst, hipStream_t st);

}  // namespace dbbc
