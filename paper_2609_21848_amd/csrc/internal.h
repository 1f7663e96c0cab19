// Internal types of libdbbc: the host-side graph, the counting plan and the
// device-resident handle.  Nothing here crosses the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dbbc.h"

namespace dbbc {

// One side of the bipartite graph in priority order.  Vertex "side rank"
// sr in [0, n) is the position of the vertex among its own side in the order
// of Definition 3 (sr 0 = highest priority).  Row sr of the CSR lists the
// neighbours on the other side, as packed words (nbr_sr << 1) | neg, sorted
// by nbr_sr (hence by priority).
struct HostSide {
  int32_t n = 0;
  std::vector<uint32_t> off;   // n + 1
  std::vector<uint32_t> adj;   // m packed entries
  std::vector<int32_t> rev;    // per entry e of row x: index of x inside the row of adj[e] >> 1
  std::vector<int32_t> cut;    // per row: number of neighbours of higher priority
  std::vector<int32_t> grank;  // side rank -> rank in the merged order of both sides
  std::vector<int32_t> orig;   // side rank -> input id
  std::vector<uint32_t> rec;   // per entry: the input record it came from (U side only)
  int64_t max_deg = 0;
};

struct HostGraph {
  int32_t n_u = 0, n_v = 0;
  int64_t m = 0;       // distinct edges
  int64_t m_in = 0;    // input records (duplicates included)
  int64_t dups_dropped = 0;
  int64_t wedges_vp = 0;
  int64_t pivots_active = 0;
  // entries of the top T x T block of side 0 (rows and columns in priority
  // order) for T = 4096, 2048, 1024; -1 where not counted at build time
  int64_t hub_nnz[3] = {-1, -1, -1};
  bool arrays = false;  // the per-row and per-entry arrays of side[] are filled
  HostSide side[2];     // 0 = U, 1 = V
};

// The graph is built on the device (build.hip, build_device_graph), which
// fills the sizes above; the arrays of side[] are copied from the device
// only for the host planner (per-vertex plans).

// ---- counting plan -----------------------------------------------------------

// A segment is a run of consecutive CSR entries of one row, all of which end
// a wedge of the same work item; g is the negative-bit of the item's first
// edge of those wedges (pivot-mid edge, or tail-mid edge for reverse items).
struct Segment {
  uint32_t start;   // absolute index into the other side's adj array
  uint32_t len_g;   // (len << 1) | g
};

enum ItemKind : uint8_t {
  kForwardWindow = 0,  // pivot inside the window, endpoints inside the window
  kReverseTail = 1,    // endpoint below the window, pivot in the reverse window
  kForwardTail = 2,    // pivot below the window, counted from the pivot
  kReverseMid = 3,     // endpoint below the window, pivot in the window but
                       // not in the reverse window
};

// Small items are packed into groups that one wavefront counts in a single
// hash table; a group holds at most this many wedges (the table has twice as
// many slots).  Inside a group, segments carry the item's index in the group
// in the high half of len_g: (index << 16) | (len << 1) | g.
constexpr uint32_t kSmallGroupWork = 512;
// ... and at most this many items (the walk's staging tags of a group's
// runs, item index << 1 | g with a presence bit, fit 16 bits).
constexpr uint32_t kSmallMaxItems = 16383;

// Reverse items keep two 8-bit counters per key (symmetric, asymmetric), so
// a reverse item (or item part) has at most this many segments.
constexpr uint32_t kReverseMaxSegs = 255;
// ... and at most this many in a count plan, whose reverse kernel sums the
// counters' squares and products with signed 8-bit matrix products.
constexpr uint32_t kReverseCountMaxSegs = 127;

// Flags of an item.
enum : uint32_t {
  kItemMultiPart = 1u,  // partial counts go to a global accumulator
  kItemHubPairs = 2u,   // keys below hub_T are flushed to the hub-pair buffer
  kItemPacked = 4u,     // per-vertex direct item: p and n share one 32-bit word
};

struct Item {
  uint32_t seg_begin;
  uint32_t seg_count;
  int32_t owner;      // side rank of the pivot (forward) or endpoint (reverse)
  int32_t key_lo;     // keys counted lie in [key_lo, key_hi)
  int32_t key_hi;
  int32_t acc_slot;   // multi-part accumulator slot (or -1)
  uint32_t flags;
  uint32_t side;      // side of the owner and of the keys (0 = U, 1 = V)
  uint32_t work;      // wedges of the item (saturated at 2^32 - 1)
  uint32_t graph;     // index of the item's graph in a batch (0 alone)
};

struct Reduce {       // one multi-part accumulator to reduce after its parts
  int32_t acc_slot;   // first slot; the parts use acc_slot .. acc_slot + n_parts - 1
  int32_t n_parts;
  int32_t owner;
  int32_t key_lo, key_hi;
  uint32_t flags;
  uint32_t side;
  uint32_t graph;
};

struct PlanParams {
  int32_t hub_T = 0;
  int32_t window_L = 0;
  int32_t reverse_L = 0;
  int32_t small_work = 0;
  int32_t part_work = 0;
  bool per_vertex = false;  // plan for the per-vertex pass (no multi-part items)
  bool wide_all = false;    // per-vertex plans: flag every run kMidWide
  bool host_planner = false;  // count plans: make the plan on the host
  bool operator==(const PlanParams& o) const {
    return hub_T == o.hub_T && window_L == o.window_L && reverse_L == o.reverse_L &&
           small_work == o.small_work && part_work == o.part_work && per_vertex == o.per_vertex &&
           wide_all == o.wide_all && host_planner == o.host_planner;
  }
};

// Largest reverse window: keys of a reverse item index a per-wavefront LDS
// array of this many counters.
constexpr int32_t kMaxReverseL = 4096;

// Largest dense block of the per-vertex pass: the hub tally keeps 32-bit p
// and n per hub endpoint in LDS.
constexpr int32_t kMaxPVHubT = 4096;
// Work of one part of a hub pivot's tally (parts of one pivot add into its row).
constexpr int64_t kHubTallyPartWork = int64_t{1} << 16;

// Key window of a direct item of the per-vertex pass (32-bit counters in
// LDS); wider windows are split into items that share their runs.
constexpr int32_t kPVWindow = 16384;
// Items whose keys' p and n stay below 2^16 pack p and n into one 32-bit
// word and take twice the window (the largest window_L: one walk per pivot);
// see pv_packed.
constexpr int32_t kPVWindowPacked = 2 * kPVWindow;

// Whether a per-vertex direct item may pack its counters: a key gets at most
// one wedge per run, and a pair's p + n is at most the key's degree.  So an
// item with fewer than 2^16 runs packs; so does a hub pivot's item when every
// key past the dense block has degree below 2^16 (deg_T: the degree of the
// side's row T, the largest among its rows from T on; 0 when T is the side's
// size): its keys below T are hub pairs, whose counters are never read, and
// an overflow there stays inside the key's own word.
constexpr bool pv_packed(uint32_t seg_count, bool hub, int64_t deg_T) {
  return seg_count < 65536u || (hub && deg_T < 65536);
}

// Flag in a per-vertex plan's run mid (seg_mid, small_seg_mid): the mid's
// degree times the largest degree of the keys' side reaches 2^32, so an edge
// of the run may lie in 2^32 or more butterflies and its per-edge credits
// cannot share one 64-bit word (balanced low, unbalanced high).  Side ranks
// are below 2^30, so the bit is free.
constexpr uint32_t kMidWide = 1u << 30;

struct HostPlan {
  PlanParams p;
  int32_t L[2] = {0, 0};  // window per side
  int32_t R[2] = {0, 0};  // reverse window per side (R <= L)
  int32_t T[2] = {0, 0};  // hub block rows per side (pairs on that side)
  std::vector<Segment> segs;
  std::vector<Item> small_items;   // items counted with per-wavefront hash counters
  std::vector<Item> small_groups;  // ... packed into groups (segments in small_segs)
  std::vector<Segment> small_segs; // tagged segments of the groups
  // per-vertex plans only: the mid (row) of every run, the position of the
  // run's first edge in its side's CSR (the pivot-mid edge of forward runs,
  // the endpoint-mid edge of reverse runs), and the owner of every item of
  // every group (a group's owners start at its acc_slot)
  std::vector<uint32_t> seg_mid, small_seg_mid;
  std::vector<uint32_t> seg_edge, small_seg_edge;
  std::vector<int32_t> small_owner;
  int32_t key_bits[2] = {1, 1};    // per side: bits of a side rank in a group hash key
  std::vector<Item> direct_items;  // workgroup direct arrays over [0, L)
  std::vector<Item> hash_items;    // workgroup hash counters, large tail pivots
  std::vector<Item> reverse_items; // per-wavefront direct arrays over [0, R)
  std::vector<Reduce> reduces;
  // list lengths (direct, reverse, small groups, hash, reduces) once the
  // lists live on the device only
  int32_t n_items_kept[5] = {0, 0, 0, 0, 0};
  int32_t n_reverse_side0 = 0;  // reverse items are listed side 0 first
  int32_t n_direct_side0 = 0;   // per-vertex plans: direct items side 0 first
  int32_t acc_slots = 0;
  int32_t acc_width = 0;           // max window over the sides
  // per sparse kernel (0 = direct, 1 = small, 2 = hash, 3 = reverse):
  // wedges and segments
  int64_t k_wedges[4] = {0, 0, 0, 0};
  int64_t k_segs[4] = {0, 0, 0, 0};
  int64_t w_sparse = 0;            // wedges tallied by the sparse kernels
  int64_t w_skipped = 0;           // wedges of items that cannot contribute
  // dense hub block per side s (pairs on s): row-major int8 matrices
  // [T[s] x T[1-s]] of signs (B) and of signs masked to lower-priority mids (Bm)
  std::vector<int8_t> hub_B[2], hub_Bm[2];
  // per-vertex plans with a dense block: for every hub pivot x < T[s] (one
  // item each, both sides, side 0 first), the runs of its sparse wedges
  // toward hub endpoints w < T[s] (mids y >= T[1 - s]), so that a tally of
  // these alone gives the hub pairs' sparse counts before the dense block
  // completes them; the items' keys are [x + 1, T[s]); a heavy pivot's runs
  // are split over several items (parts) of the same owner
  std::vector<Segment> hub_segs;
  std::vector<Item> hub_items;
  int32_t n_hub_side0 = 0;
};

// Sizes a plan is checked against before its 32-bit indices are formed:
// runs are addressed by uint32 indices (Item::seg_begin), work lists and
// reduces are launched with int32 counts, accumulator slots are int32.
struct PlanSizes {
  uint64_t runs = 0;       // runs of the plan
  uint64_t items = 0;      // the longest list of items of one kind
  uint64_t reduces = 0;    // multi-part reduces
  uint64_t acc_slots = 0;  // multi-part accumulator slots
};
// DBBC_OK, or DBBC_E_TOO_LARGE with err set when a size exceeds its type.
int check_plan_sizes(const PlanSizes& z, std::string& err);

// hub_slots: dense-block tiles (128 x 128 workgroups) the device runs at
// once; the default block is trimmed so that its upper triangle of tiles
// fits in one round.
PlanParams default_params(const HostGraph& g, int32_t hub_slots = 512);
// Checks of the plan knobs (a DBBC status; err filled on failure).
int check_plan_params(const PlanParams& p, std::string& err);
// The windows L, R, the dense block T per side and the accumulator width of
// a plan of a graph with n[s] vertices per side.
void plan_windows(const int32_t n[2], const PlanParams& p, HostPlan& plan);
int make_plan(const HostGraph& g, const PlanParams& p, HostPlan& plan, std::string& err);

}  // namespace dbbc
