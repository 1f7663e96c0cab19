// The C ABI of libdbbc (include/dbbc.h): graph handles, plans and the
// stream-ordered launch sequence of a count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "build_dev.h"
#include "devmem.h"
#include "internal.h"
#include "kernels.h"
#include "plan_dev.h"

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

#define HIP_TRY(expr)                                                                \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(e_ == hipErrorOutOfMemory ? DBBC_E_OOM : DBBC_E_DEVICE,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                \
  } while (0)

struct DeviceInfo {
  int id = -1;
  int cus = 0;
  bool ok = false;
};

int current_device(DeviceInfo& di) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(DBBC_E_NO_DEVICE, "no HIP device");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(DBBC_E_NO_DEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(DBBC_E_NO_DEVICE, std::string("device is ") + prop.gcnArchName + ", need gfx950");
  di.id = dev;
  di.cus = prop.multiProcessorCount;
  di.ok = true;
  return DBBC_OK;
}

using dbbc::DevBuf;

// Copy v into b, growing b only when v does not fit.
template <class T>
hipError_t upload_reuse(DevBuf& b, const std::vector<T>& v, hipStream_t st) {
  hipError_t e = b.reserve(v.size() * sizeof(T));
  if (e != hipSuccess || v.empty()) return e;
  return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

template <class T>
hipError_t upload(DevBuf& b, const std::vector<T>& v, hipStream_t st) {
  hipError_t e = b.alloc(v.size() * sizeof(T));
  if (e != hipSuccess || v.empty()) return e;
  return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}


// Control block of a count: [0, 4) the result slot of a lone count,
// [4] kernel error bits, [8, 16) sixteen uint32 work-queue heads.
constexpr size_t kCtlWords = 16;
constexpr size_t kCtlErr = 4;
constexpr size_t kCtlQueues = 8;

struct DevPlan {
  dbbc::HostPlan host;
  DevBuf segs, small_segs, small_groups, direct_items, hash_items, reverse_items, reduces, acc, sides;
  DevBuf seg_mid, small_seg_mid, small_owner;  // per-vertex plans
  DevBuf seg_edge, small_seg_edge;
  DevBuf hub_pairs[2], hub_B[2], hub_Bm[2];
  int32_t hub_K[2] = {0, 0};
  // per-vertex plans with a dense block: hub tally runs and items, the
  // transposed signs, the counts Zc and Zc', the hub edges' CSR positions,
  // the digit planes of the completed counts, and the digits per value
  DevBuf hub_items, hub_segs;
  DevBuf hub_Bt[2], hub_Bmt[2], hub_Zc[2], hub_Zcp[2], hub_pos[2], hub_rows[2], hub_cols[2];
  int32_t hub_D[2] = {0, 0};
  dbbc::DevSideConst side[2] = {};  // host copy of the side table
  bool any_wide = false;  // per-vertex plans: some run keeps two-word edge credits
  bool valid = false;
  size_t bytes() const {
    size_t b = segs.bytes + small_segs.bytes + small_groups.bytes + direct_items.bytes +
               hash_items.bytes + reverse_items.bytes + reduces.bytes + acc.bytes + sides.bytes +
               seg_mid.bytes + small_seg_mid.bytes + small_owner.bytes + seg_edge.bytes +
               small_seg_edge.bytes;
    b += hub_items.bytes + hub_segs.bytes;
    for (int s = 0; s < 2; ++s)
      b += hub_pairs[s].bytes + hub_B[s].bytes + hub_Bm[s].bytes + hub_Bt[s].bytes + hub_Bmt[s].bytes +
           hub_Zc[s].bytes + hub_Zcp[s].bytes + hub_pos[s].bytes + hub_rows[s].bytes + hub_cols[s].bytes;
    return b;
  }
};

// HIP events around one kernel launch of a timed count.
struct KernelRec {
  std::string name;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int64_t wedges = 0, segments = 0, items = 0, macs = 0;
  float ms = 0.f;
};

// One dense hub launch (both sides of one graph).
struct HubLaunch {
  dbbc::HubArgs a[2];
  int n = 0;
  int64_t tiles = 0, macs = 0;
  const char* name = "hub";
};

// Everything one count (of one graph or of a batch) launches.
struct LaunchSet {
  const dbbc::Item* direct = nullptr;
  const dbbc::Item* reverse = nullptr;
  const dbbc::Item* small = nullptr;
  const dbbc::Item* hash = nullptr;
  const dbbc::Reduce* reduces = nullptr;
  int32_t n[5] = {0, 0, 0, 0, 0};  // direct, reverse, small, hash, reduces
  int64_t wedges[4] = {0, 0, 0, 0}, segs[4] = {0, 0, 0, 0};  // direct, small, hash, reverse
  const dbbc::DevSideConst* sides = nullptr;
  unsigned long long* res = nullptr;
  size_t n_res = 0;  // result words zeroed before the count
  unsigned long long* ctl = nullptr;
  std::vector<std::pair<unsigned long long*, size_t>> zero;  // hub-pair buffers
  std::vector<HubLaunch> hubs;
  uint32_t long_len = 0;
  int cus = 0;
};

// Begin / end one timed launch on stream st (no-ops when recs is null).
struct Timing {
  std::vector<KernelRec>* recs;
  size_t used = 0;
  hipStream_t st;
  int begin(hipStream_t s, const char* name, int64_t wedges, int64_t segs, int64_t items, int64_t macs) {
    if (!recs) return DBBC_OK;
    st = s;
    if (used == recs->size()) recs->emplace_back();
    KernelRec& r = (*recs)[used];
    for (auto& e : r.ev)
      if (!e) HIP_TRY(hipEventCreate(&e));
    r.name = name;
    r.wedges = wedges;
    r.segments = segs;
    r.items = items;
    r.macs = macs;
    HIP_TRY(hipEventRecord(r.ev[0], st));
    return DBBC_OK;
  }
  int end() {
    if (!recs) return DBBC_OK;
    HIP_TRY(hipEventRecord((*recs)[used++].ev[1], st));
    return DBBC_OK;
  }
};

#define RC_TRY(expr)                \
  do {                              \
    int rc_ = (expr);               \
    if (rc_ != DBBC_OK) return rc_; \
  } while (0)

// Enqueue a whole count on stream st.  Every buffer the kernels accumulate
// into is cleared by a fill kernel first (never a memset node, so that the
// sequence can be captured into a HIP graph and replayed).  The kernels run
// one after the other: the direct and reverse kernels each need most of a
// CU's LDS, so they cannot share CUs, and running them side by side on
// several streams was measured slower than in sequence.
int enqueue(const LaunchSet& L, hipStream_t st, Timing& tm) {
  HIP_TRY(dbbc::launch_fill_u64(L.ctl, kCtlWords, 0ull, st));
  if (L.res != L.ctl) HIP_TRY(dbbc::launch_fill_u64(L.res, L.n_res, 0ull, st));
  for (const auto& z : L.zero) HIP_TRY(dbbc::launch_fill_u64(z.first, z.second, 0ull, st));
  unsigned long long* err = L.ctl + kCtlErr;
  uint32_t* queues = reinterpret_cast<uint32_t*>(L.ctl + kCtlQueues);
  const int cus = L.cus;
  {
    dbbc::DirectArgs a{};
    a.items = L.direct;
    a.sides = L.sides;
    a.queue = queues + 0;
    a.res = L.res;
    a.err = err;
    a.n_items = L.n[0];
    a.long_len = L.long_len;
    RC_TRY(tm.begin(st, "direct", L.wedges[0], L.segs[0], a.n_items, 0));
    HIP_TRY(dbbc::launch_direct(a, std::min<int>(cus, std::max(1, a.n_items)), st));
    RC_TRY(tm.end());
  }
  {
    dbbc::SmallArgs a{};
    a.items = L.reverse;
    a.sides = L.sides;
    a.res = L.res;
    a.err = err;
    a.n_items = L.n[1];
    a.long_len = L.long_len;
    RC_TRY(tm.begin(st, "reverse", L.wedges[3], L.segs[3], a.n_items, 0));
    HIP_TRY(dbbc::launch_reverse(a, std::min<int>(cus, std::max(1, (a.n_items + 15) / 16)), st));
    RC_TRY(tm.end());
  }
  {
    dbbc::SmallArgs a{};
    a.items = L.small;
    a.sides = L.sides;
    a.res = L.res;
    a.err = err;
    a.n_items = L.n[2];
    a.long_len = L.long_len;
    RC_TRY(tm.begin(st, "small", L.wedges[1], L.segs[1], a.n_items, 0));
    HIP_TRY(dbbc::launch_small(a, std::min<int>(4 * cus, std::max(1, (a.n_items + 3) / 4)), st));
    RC_TRY(tm.end());
  }
  {
    dbbc::HashArgs a{};
    a.items = L.hash;
    a.sides = L.sides;
    a.queue = queues + 2;
    a.res = L.res;
    a.err = err;
    a.n_items = L.n[3];
    a.long_len = L.long_len;
    RC_TRY(tm.begin(st, "hash", L.wedges[2], L.segs[2], a.n_items, 0));
    HIP_TRY(dbbc::launch_hash(a, std::min<int>(cus, std::max(1, a.n_items)), st));
    RC_TRY(tm.end());
  }
  {
    dbbc::ReduceArgs a{};
    a.reduces = L.reduces;
    a.sides = L.sides;
    a.res = L.res;
    a.err = err;
    a.n_reduces = L.n[4];
    RC_TRY(tm.begin(st, "reduce", 0, 0, a.n_reduces, 0));
    HIP_TRY(dbbc::launch_reduce(a, 4 * cus, st));
    RC_TRY(tm.end());
  }
  for (const HubLaunch& h : L.hubs) {
    RC_TRY(tm.begin(st, h.name, 0, 0, h.tiles, h.macs));
    HIP_TRY(dbbc::launch_hub(h.a, h.n, st));
    RC_TRY(tm.end());
  }
  return DBBC_OK;
}

// Dense hub launches of a graph's plan, results into res (its slot); the
// hub-pair partials in hub_xy[s] (default: the plan's own buffers).
void add_hub_launches(DevPlan& d, unsigned long long* res, LaunchSet& L, int32_t* const* hub_xy = nullptr) {
  const dbbc::HostPlan& hp = d.host;
  HubLaunch h{};
  for (int s = 0; s < 2; ++s) {
    if (hp.T[s] == 0) continue;
    int32_t* xy = hub_xy ? hub_xy[s] : d.hub_pairs[s].as<int32_t>();
    // two int32 T x T planes, cleared as T x T 64-bit words
    L.zero.push_back({reinterpret_cast<unsigned long long*>(xy), static_cast<size_t>(hp.T[s]) * hp.T[s]});
    dbbc::HubArgs& a = h.a[h.n++];
    a.Bm = d.hub_Bm[s].as<int8_t>();
    a.B = d.hub_B[s].as<int8_t>();
    a.hub_xy = xy;
    a.res = res;
    a.T = hp.T[s];
    a.K = d.hub_K[s];
    // two contractions over K for every tile of the upper triangle
    const int64_t nt = a.T / 128;
    const int64_t tiles = nt * (nt + 1) / 2;
    h.tiles += tiles;
    h.macs += 2 * tiles * 128 * 128 * static_cast<int64_t>(a.K);
  }
  if (h.n > 0) L.hubs.push_back(h);
}

}  // namespace

struct dbbc_graph {
  dbbc::DevAlloc al;  // where the handle's device memory comes from (declared first: freed last)
  dbbc::HostGraph host;
  DeviceInfo dev;
  DevBuf adj[2], off[2];
  DevBuf ctl;
  unsigned long long* pinned = nullptr;  // host mirror of ctl
  DevPlan plan;
  uint64_t plan_gen = 0;  // bumped whenever the device plan is rebuilt
  DevPlan pv_plan;        // plan of the per-vertex pass
  DevBuf orig[2];         // side rank -> input id, per side
  DevBuf rev[2], cut[2], grank[2];  // per entry: position in the other row; per row: higher-priority
                                    // prefix; per row: global rank (the planners' input)
  DevBuf pv_out[2][2];    // per-vertex outputs [side][balanced, unbalanced]
  DevBuf pv_keys[2];      // per side: the direct items' key credits by rank (balanced, then unbalanced)
  DevBuf pe_out[2][3];    // per-edge credits by CSR position [side][packed, wide bal, wide unb]
  DevBuf edge_rec, edge_pos_v;  // U-CSR position -> input record, -> V-CSR position
  DevBuf pe_tmp;          // stands in for a NULL per-edge output
  DevBuf raw_ids[2];      // graphs read from text: compact -> raw id per side
  std::vector<KernelRec> timers;  // events are reused across timed counts
  size_t timers_used = 0;
  bool timed_valid = false;
  bool in_flight = false;  // an asynchronous count awaits dbbc_count_read
  mutable bool defaults_valid = false;  // default plan knobs, computed once
  mutable dbbc::PlanParams defaults;
  ~dbbc_graph() {
    if (pinned) (void)hipHostFree(pinned);
    for (auto& t : timers)
      for (auto& e : t.ev)
        if (e) (void)hipEventDestroy(e);
  }
};

struct dbbc_batch {
  dbbc::DevAlloc al;  // the allocator of the batch's first graph at creation
  std::vector<dbbc_graph*> gs;
  std::vector<uint64_t> gens;  // plan generation of each graph at creation
  DeviceInfo dev;
  DevBuf direct, reverse, small, hash, reduces, sides, srcs, res, ctl;
  LaunchSet L;
  unsigned long long* pinned = nullptr;  // k result slots, then the error word
  size_t pinned_words = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~dbbc_batch() {
    drop_graph();
    if (cap) (void)hipStreamDestroy(cap);
    if (pinned) (void)hipHostFree(pinned);
  }
};

namespace {

// The handle takes over the device arrays of its build.
void take_csr(dbbc_graph* g, dbbc::DeviceCsr& csr) {
  for (int s = 0; s < 2; ++s) {
    g->adj[s] = std::move(csr.adj[s]);
    g->off[s] = std::move(csr.off[s]);
    g->rev[s] = std::move(csr.rev[s]);
    g->cut[s] = std::move(csr.cut[s]);
    g->grank[s] = std::move(csr.grank[s]);
    g->orig[s] = std::move(csr.ord[s]);
  }
  g->edge_rec = std::move(csr.rec);
}

dbbc::DevGraphView view_of(const dbbc_graph* g) {
  dbbc::DevGraphView v;
  v.n[0] = g->host.n_u;
  v.n[1] = g->host.n_v;
  v.m = g->host.m;
  for (int s = 0; s < 2; ++s) {
    v.off[s] = g->off[s].as<uint32_t>();
    v.adj[s] = g->adj[s].as<uint32_t>();
    v.rev[s] = g->rev[s].as<int32_t>();
    v.cut[s] = g->cut[s].as<int32_t>();
    v.grank[s] = g->grank[s].as<int32_t>();
    v.ord[s] = g->orig[s].as<int32_t>();
    v.max_deg[s] = g->host.side[s].max_deg;
  }
  v.rec = g->edge_rec.as<uint32_t>();
  return v;
}

// The host copy of the graph's arrays (for the host planner), made once.
int ensure_host(dbbc_graph* g, hipStream_t st) {
  if (g->host.arrays) return DBBC_OK;
  std::string err;
  const int rc = dbbc::fetch_host_arrays(view_of(g), g->host, st, err);
  return rc == DBBC_OK ? DBBC_OK : fail(rc, err);
}

// Plans are made on the device unless the caller asks for the host planner,
// or the graph's entries or candidate items (three per vertex, four in a
// per-vertex plan) exceed the int sizes of the device scans.
bool plans_on_device(const dbbc_graph* g, const dbbc::PlanParams& p) {
  if (p.host_planner) return false;
  const int64_t kinds = p.per_vertex ? 4 : 3;
  return kinds * (static_cast<int64_t>(g->host.n_u) + g->host.n_v) + 1 <= INT32_MAX && g->host.m + 1 <= INT32_MAX;
}

int ensure_plan_into(dbbc_graph* g, const dbbc::PlanParams& p, hipStream_t st, DevPlan& d) {
  if (d.valid && d.host.p == p) return DBBC_OK;
  d.valid = false;
  if (&d == &g->plan) ++g->plan_gen;
  std::string err;
  dbbc::HostPlan hp;
  int rc;
  const bool on_device = plans_on_device(g, p);
  for (DevBuf* b : {&d.seg_mid, &d.small_seg_mid, &d.seg_edge, &d.small_seg_edge, &d.small_owner, &d.hub_items,
                    &d.hub_segs})
    b->release();
  if (on_device) {
    dbbc::DevPlanLists out;
    rc = dbbc::make_plan_device(view_of(g), p, st, hp, out, err);
    if (rc != DBBC_OK) return fail(rc, err);
    d.segs = std::move(out.segs);
    d.small_segs = std::move(out.small_segs);
    d.small_groups = std::move(out.small_groups);
    d.direct_items = std::move(out.direct_items);
    d.hash_items = std::move(out.hash_items);
    d.reverse_items = std::move(out.reverse_items);
    d.reduces = std::move(out.reduces);
    d.acc = std::move(out.acc);
    d.seg_mid = std::move(out.seg_mid);
    d.seg_edge = std::move(out.seg_edge);
    d.small_seg_mid = std::move(out.small_seg_mid);
    d.small_seg_edge = std::move(out.small_seg_edge);
    d.small_owner = std::move(out.small_owner);
    d.hub_items = std::move(out.hub_items);
    d.hub_segs = std::move(out.hub_segs);
    for (int s = 0; s < 2; ++s) {
      d.hub_B[s] = std::move(out.hub_B[s]);
      d.hub_Bm[s] = std::move(out.hub_Bm[s]);
      d.hub_K[s] = out.hub_K[s];
      d.hub_Bt[s] = std::move(out.hub_Bt[s]);
      d.hub_Bmt[s] = std::move(out.hub_Bmt[s]);
      d.hub_Zc[s] = std::move(out.hub_Zc[s]);
      d.hub_Zcp[s] = std::move(out.hub_Zcp[s]);
      d.hub_pos[s] = std::move(out.hub_pos[s]);
    }
    d.any_wide = out.any_wide;
  } else {
    rc = ensure_host(g, st);
    if (rc != DBBC_OK) return rc;
    try {
      rc = dbbc::make_plan(g->host, p, hp, err);
    } catch (const std::bad_alloc&) {
      return fail(DBBC_E_OOM, "host allocation failed while planning");
    }
    if (rc != DBBC_OK) return fail(rc, err);
    HIP_TRY(upload(d.segs, hp.segs, st));
    HIP_TRY(upload(d.seg_mid, hp.seg_mid, st));
    HIP_TRY(upload(d.small_seg_mid, hp.small_seg_mid, st));
    HIP_TRY(upload(d.seg_edge, hp.seg_edge, st));
    HIP_TRY(upload(d.small_seg_edge, hp.small_seg_edge, st));
    HIP_TRY(upload(d.small_owner, hp.small_owner, st));
    HIP_TRY(upload(d.small_segs, hp.small_segs, st));
    HIP_TRY(upload(d.small_groups, hp.small_groups, st));
    HIP_TRY(upload(d.direct_items, hp.direct_items, st));
    HIP_TRY(upload(d.hash_items, hp.hash_items, st));
    HIP_TRY(upload(d.reverse_items, hp.reverse_items, st));
    HIP_TRY(upload(d.reduces, hp.reduces, st));
    HIP_TRY(d.acc.alloc(static_cast<size_t>(hp.acc_slots) * hp.acc_width * sizeof(uint32_t)));
    if (p.per_vertex) {
      HIP_TRY(upload(d.hub_items, hp.hub_items, st));
      HIP_TRY(upload(d.hub_segs, hp.hub_segs, st));
    }
    hp.n_items_kept[0] = static_cast<int32_t>(d.direct_items.bytes / sizeof(dbbc::Item));
    hp.n_items_kept[1] = static_cast<int32_t>(d.reverse_items.bytes / sizeof(dbbc::Item));
    hp.n_items_kept[2] = static_cast<int32_t>(d.small_groups.bytes / sizeof(dbbc::Item));
    hp.n_items_kept[3] = static_cast<int32_t>(d.hash_items.bytes / sizeof(dbbc::Item));
    hp.n_items_kept[4] = static_cast<int32_t>(d.reduces.bytes / sizeof(dbbc::Reduce));
  }
  for (int s = 0; s < 2; ++s) {
    d.hub_pairs[s].release();
    if (!on_device) {
      for (DevBuf* b : {&d.hub_B[s], &d.hub_Bm[s], &d.hub_Bt[s], &d.hub_Bmt[s], &d.hub_Zc[s], &d.hub_Zcp[s],
                        &d.hub_pos[s]})
        b->release();
      d.hub_K[s] = 0;
    }
    d.hub_rows[s].release();
    d.hub_cols[s].release();
    d.hub_D[s] = 0;
    const int32_t T = hp.T[s], TO = hp.T[1 - s];
    if (T == 0) continue;
    HIP_TRY(d.hub_pairs[s].alloc(2 * static_cast<size_t>(T) * T * sizeof(int32_t)));
    if (p.per_vertex) {
      // a pair's counts are at most the side's largest degree: digits of
      // kHubDigitBits bits, enough for that bound with a signed top digit
      int32_t D = 1;
      while ((int64_t{1} << (dbbc::kHubDigitBits * D)) <= g->host.side[s].max_deg) ++D;
      d.hub_D[s] = D;
      HIP_TRY(d.hub_rows[s].alloc(2 * static_cast<size_t>(D) * T * T));
      HIP_TRY(d.hub_cols[s].alloc(2 * static_cast<size_t>(D) * T * T));
    }
    if (on_device) continue;  // the device planner wrote B, Bm and the credit products' constants
    // pad the contraction dimension to a multiple of kHubKPad
    const int32_t K = (TO + dbbc::kHubKPad - 1) / dbbc::kHubKPad * dbbc::kHubKPad;
    std::vector<int8_t> B(static_cast<size_t>(T) * K, 0), Bm(static_cast<size_t>(T) * K, 0);
    for (int32_t x = 0; x < T; ++x) {
      std::memcpy(&B[static_cast<size_t>(x) * K], &hp.hub_B[s][static_cast<size_t>(x) * TO], TO);
      std::memcpy(&Bm[static_cast<size_t>(x) * K], &hp.hub_Bm[s][static_cast<size_t>(x) * TO], TO);
    }
    if (p.per_vertex) {
      // the credit products' constants: B and Bm transposed (rows y), Zc[x][y]
      // = #{w > x : B[w][y] != 0}, Zc'[w][y] = #{x < w : Bm[x][y] != 0}, and
      // the CSR position of every hub edge (x, y) of this side
      const size_t TK = static_cast<size_t>(T) * K;
      std::vector<int8_t> Bt(TK, 0), Bmt(TK, 0);
      std::vector<int32_t> Zc(TK, 0), Zcp(TK, 0), pos(TK, -1);
      for (int32_t x = 0; x < T; ++x)
        for (int32_t y = 0; y < K; ++y) {
          Bt[static_cast<size_t>(y) * T + x] = B[static_cast<size_t>(x) * K + y];
          Bmt[static_cast<size_t>(y) * T + x] = Bm[static_cast<size_t>(x) * K + y];
        }
      for (int32_t y = 0; y < K; ++y) {
        int32_t below = 0;  // rows w > x with B[w][y] != 0, for x from the bottom up
        for (int32_t x = T - 1; x >= 0; --x) {
          Zc[static_cast<size_t>(x) * K + y] = below;
          below += B[static_cast<size_t>(x) * K + y] != 0;
        }
        int32_t above = 0;  // rows x < w with Bm[x][y] != 0
        for (int32_t w = 0; w < T; ++w) {
          Zcp[static_cast<size_t>(w) * K + y] = above;
          above += Bm[static_cast<size_t>(w) * K + y] != 0;
        }
      }
      const dbbc::HostSide& S = g->host.side[s];
      for (int32_t x = 0; x < T; ++x)
        for (uint32_t q = S.off[x]; q < S.off[x + 1]; ++q) {
          const int32_t y = static_cast<int32_t>(S.adj[q] >> 1);
          if (y >= TO) break;  // rows are sorted by rank
          pos[static_cast<size_t>(x) * K + y] = static_cast<int32_t>(q);
        }
      HIP_TRY(upload(d.hub_Bt[s], Bt, st));
      HIP_TRY(upload(d.hub_Bmt[s], Bmt, st));
      HIP_TRY(upload(d.hub_Zc[s], Zc, st));
      HIP_TRY(upload(d.hub_Zcp[s], Zcp, st));
      HIP_TRY(upload(d.hub_pos[s], pos, st));
      HIP_TRY(hipStreamSynchronize(st));  // the host vectors leave scope
    }
    HIP_TRY(upload(d.hub_B[s], B, st));
    HIP_TRY(upload(d.hub_Bm[s], Bm, st));
    d.hub_K[s] = K;
    hp.hub_B[s].clear();
    hp.hub_B[s].shrink_to_fit();
    hp.hub_Bm[s].clear();
    hp.hub_Bm[s].shrink_to_fit();
  }
  for (int s = 0; s < 2; ++s) {
    dbbc::DevSideConst& c = d.side[s];
    c = dbbc::DevSideConst{};
    c.other_adj = g->adj[1 - s].as<uint32_t>();
    c.segs = d.segs.as<dbbc::Segment>();
    c.small_segs = d.small_segs.as<dbbc::Segment>();
    c.hub_xy = d.hub_pairs[s].as<int32_t>();
    c.acc = d.acc.as<uint32_t>();
    c.T = hp.T[s];
    c.R = hp.R[s];
    c.key_bits = hp.key_bits[s];
    c.acc_width = hp.acc_width;
    if (p.per_vertex) {
      c.seg_mid = d.seg_mid.as<uint32_t>();
      c.small_seg_mid = d.small_seg_mid.as<uint32_t>();
      c.small_owner = d.small_owner.as<int32_t>();
      c.orig = g->orig[s].as<int32_t>();
      c.orig_mid = g->orig[1 - s].as<int32_t>();
      c.bal = g->pv_out[s][0].as<unsigned long long>();
      c.unb = g->pv_out[s][1].as<unsigned long long>();
      c.bal_mid = g->pv_out[1 - s][0].as<unsigned long long>();
      c.unb_mid = g->pv_out[1 - s][1].as<unsigned long long>();
      c.key_bal = g->pv_keys[s].as<unsigned long long>();
      c.key_unb = c.key_bal + dbbc::kPVKeyRanks;
      c.seg_edge = d.seg_edge.as<uint32_t>();
      c.small_seg_edge = d.small_seg_edge.as<uint32_t>();
      c.epack = g->pe_out[s][0].as<unsigned long long>();
      c.ewb = g->pe_out[s][1].as<unsigned long long>();
      c.ewu = g->pe_out[s][2].as<unsigned long long>();
      c.epack_o = g->pe_out[1 - s][0].as<unsigned long long>();
      c.ewb_o = g->pe_out[1 - s][1].as<unsigned long long>();
      c.ewu_o = g->pe_out[1 - s][2].as<unsigned long long>();
    }
  }
  HIP_TRY(d.sides.alloc(sizeof(d.side)));
  HIP_TRY(hipMemcpyAsync(d.sides.p, d.side, sizeof(d.side), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (!on_device) {
    d.any_wide = false;
    for (const auto* v : {&hp.seg_mid, &hp.small_seg_mid})
      for (uint32_t mid : *v) d.any_wide = d.any_wide || (mid & dbbc::kMidWide) != 0;
  }
  // the host plan keeps only what later launches need
  hp.segs.clear();
  hp.segs.shrink_to_fit();
  hp.seg_mid.clear();
  hp.seg_mid.shrink_to_fit();
  hp.small_seg_mid.clear();
  hp.small_seg_mid.shrink_to_fit();
  hp.seg_edge.clear();
  hp.seg_edge.shrink_to_fit();
  hp.small_seg_edge.clear();
  hp.small_seg_edge.shrink_to_fit();
  hp.small_owner.clear();
  hp.small_owner.shrink_to_fit();
  hp.hub_items.clear();
  hp.hub_items.shrink_to_fit();
  hp.hub_segs.clear();
  hp.hub_segs.shrink_to_fit();
  hp.small_segs.clear();
  hp.small_segs.shrink_to_fit();
  hp.small_items.clear();
  hp.small_items.shrink_to_fit();
  for (auto* v : {&hp.small_groups, &hp.direct_items, &hp.hash_items, &hp.reverse_items}) {
    v->clear();
    v->shrink_to_fit();
  }
  hp.reduces.clear();
  hp.reduces.shrink_to_fit();
  d.host = std::move(hp);
  d.valid = true;
  return DBBC_OK;
}

int ensure_plan(dbbc_graph* g, const dbbc::PlanParams& p, hipStream_t st) {
  return ensure_plan_into(g, p, st, g->plan);
}

// Runs of at least this many entries are streamed by a whole wavefront.
constexpr int32_t kDefaultLongLen = 128;

int params_from(const dbbc_graph* g, const dbbc_options* opt, dbbc::PlanParams& p, uint32_t& long_len) {
  if (!g->defaults_valid) {
    g->defaults = dbbc::default_params(g->host, 2 * g->dev.cus);  // two hub workgroups per CU
    g->defaults_valid = true;
  }
  p = g->defaults;
  long_len = kDefaultLongLen;
  if (!opt) return DBBC_OK;
  if (opt->flags & ~(DBBC_OPT_TIME_KERNELS | DBBC_OPT_WIDE_EDGES | DBBC_OPT_HOST_PLAN))
    return fail(DBBC_E_INVALID_ARG, "unknown dbbc_options flag");
  p.host_planner = (opt->flags & DBBC_OPT_HOST_PLAN) != 0;
  if (opt->hub_T >= 0) p.hub_T = opt->hub_T;
  if (opt->window_L >= 0) p.window_L = opt->window_L;
  if (opt->reverse_L >= 0) p.reverse_L = opt->reverse_L;
  if (opt->window_L >= 0 && opt->reverse_L < 0) p.reverse_L = std::min(p.reverse_L, p.window_L);
  if (opt->small_work >= 0) p.small_work = opt->small_work;
  if (opt->part_work >= 0) p.part_work = opt->part_work;
  if (opt->long_len >= 0) {
    if (opt->long_len < 16 || opt->long_len > 65536)
      return fail(DBBC_E_INVALID_ARG, "long_len must be in [16, 65536]");
    long_len = static_cast<uint32_t>(opt->long_len);
  }
  if (p.hub_T > p.window_L) p.hub_T = std::min(p.hub_T, p.window_L);
  return DBBC_OK;
}

// The launch set of a lone count of g (results into g's control block).
LaunchSet lone_launches(dbbc_graph* g, uint32_t long_len) {
  DevPlan& d = g->plan;
  const dbbc::HostPlan& hp = d.host;
  LaunchSet L;
  L.direct = d.direct_items.as<dbbc::Item>();
  L.reverse = d.reverse_items.as<dbbc::Item>();
  L.small = d.small_groups.as<dbbc::Item>();
  L.hash = d.hash_items.as<dbbc::Item>();
  L.reduces = d.reduces.as<dbbc::Reduce>();
  for (int k = 0; k < 5; ++k) L.n[k] = hp.n_items_kept[k];
  for (int k = 0; k < 4; ++k) {
    L.wedges[k] = hp.k_wedges[k];
    L.segs[k] = hp.k_segs[k];
  }
  L.sides = d.sides.as<dbbc::DevSideConst>();
  L.ctl = g->ctl.as<unsigned long long>();
  L.res = L.ctl;
  L.n_res = dbbc::kResStride;
  add_hub_launches(d, L.res, L);
  L.long_len = long_len;
  L.cus = g->dev.cus;
  return L;
}

int check_graph(const dbbc_graph* g) {
  if (!g) return fail(DBBC_E_INVALID_ARG, "NULL graph");
  if (g->in_flight) return fail(DBBC_E_INVALID_ARG, "the graph has an asynchronous count in flight");
  return DBBC_OK;
}

void read_counts(const dbbc_graph* g, const unsigned long long* slot, dbbc_counts* out) {
  out->balanced = static_cast<int64_t>(slot[dbbc::kResBalanced]);
  out->unbalanced = static_cast<int64_t>(slot[dbbc::kResUnbalanced]);
  out->total = static_cast<int64_t>(slot[dbbc::kResTotal]);
  out->wedges = g->host.wedges_vp;
}

// Plan (if needed) and enqueue a lone count of g, then the copy of its
// control block to pinned host memory.
int enqueue_lone(dbbc_graph* g, const dbbc_options* opt, hipStream_t st) {
  dbbc::PlanParams p;
  uint32_t long_len = 0;
  int rc = params_from(g, opt, p, long_len);
  if (rc != DBBC_OK) return rc;
  rc = ensure_plan(g, p, st);
  if (rc != DBBC_OK) return rc;
  const bool timed = opt && (opt->flags & DBBC_OPT_TIME_KERNELS);
  g->timed_valid = false;
  Timing tm{timed ? &g->timers : nullptr, 0, st};
  const LaunchSet L = lone_launches(g, long_len);
  rc = enqueue(L, st, tm);
  g->timers_used = tm.used;
  if (rc != DBBC_OK) return rc;
  HIP_TRY(hipMemcpyAsync(g->pinned, g->ctl.p, kCtlWords * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, st));
  return DBBC_OK;
}

int finish_lone(dbbc_graph* g, dbbc_counts* out_host, bool timed) {
  if (g->pinned[kCtlErr] != 0)
    return fail(DBBC_E_DEVICE, "a kernel reported an internal error (bits: 1 hash table full, 2 LDS layout; got " +
                                   std::to_string(g->pinned[kCtlErr]) + ")");
  if (timed) {
    for (size_t i = 0; i < g->timers_used; ++i) {
      KernelRec& t = g->timers[i];
      HIP_TRY(hipEventElapsedTime(&t.ms, t.ev[0], t.ev[1]));
    }
    g->timed_valid = true;
  }
  read_counts(g, g->pinned, out_host);
  return DBBC_OK;
}

}  // namespace

extern "C" {

const char* dbbc_version(void) { return "0.2.0"; }

const char* dbbc_last_error(void) { return g_last_error.c_str(); }

const char* dbbc_status_string(int status) {
  switch (status) {
    case DBBC_OK: return "ok";
    case DBBC_E_INVALID_ARG: return "invalid argument";
    case DBBC_E_ID_RANGE: return "vertex id out of range";
    case DBBC_E_SIGN: return "sign not +1 or -1";
    case DBBC_E_DUPLICATE: return "duplicate edge";
    case DBBC_E_OOM: return "out of memory";
    case DBBC_E_DEVICE: return "device error";
    case DBBC_E_TOO_LARGE: return "graph too large";
    case DBBC_E_NO_DEVICE: return "no gfx950 device";
    case DBBC_E_PARSE: return "malformed edge record";
    default: return "unknown status";
  }
}

int dbbc_graph_create(int32_t n_u, int32_t n_v, int64_t m, const int32_t* u, const int32_t* v,
                      const int8_t* sign, uint32_t flags, const dbbc_allocator* alloc, void* hip_stream,
                      dbbc_graph** out) {
  g_last_error.clear();
  if (!out) return fail(DBBC_E_INVALID_ARG, "out must not be NULL");
  if (flags & ~(DBBC_INPUT_DEVICE | DBBC_DUP_REJECT)) return fail(DBBC_E_INVALID_ARG, "unknown flag");
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(DBBC_E_INVALID_ARG, "an allocator needs both its alloc and its free function");
  // argument checks that need no device (the records themselves are checked
  // by the device build)
  if (n_u <= 0 || n_v <= 0 || m < 0) return fail(DBBC_E_INVALID_ARG, "n_u and n_v must be positive and m non-negative");
  if (static_cast<int64_t>(n_u) + n_v >= (int64_t(1) << 30) || m >= (int64_t(1) << 31) - 1)
    return fail(DBBC_E_TOO_LARGE, "graph too large: need n_u + n_v < 2^30 and m < 2^31 - 1");
  if (m > 0 && (!u || !v || !sign)) return fail(DBBC_E_INVALID_ARG, "edge arrays must not be NULL");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  DeviceInfo di;
  int rc = current_device(di);
  if (rc != DBBC_OK) return rc;
  std::unique_ptr<dbbc_graph> g(new (std::nothrow) dbbc_graph());
  if (!g) return fail(DBBC_E_OOM, "host allocation failed");
  g->dev = di;
  if (alloc) g->al.a = *alloc;
  g->al.stream = hip_stream;
  dbbc::AllocScope scope(g->al, hip_stream);
  std::string err;
  dbbc::DeviceCsr csr;
  rc = dbbc::build_device_graph(n_u, n_v, m, u, v, sign, flags, st, g->host, csr, err);
  if (rc != DBBC_OK) return fail(rc, err);
  take_csr(g.get(), csr);
  HIP_TRY(g->ctl.alloc(kCtlWords * sizeof(unsigned long long)));
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&g->pinned), kCtlWords * sizeof(unsigned long long),
                        hipHostMallocDefault));
  HIP_TRY(hipStreamSynchronize(st));
  *out = g.release();
  return DBBC_OK;
}

int dbbc_graph_create_text(const char* text, int64_t len, uint32_t flags, const dbbc_allocator* alloc,
                           void* hip_stream, dbbc_graph** out, dbbc_text_info* info) {
  g_last_error.clear();
  if (!out) return fail(DBBC_E_INVALID_ARG, "out must not be NULL");
  if (flags & ~(DBBC_INPUT_DEVICE | DBBC_DUP_REJECT)) return fail(DBBC_E_INVALID_ARG, "unknown flag");
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(DBBC_E_INVALID_ARG, "an allocator needs both its alloc and its free function");
  if (len < 0 || (len > 0 && !text)) return fail(DBBC_E_INVALID_ARG, "text must not be NULL and len non-negative");
  if (len >= (int64_t(1) << 31) - 1) return fail(DBBC_E_TOO_LARGE, "text longer than 2^31 - 2 bytes");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  DeviceInfo di;
  int rc = current_device(di);
  if (rc != DBBC_OK) return rc;
  std::unique_ptr<dbbc_graph> g(new (std::nothrow) dbbc_graph());
  if (!g) return fail(DBBC_E_OOM, "host allocation failed");
  g->dev = di;
  if (alloc) g->al.a = *alloc;
  g->al.stream = hip_stream;
  dbbc::AllocScope scope(g->al, hip_stream);
  std::string err;
  dbbc::DeviceCsr csr;
  dbbc::IngestOut io;
  rc = dbbc::ingest_text(text, len, flags, st, g->host, csr, io, err);
  if (rc != DBBC_OK) return fail(rc, err);
  take_csr(g.get(), csr);
  for (int s = 0; s < 2; ++s) g->raw_ids[s] = std::move(io.raw[s]);
  HIP_TRY(g->ctl.alloc(kCtlWords * sizeof(unsigned long long)));
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&g->pinned), kCtlWords * sizeof(unsigned long long),
                        hipHostMallocDefault));
  HIP_TRY(hipStreamSynchronize(st));
  if (info) *info = dbbc_text_info{io.lines, io.records, g->host.n_u, g->host.n_v};
  *out = g.release();
  return DBBC_OK;
}

int dbbc_graph_raw_ids(const dbbc_graph* g, int32_t side, int64_t* out, void* hip_stream) {
  g_last_error.clear();
  if (!g || !out || side < 0 || side > 1) return fail(DBBC_E_INVALID_ARG, "NULL argument or side not 0 / 1");
  if (!g->raw_ids[side].p) return fail(DBBC_E_INVALID_ARG, "the graph was not read from text");
  const size_t n = static_cast<size_t>(side == 0 ? g->host.n_u : g->host.n_v);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  HIP_TRY(hipMemcpyAsync(out, g->raw_ids[side].p, n * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return DBBC_OK;
}

int dbbc_graph_stats(const dbbc_graph* g, dbbc_stats* out) {
  if (!g || !out) return fail(DBBC_E_INVALID_ARG, "NULL argument");
  dbbc_stats s{};
  s.n_u = g->host.n_u;
  s.n_v = g->host.n_v;
  s.m = g->host.m;
  s.dups_dropped = g->host.dups_dropped;
  s.max_deg_u = g->host.side[0].max_deg;
  s.max_deg_v = g->host.side[1].max_deg;
  size_t b = g->ctl.bytes + g->plan.bytes() + g->pv_plan.bytes() + g->edge_rec.bytes +
             g->edge_pos_v.bytes + g->pe_tmp.bytes;
  for (int k = 0; k < 2; ++k) {
    b += g->adj[k].bytes + g->off[k].bytes + g->orig[k].bytes + g->raw_ids[k].bytes + g->rev[k].bytes +
         g->cut[k].bytes + g->grank[k].bytes;
    for (int j = 0; j < 2; ++j) b += g->pv_out[k][j].bytes;
    b += g->pv_keys[k].bytes;
    for (int j = 0; j < 3; ++j) b += g->pe_out[k][j].bytes;
  }
  s.device_bytes = static_cast<int64_t>(b);
  s.wedges_vp = g->host.wedges_vp;
  s.pivots_active = g->host.pivots_active;
  *out = s;
  return DBBC_OK;
}

int dbbc_count(dbbc_graph* g, const dbbc_options* opt, dbbc_counts* out_host, void* hip_stream) {
  g_last_error.clear();
  if (!out_host) return fail(DBBC_E_INVALID_ARG, "NULL argument");
  int rc = check_graph(g);
  if (rc != DBBC_OK) return rc;
  dbbc::AllocScope scope(g->al, hip_stream);

  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  rc = enqueue_lone(g, opt, st);
  if (rc != DBBC_OK) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  return finish_lone(g, out_host, opt && (opt->flags & DBBC_OPT_TIME_KERNELS));
}

int dbbc_count_explicit(dbbc_graph* g, dbbc_counts* out_host, void* hip_stream) {
  g_last_error.clear();
  if (!out_host) return fail(DBBC_E_INVALID_ARG, "NULL argument");
  int rc = check_graph(g);
  if (rc != DBBC_OK) return rc;
  dbbc::AllocScope scope(g->al, hip_stream);

  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  rc = ensure_host(g, st);
  if (rc != DBBC_OK) return rc;
  const dbbc::HostGraph& hg = g->host;
  // the most wedges of one pivot (the list a workgroup holds at once)
  int64_t cap = 1;
  for (int s = 0; s < 2; ++s) {
    const dbbc::HostSide& S = hg.side[s];
    const dbbc::HostSide& O = hg.side[1 - s];
    for (int32_t x = 0; x < S.n; ++x) {
      int64_t wx = 0;
      for (uint32_t e = S.off[x] + static_cast<uint32_t>(S.cut[x]); e < S.off[x + 1]; ++e) {
        const uint32_t y = S.adj[e] >> 1;
        wx += static_cast<int64_t>(O.off[y + 1] - O.off[y]) - 1 - S.rev[e];
      }
      cap = std::max(cap, wx);
    }
  }
  const int64_t nmax = std::max<int64_t>(hg.n_u, hg.n_v);
  const int64_t per_wg = 16 * nmax + cap;
  const int64_t budget = int64_t(8) << 30;  // scratch of all workgroups
  const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(2 * g->dev.cus, budget / per_wg)));
  DevBuf scratch, lists;
  HIP_TRY(scratch.alloc(static_cast<size_t>(grid) * 16 * static_cast<size_t>(nmax)));
  HIP_TRY(lists.alloc(static_cast<size_t>(grid) * static_cast<size_t>(cap)));
  unsigned long long* ctl = g->ctl.as<unsigned long long>();
  HIP_TRY(dbbc::launch_fill_u64(ctl, kCtlWords, 0ull, st));
  uint32_t* queues = reinterpret_cast<uint32_t*>(ctl + kCtlQueues);
  for (int s = 0; s < 2; ++s) {
    // counters start at zero (the layout differs per side: clear it all)
    HIP_TRY(dbbc::launch_fill_u64(scratch.as<unsigned long long>(), static_cast<size_t>(grid) * 2 * nmax, 0ull, st));
    dbbc::ExplicitArgs a{};
    a.off_s = g->off[s].as<uint32_t>();
    a.adj_s = g->adj[s].as<uint32_t>();
    a.rev_s = g->rev[s].as<int32_t>();
    a.cut_s = g->cut[s].as<int32_t>();
    a.off_o = g->off[1 - s].as<uint32_t>();
    a.adj_o = g->adj[1 - s].as<uint32_t>();
    a.n_s = hg.side[s].n;
    a.scratch = scratch.as<uint32_t>();
    a.lists = lists.as<uint8_t>();
    a.list_cap = cap;
    a.queue = queues + s;
    a.res = ctl;
    a.err = ctl + kCtlErr;
    HIP_TRY(dbbc::launch_explicit(a, std::min<int>(grid, std::max(1, a.n_s)), st));
  }
  HIP_TRY(hipMemcpyAsync(g->pinned, g->ctl.p, kCtlWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (g->pinned[kCtlErr]) return fail(DBBC_E_DEVICE, "explicit count: a pivot's wedges exceeded its list");
  out_host->balanced = static_cast<int64_t>(g->pinned[dbbc::kResBalanced]);
  out_host->unbalanced = static_cast<int64_t>(g->pinned[dbbc::kResUnbalanced]);
  out_host->total = static_cast<int64_t>(g->pinned[dbbc::kResTotal]);
  out_host->wedges = hg.wedges_vp;
  return DBBC_OK;
}

int dbbc_graph_plan(dbbc_graph* g, const dbbc_options* opt, void* hip_stream) {
  g_last_error.clear();
  int rc = check_graph(g);
  if (rc != DBBC_OK) return rc;
  dbbc::AllocScope scope(g->al, hip_stream);

  dbbc::PlanParams p;
  uint32_t long_len = 0;
  rc = params_from(g, opt, p, long_len);
  if (rc != DBBC_OK) return rc;
  return ensure_plan(g, p, static_cast<hipStream_t>(hip_stream));
}

int dbbc_count_async(dbbc_graph* g, const dbbc_options* opt, void* hip_stream) {
  g_last_error.clear();
  int rc = check_graph(g);
  if (rc != DBBC_OK) return rc;
  dbbc::AllocScope scope(g->al, hip_stream);

  if (opt && (opt->flags & DBBC_OPT_TIME_KERNELS))
    return fail(DBBC_E_INVALID_ARG, "kernel timing needs dbbc_count");
  rc = enqueue_lone(g, opt, static_cast<hipStream_t>(hip_stream));
  if (rc != DBBC_OK) return rc;
  g->in_flight = true;
  return DBBC_OK;
}

int dbbc_count_read(dbbc_graph* g, dbbc_counts* out_host) {
  g_last_error.clear();
  if (!g || !out_host) return fail(DBBC_E_INVALID_ARG, "NULL argument");
  if (!g->in_flight) return fail(DBBC_E_INVALID_ARG, "no asynchronous count on this graph");
  g->in_flight = false;
  return finish_lone(g, out_host, false);
}

}  // extern "C"

namespace {

// Direct items' keys lie below the window, at most 32,768 ranks (the widest
// window_L), so the rank-indexed key sums cover them.
static_assert(dbbc::kPVKeyRanks >= dbbc::kPVWindowPacked && dbbc::kPVWindowPacked == 32768,
              "key sums cover the widest window");

// The per-vertex pass, with per-edge credits when edge is set: tally and
// credit walks over every item of the per-vertex plan, then (per-edge) the
// combination of the two CSRs' credits into input-record order.
int local_counts(dbbc_graph* g, const dbbc_options* opt, int64_t* const vout[2][2], bool edge,
                 int64_t* bal_e, int64_t* unb_e, dbbc_counts* out_host, hipStream_t st) {
  int rc = check_graph(g);
  if (rc != DBBC_OK) return rc;
  dbbc::AllocScope scope(g->al, st);

  if (opt && (opt->flags & DBBC_OPT_TIME_KERNELS))
    return fail(DBBC_E_INVALID_ARG, "kernel timing needs dbbc_count");
  dbbc::PlanParams p;
  uint32_t long_len = 0;
  rc = params_from(g, opt, p, long_len);
  if (rc != DBBC_OK) return rc;
  p.per_vertex = true;
  p.hub_T = std::min(p.hub_T, dbbc::kMaxPVHubT);
  p.wide_all = edge && opt && (opt->flags & DBBC_OPT_WIDE_EDGES);
  const int32_t n[2] = {g->host.n_u, g->host.n_v};
  const size_t m = static_cast<size_t>(g->host.m);
  for (int s = 0; s < 2; ++s) {
    for (int k = 0; k < 2; ++k)
      HIP_TRY(g->pv_out[s][k].reserve(static_cast<size_t>(n[s]) * sizeof(unsigned long long)));
    HIP_TRY(g->pv_keys[s].reserve(2 * static_cast<size_t>(dbbc::kPVKeyRanks) * sizeof(unsigned long long)));
  }
  if (edge) {
    for (int s = 0; s < 2; ++s)
      for (int k = 0; k < 3; ++k) HIP_TRY(g->pe_out[s][k].reserve(m * sizeof(unsigned long long)));
    if (!g->edge_pos_v.p && m > 0) {  // U-CSR position -> V-CSR position of every edge
      HIP_TRY(g->edge_pos_v.alloc(m * sizeof(uint32_t)));
      std::string err;
      rc = dbbc::edge_positions_device(view_of(g), g->edge_pos_v.as<uint32_t>(), st, err);
      if (rc != DBBC_OK) return fail(rc, err);
    }
  }
  rc = ensure_plan_into(g, p, st, g->pv_plan);
  if (rc != DBBC_OK) return rc;
  DevPlan& d = g->pv_plan;
  const dbbc::HostPlan& hp = d.host;
  // the per-edge buffers may have been allocated after the plan's side table
  if (edge && d.side[0].epack != g->pe_out[0][0].as<unsigned long long>()) {
    for (int s = 0; s < 2; ++s) {
      d.side[s].epack = g->pe_out[s][0].as<unsigned long long>();
      d.side[s].ewb = g->pe_out[s][1].as<unsigned long long>();
      d.side[s].ewu = g->pe_out[s][2].as<unsigned long long>();
      d.side[s].epack_o = g->pe_out[1 - s][0].as<unsigned long long>();
      d.side[s].ewb_o = g->pe_out[1 - s][1].as<unsigned long long>();
      d.side[s].ewu_o = g->pe_out[1 - s][2].as<unsigned long long>();
    }
    HIP_TRY(hipMemcpyAsync(d.sides.p, d.side, sizeof(d.side), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  unsigned long long* ctl = g->ctl.as<unsigned long long>();
  HIP_TRY(dbbc::launch_fill_u64(ctl, kCtlWords, 0ull, st));
  for (int s = 0; s < 2; ++s) {
    for (int k = 0; k < 2; ++k)
      HIP_TRY(dbbc::launch_fill_u64(g->pv_out[s][k].as<unsigned long long>(), static_cast<size_t>(n[s]), 0ull, st));
    for (int k = 0; k < 3 && edge; ++k)
      HIP_TRY(dbbc::launch_fill_u64(g->pe_out[s][k].as<unsigned long long>(), m, 0ull, st));
  }
  unsigned long long* err = ctl + kCtlErr;
  uint32_t* queues = reinterpret_cast<uint32_t*>(ctl + kCtlQueues);
  const dbbc::DevSideConst* sides = d.sides.as<dbbc::DevSideConst>();
  const int cus = g->dev.cus;
  if (hp.T[0] > 0) {
    // The dense block (hubpv.hip): the hub pairs' sparse counts, completed
    // and credited by the block's products, then the credits of the block's
    // wedges; the sparse kernels below read the completed counts.
    dbbc::HubTallyArgs ta[2];
    for (int s = 0; s < 2; ++s) {
      HIP_TRY(dbbc::launch_fill_u64(d.hub_pairs[s].as<unsigned long long>(),
                                    static_cast<size_t>(hp.T[s]) * hp.T[s], 0ull, st));
      const int32_t lo = s == 0 ? 0 : hp.n_hub_side0;
      const int32_t hi = s == 0 ? hp.n_hub_side0 : static_cast<int32_t>(d.hub_items.bytes / sizeof(dbbc::Item));
      ta[s] = dbbc::HubTallyArgs{};
      ta[s].items = d.hub_items.as<dbbc::Item>() + lo;
      ta[s].segs = d.hub_segs.as<dbbc::Segment>();
      ta[s].other_adj = g->adj[1 - s].as<uint32_t>();
      ta[s].hub_xy = d.hub_pairs[s].as<int32_t>();
      ta[s].n_items = hi - lo;
      ta[s].T = hp.T[s];
      ta[s].long_len = long_len;
    }
    HIP_TRY(dbbc::launch_pv_hub_tally(ta, 2, 4 * cus, st));
    dbbc::HubArgs ha[2];
    for (int s = 0; s < 2; ++s) {
      ha[s] = dbbc::HubArgs{};
      ha[s].Bm = d.hub_Bm[s].as<int8_t>();
      ha[s].B = d.hub_B[s].as<int8_t>();
      ha[s].hub_xy = d.hub_pairs[s].as<int32_t>();
      ha[s].res = ctl;
      ha[s].T = hp.T[s];
      ha[s].K = d.hub_K[s];
      ha[s].orig = g->orig[s].as<int32_t>();
      ha[s].bal = g->pv_out[s][0].as<unsigned long long>();
      ha[s].unb = g->pv_out[s][1].as<unsigned long long>();
    }
    HIP_TRY(dbbc::launch_hub(ha, 2, st));
    for (int s = 0; s < 2; ++s) {
      dbbc::HubDigitArgs da{};
      da.hub_xy = d.hub_pairs[s].as<int32_t>();
      da.rows = d.hub_rows[s].as<int8_t>();
      da.cols = d.hub_cols[s].as<int8_t>();
      da.T = hp.T[s];
      da.D = d.hub_D[s];
      HIP_TRY(dbbc::launch_hub_digits(da, st));
      for (int role = 0; role < (edge ? 2 : 1); ++role) {
        dbbc::HubCreditArgs ca{};
        const bool pm = role == 0;  // pivot-mid edges and mids; else end-mid edges
        ca.A = pm ? d.hub_rows[s].as<int8_t>() : d.hub_cols[s].as<int8_t>();
        ca.Bt = pm ? d.hub_Bt[s].as<int8_t>() : d.hub_Bmt[s].as<int8_t>();
        ca.E = pm ? d.hub_Bm[s].as<int8_t>() : d.hub_B[s].as<int8_t>();
        ca.Zc = pm ? d.hub_Zc[s].as<int32_t>() : d.hub_Zcp[s].as<int32_t>();
        ca.pos = edge ? d.hub_pos[s].as<int32_t>() : nullptr;
        ca.orig_mid = pm ? g->orig[1 - s].as<int32_t>() : nullptr;
        ca.bal_mid = g->pv_out[1 - s][0].as<unsigned long long>();
        ca.unb_mid = g->pv_out[1 - s][1].as<unsigned long long>();
        ca.ewb = g->pe_out[s][1].as<unsigned long long>();
        ca.ewu = g->pe_out[s][2].as<unsigned long long>();
        ca.epack = g->pe_out[s][0].as<unsigned long long>();
        ca.off = g->off[s].as<uint32_t>();
        ca.n = s ? g->host.n_v : g->host.n_u;
        ca.max_deg_other = static_cast<unsigned long long>(g->host.side[1 - s].max_deg);
        ca.wide_all = hp.p.wide_all ? 1 : 0;
        ca.T = hp.T[s];
        ca.K = d.hub_K[s];
        ca.D = d.hub_D[s];
        ca.upper = pm ? 1 : 0;
        HIP_TRY(dbbc::launch_hub_credit(ca, st));
      }
    }
  }
  // direct items: one launch per side; their key credits are summed by rank
  // and added to the outputs after both launches
  for (int s = 0; s < 2; ++s)
    HIP_TRY(dbbc::launch_fill_u64(g->pv_keys[s].as<unsigned long long>(), 2 * static_cast<size_t>(dbbc::kPVKeyRanks),
                                  0ull, st));
  for (int s = 0; s < 2; ++s) {
    const int32_t lo = s == 0 ? 0 : hp.n_direct_side0;
    const int32_t hi = s == 0 ? hp.n_direct_side0 : hp.n_items_kept[0];
    dbbc::DirectArgs a{};
    a.items = d.direct_items.as<dbbc::Item>() + lo;
    a.sides = sides;
    a.queue = queues + s;
    a.res = ctl;
    a.err = err;
    a.n_items = hi - lo;
    a.long_len = long_len;
    const int grid = std::min<int>(cus, std::max(1, a.n_items));
    HIP_TRY(edge ? dbbc::launch_pe_direct(a, grid, st) : dbbc::launch_pv_direct(a, grid, st));
  }
  for (int s = 0; s < 2; ++s) HIP_TRY(dbbc::launch_pv_key_flush(sides, s, hp.L[s], st));
  // reverse items: one launch per side (their key credits are summed per
  // workgroup for one side's reverse window)
  for (int s = 0; s < 2; ++s) {
    const int32_t lo = s == 0 ? 0 : hp.n_reverse_side0;
    const int32_t hi = s == 0 ? hp.n_reverse_side0 : hp.n_items_kept[1];
    dbbc::SmallArgs a{};
    a.items = d.reverse_items.as<dbbc::Item>() + lo;
    a.sides = sides;
    a.res = ctl;
    a.err = err;
    a.n_items = hi - lo;
    a.long_len = long_len;
    const int grid = std::min<int>(cus, std::max(1, (a.n_items + 7) / 8));
    HIP_TRY(edge ? dbbc::launch_pe_reverse(a, grid, st) : dbbc::launch_pv_reverse(a, grid, st));
  }
  {
    dbbc::SmallArgs a{};
    a.items = d.small_groups.as<dbbc::Item>();
    a.sides = sides;
    a.res = ctl;
    a.err = err;
    a.n_items = hp.n_items_kept[2];
    a.long_len = long_len;
    const int grid = std::min<int>(3 * cus, std::max(1, (a.n_items + 3) / 4));
    HIP_TRY(edge ? dbbc::launch_pe_small(a, grid, st) : dbbc::launch_pv_small(a, grid, st));
  }
  {
    dbbc::HashArgs a{};
    a.items = d.hash_items.as<dbbc::Item>();
    a.sides = sides;
    a.queue = queues + 2;
    a.res = ctl;
    a.err = err;
    a.n_items = hp.n_items_kept[3];
    a.long_len = long_len;
    const int grid = std::min<int>(cus, std::max(1, a.n_items));
    HIP_TRY(edge ? dbbc::launch_pe_hash(a, grid, st) : dbbc::launch_pv_hash(a, grid, st));
  }
  if (edge) {
    const size_t m_in = static_cast<size_t>(g->host.m_in);
    // duplicate records (dropped from the graph) read 0
    const bool dups = g->host.m_in > g->host.m;
    dbbc::EdgeCombineArgs a{};
    for (int s = 0; s < 2; ++s) {
      a.e_pack[s] = g->pe_out[s][0].as<unsigned long long>();
      a.e_wb[s] = g->pe_out[s][1].as<unsigned long long>();
      a.e_wu[s] = g->pe_out[s][2].as<unsigned long long>();
    }
    a.rec = g->edge_rec.as<uint32_t>();
    a.pos_v = g->edge_pos_v.as<uint32_t>();
    a.m = g->host.m;
    // runs flagged wide, or the dense block's credits (kept in the two-word form)
    a.wide = d.any_wide || hp.T[0] > 0 || hp.T[1] > 0 ? 1 : 0;
    a.off_u = g->off[0].as<uint32_t>();
    a.off_v = g->off[1].as<uint32_t>();
    a.adj_u = g->adj[0].as<uint32_t>();
    a.n_u = g->host.n_u;
    a.n_v = g->host.n_v;
    a.max_deg_u = static_cast<unsigned long long>(g->host.side[0].max_deg);
    a.max_deg_v = static_cast<unsigned long long>(g->host.side[1].max_deg);
    a.wide_all = hp.p.wide_all ? 1 : 0;
    // the combine kernel writes both outputs: a NULL one goes to a buffer of
    // the graph's
    DevBuf& tmp = g->pe_tmp;
    if (!bal_e || !unb_e) HIP_TRY(tmp.reserve(m_in * sizeof(long long)));
    a.out_bal = reinterpret_cast<long long*>(bal_e ? bal_e : tmp.as<int64_t>());
    a.out_unb = reinterpret_cast<long long*>(unb_e ? unb_e : tmp.as<int64_t>());
    if (dups) {
      if (bal_e) HIP_TRY(dbbc::launch_fill_u64(reinterpret_cast<unsigned long long*>(bal_e), m_in, 0ull, st));
      if (unb_e) HIP_TRY(dbbc::launch_fill_u64(reinterpret_cast<unsigned long long*>(unb_e), m_in, 0ull, st));
    }
    const int grid = static_cast<int>(std::min<int64_t>(8 * cus, std::max<int64_t>(1, (a.m + 255) / 256)));
    HIP_TRY(dbbc::launch_edge_combine(a, grid, st));
  }
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < 2; ++k)
      if (vout[s][k])
        HIP_TRY(hipMemcpyAsync(vout[s][k], g->pv_out[s][k].p, static_cast<size_t>(n[s]) * sizeof(int64_t),
                               hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(g->pinned, g->ctl.p, kCtlWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  dbbc_counts c{};
  rc = finish_lone(g, &c, false);
  if (rc != DBBC_OK) return rc;
  if (out_host) *out_host = c;
  return DBBC_OK;
}

// ---- the count without allocation --------------------------------------------
//
// dbbc_count_noalloc runs the kernels of dbbc_count on a graph already
// planned for its options, with every buffer the kernels write -- the
// control block (result slot, error bits, work-queue heads), the side table,
// the multi-part accumulators and the dense block's hub-pair partials -- in
// one file-scope device array instead of the plan's buffers.  Each GPU the
// library runs on holds its own copy of the array until the process ends;
// calls on one GPU share it, so calls that overlap on one GPU race.

constexpr size_t kNoAllocScratchBytes = DBBC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// The array's device address on each device, looked up once per device with
// that device current (the host-side name is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(DBBC_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DBBC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return DBBC_OK;
}

constexpr size_t round256(size_t n) { return (n + 255) / 256 * 256; }

}  // namespace

extern "C" {

int dbbc_count_noalloc(dbbc_graph* g, const dbbc_options* opt, dbbc_counts* out_host, void* hip_stream) {
  g_last_error.clear();
  if (!out_host) return fail(DBBC_E_INVALID_ARG, "NULL argument");
  int rc = check_graph(g);
  if (rc != DBBC_OK) return rc;
  if (opt && (opt->flags & DBBC_OPT_TIME_KERNELS))
    return fail(DBBC_E_INVALID_ARG, "kernel timing needs dbbc_count");
  dbbc::PlanParams p;
  uint32_t long_len = 0;
  rc = params_from(g, opt, p, long_len);
  if (rc != DBBC_OK) return rc;
  DevPlan& d = g->plan;
  if (!d.valid || !(d.host.p == p))
    return fail(DBBC_E_INVALID_ARG,
                "the graph has no plan for these options: plan it first (dbbc_graph_plan or dbbc_count)");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != g->dev.id) return fail(DBBC_E_INVALID_ARG, "the graph lives on another device than the current one");
  const dbbc::HostPlan& hp = d.host;
  // scratch layout: control block, side table, accumulators, hub-pair planes
  const size_t off_sides = round256(kCtlWords * sizeof(unsigned long long));
  const size_t off_acc = off_sides + round256(sizeof(d.side));
  const size_t acc_bytes = static_cast<size_t>(hp.acc_slots) * static_cast<size_t>(hp.acc_width) * sizeof(uint32_t);
  size_t off_hub[2], end = off_acc + round256(acc_bytes);
  for (int s = 0; s < 2; ++s) {
    off_hub[s] = end;
    end += round256(2 * static_cast<size_t>(hp.T[s]) * static_cast<size_t>(hp.T[s]) * sizeof(int32_t));
  }
  if (end > kNoAllocScratchBytes)
    return fail(DBBC_E_TOO_LARGE, "the count needs " + std::to_string(end) + " bytes of scratch, more than the " +
                                      std::to_string(kNoAllocScratchBytes) +
                                      " of dbbc_count_noalloc (a smaller hub_T or window_L needs less)");
  unsigned char* base = nullptr;
  rc = scratch_address(dev, &base);
  if (rc != DBBC_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int32_t* hub_xy[2] = {reinterpret_cast<int32_t*>(base + off_hub[0]), reinterpret_cast<int32_t*>(base + off_hub[1])};
  dbbc::DevSideConst side[2] = {d.side[0], d.side[1]};
  for (int s = 0; s < 2; ++s) {
    side[s].acc = reinterpret_cast<uint32_t*>(base + off_acc);
    side[s].hub_xy = hp.T[s] ? hub_xy[s] : nullptr;
  }
  auto* sides = reinterpret_cast<dbbc::DevSideConst*>(base + off_sides);
  HIP_TRY(dbbc::launch_store_sides(side, sides, st));
  LaunchSet L;
  L.direct = d.direct_items.as<dbbc::Item>();
  L.reverse = d.reverse_items.as<dbbc::Item>();
  L.small = d.small_groups.as<dbbc::Item>();
  L.hash = d.hash_items.as<dbbc::Item>();
  L.reduces = d.reduces.as<dbbc::Reduce>();
  for (int k = 0; k < 5; ++k) L.n[k] = hp.n_items_kept[k];
  L.sides = sides;
  L.ctl = reinterpret_cast<unsigned long long*>(base);
  L.res = L.ctl;
  L.n_res = dbbc::kResStride;
  add_hub_launches(d, L.res, L, hub_xy);
  L.long_len = long_len;
  L.cus = g->dev.cus;
  Timing tm{nullptr, 0, st};
  rc = enqueue(L, st, tm);
  if (rc != DBBC_OK) return rc;
  HIP_TRY(hipMemcpyAsync(g->pinned, L.ctl, kCtlWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return finish_lone(g, out_host, false);
}

int dbbc_count_per_vertex(dbbc_graph* g, const dbbc_options* opt, int64_t* bal_u, int64_t* bal_v,
                          int64_t* unb_u, int64_t* unb_v, dbbc_counts* out_host, void* hip_stream) {
  g_last_error.clear();
  int64_t* const outs[2][2] = {{bal_u, unb_u}, {bal_v, unb_v}};
  return local_counts(g, opt, outs, false, nullptr, nullptr, out_host, static_cast<hipStream_t>(hip_stream));
}

int dbbc_count_per_edge(dbbc_graph* g, const dbbc_options* opt, int64_t* bal_e, int64_t* unb_e,
                        dbbc_counts* out_host, void* hip_stream) {
  g_last_error.clear();
  int64_t* const outs[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  return local_counts(g, opt, outs, true, bal_e, unb_e, out_host, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

namespace {

// (Re)target batch b at the graphs gs[0..k): plan them, assemble their work
// lists on the device into b's buffers (grown only when too small) and, with
// DBBC_BATCH_CAPTURE, capture the launch sequence into a HIP graph.
int assemble_batch(dbbc_batch* b, dbbc_graph* const* gs, int32_t k, const dbbc_options* opt,
                   uint32_t flags, hipStream_t st) {
  if (k < 0 || (k > 0 && !gs)) return fail(DBBC_E_INVALID_ARG, "bad batch arguments");
  if (flags & ~DBBC_BATCH_CAPTURE) return fail(DBBC_E_INVALID_ARG, "unknown batch flag");
  if (opt && (opt->flags & DBBC_OPT_TIME_KERNELS))
    return fail(DBBC_E_INVALID_ARG, "kernel timing needs dbbc_count");
  std::unordered_set<const dbbc_graph*> seen;
  for (int32_t i = 0; i < k; ++i) {
    int rc = check_graph(gs[i]);
    if (rc != DBBC_OK) return rc;
    if (!seen.insert(gs[i]).second) return fail(DBBC_E_INVALID_ARG, "a graph appears twice in the batch");
  }
  b->drop_graph();
  b->gs.clear();
  b->gens.clear();
  b->L = LaunchSet{};
  int rc;
  uint32_t long_len = kDefaultLongLen;
  int64_t tot[5] = {0, 0, 0, 0, 0};
  LaunchSet& L = b->L;
  for (int32_t i = 0; i < k; ++i) {
    dbbc::PlanParams p;
    rc = params_from(gs[i], opt, p, long_len);
    if (rc != DBBC_OK) return rc;
    {
      dbbc::AllocScope plan_scope(gs[i]->al, st);  // a graph's plan comes from its own allocator
      rc = ensure_plan(gs[i], p, st);
    }
    if (rc != DBBC_OK) return rc;
    const dbbc::HostPlan& hp = gs[i]->plan.host;
    for (int j = 0; j < 5; ++j) tot[j] += hp.n_items_kept[j];
    for (int j = 0; j < 4; ++j) {
      L.wedges[j] += hp.k_wedges[j];
      L.segs[j] += hp.k_segs[j];
    }
  }
  for (int j = 0; j < 5; ++j)
    if (tot[j] > INT32_MAX) return fail(DBBC_E_TOO_LARGE, "too many work items in one batch");
  dbbc::AllocScope scope(b->al, st);  // the batch's own buffers
  HIP_TRY(b->res.reserve(static_cast<size_t>(std::max(k, 1)) * dbbc::kResStride * sizeof(unsigned long long)));
  HIP_TRY(b->ctl.reserve(kCtlWords * sizeof(unsigned long long)));
  const size_t words = static_cast<size_t>(k) * dbbc::kResStride + 1;
  if (words > b->pinned_words) {
    if (b->pinned) HIP_TRY(hipHostFree(b->pinned));
    b->pinned = nullptr;
    b->pinned_words = 0;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&b->pinned), words * sizeof(unsigned long long),
                          hipHostMallocDefault));
    b->pinned_words = words;
  }
  b->gs.assign(gs, gs + k);
  for (int32_t i = 0; i < k; ++i) b->gens.push_back(gs[i]->plan_gen);
  if (k == 0) return DBBC_OK;
  // Assemble the k graphs' lists into one list per kernel, on the device.
  DevBuf* lists[5] = {&b->direct, &b->reverse, &b->small, &b->hash, &b->reduces};
  std::vector<dbbc::AssembleSrc> srcs(static_cast<size_t>(5) * k);
  for (int j = 0; j < 5; ++j) {
    const size_t esz = j == 4 ? sizeof(dbbc::Reduce) : sizeof(dbbc::Item);
    HIP_TRY(lists[j]->reserve(static_cast<size_t>(tot[j]) * esz));
    uint32_t off = 0;
    for (int32_t i = 0; i < k; ++i) {
      const DevPlan& d = gs[i]->plan;
      const DevBuf* src[5] = {&d.direct_items, &d.reverse_items, &d.small_groups, &d.hash_items, &d.reduces};
      dbbc::AssembleSrc& a = srcs[static_cast<size_t>(j) * k + i];
      a.src = src[j]->p;
      a.n = static_cast<uint32_t>(d.host.n_items_kept[j]);
      a.dst_off = off;
      a.graph = static_cast<uint32_t>(i);
      off += a.n;
    }
  }
  HIP_TRY(upload_reuse(b->srcs, srcs, st));
  const dbbc::AssembleSrc* dsrc = b->srcs.as<dbbc::AssembleSrc>();
  for (int j = 0; j < 4; ++j)
    if (tot[j]) HIP_TRY(dbbc::launch_assemble_items(dsrc + static_cast<size_t>(j) * k, k, lists[j]->as<dbbc::Item>(), st));
  if (tot[4]) HIP_TRY(dbbc::launch_assemble_reduces(dsrc + static_cast<size_t>(4) * k, k, b->reduces.as<dbbc::Reduce>(), st));
  std::vector<dbbc::DevSideConst> side(static_cast<size_t>(2) * k);
  for (int32_t i = 0; i < k; ++i) {
    side[2 * static_cast<size_t>(i)] = gs[i]->plan.side[0];
    side[2 * static_cast<size_t>(i) + 1] = gs[i]->plan.side[1];
  }
  HIP_TRY(upload_reuse(b->sides, side, st));
  HIP_TRY(hipStreamSynchronize(st));
  L.direct = b->direct.as<dbbc::Item>();
  L.reverse = b->reverse.as<dbbc::Item>();
  L.small = b->small.as<dbbc::Item>();
  L.hash = b->hash.as<dbbc::Item>();
  L.reduces = b->reduces.as<dbbc::Reduce>();
  for (int j = 0; j < 5; ++j) L.n[j] = static_cast<int32_t>(tot[j]);
  L.sides = b->sides.as<dbbc::DevSideConst>();
  L.ctl = b->ctl.as<unsigned long long>();
  L.res = b->res.as<unsigned long long>();
  L.n_res = static_cast<size_t>(k) * dbbc::kResStride;
  for (int32_t i = 0; i < k; ++i)
    add_hub_launches(gs[i]->plan, L.res + static_cast<size_t>(i) * dbbc::kResStride, L);
  L.long_len = long_len;
  L.cus = b->dev.cus;
  if (flags & DBBC_BATCH_CAPTURE) {
    if (!b->cap) HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    Timing tm{nullptr, 0, b->cap};
    rc = enqueue(L, b->cap, tm);
    const hipError_t e = hipStreamEndCapture(b->cap, &b->graph);
    if (rc != DBBC_OK) return rc;
    HIP_TRY(e);
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  return DBBC_OK;
}

}  // namespace

extern "C" {

int dbbc_batch_create(dbbc_graph* const* gs, int32_t k, const dbbc_options* opt, uint32_t flags,
                      void* hip_stream, dbbc_batch** out) {
  g_last_error.clear();
  if (!out) return fail(DBBC_E_INVALID_ARG, "bad batch arguments");
  if (k < 0 || (k > 0 && !gs) || (flags & ~DBBC_BATCH_CAPTURE))
    return assemble_batch(nullptr, gs, k, opt, flags, nullptr);  // reports the argument error
  for (int32_t i = 0; i < k; ++i) {
    const int rc = check_graph(gs[i]);
    if (rc != DBBC_OK) return rc;
  }
  std::unique_ptr<dbbc_batch> b(new (std::nothrow) dbbc_batch());
  if (!b) return fail(DBBC_E_OOM, "host allocation failed");
  int rc = current_device(b->dev);
  if (rc != DBBC_OK) return rc;
  if (k > 0) b->al = gs[0]->al;
  rc = assemble_batch(b.get(), gs, k, opt, flags, static_cast<hipStream_t>(hip_stream));
  if (rc != DBBC_OK) return rc;
  *out = b.release();
  return DBBC_OK;
}

int dbbc_batch_reset(dbbc_batch* b, dbbc_graph* const* gs, int32_t k, const dbbc_options* opt,
                     uint32_t flags, void* hip_stream) {
  g_last_error.clear();
  if (!b) return fail(DBBC_E_INVALID_ARG, "NULL batch");
  const int rc = assemble_batch(b, gs, k, opt, flags, static_cast<hipStream_t>(hip_stream));
  if (rc != DBBC_OK) {  // leave an empty batch behind
    b->drop_graph();
    b->gs.clear();
    b->gens.clear();
    b->L = LaunchSet{};
  }
  return rc;
}

int dbbc_batch_launch(dbbc_batch* b, void* hip_stream) {
  g_last_error.clear();
  if (!b) return fail(DBBC_E_INVALID_ARG, "NULL batch");
  const size_t k = b->gs.size();
  if (k == 0) return DBBC_OK;
  for (size_t i = 0; i < k; ++i)
    if (!b->gs[i]->plan.valid || b->gs[i]->plan_gen != b->gens[i])
      return fail(DBBC_E_INVALID_ARG, "a graph of the batch was planned again since the batch was made");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (b->exec) {
    HIP_TRY(hipGraphLaunch(b->exec, st));
  } else {
    Timing tm{nullptr, 0, st};
    int rc = enqueue(b->L, st, tm);
    if (rc != DBBC_OK) return rc;
  }
  HIP_TRY(hipMemcpyAsync(b->pinned, b->res.p, k * dbbc::kResStride * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(b->pinned + k * dbbc::kResStride, b->ctl.as<unsigned long long>() + kCtlErr,
                         sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  return DBBC_OK;
}

int dbbc_batch_read(const dbbc_batch* b, dbbc_counts* out_host) {
  g_last_error.clear();
  if (!b || (!out_host && !b->gs.empty())) return fail(DBBC_E_INVALID_ARG, "NULL argument");
  const size_t k = b->gs.size();
  if (k == 0) return DBBC_OK;
  if (b->pinned[k * dbbc::kResStride] != 0)
    return fail(DBBC_E_DEVICE, "a kernel reported an internal error (bits: 1 hash table full, 2 LDS layout; got " +
                                   std::to_string(b->pinned[k * dbbc::kResStride]) + ")");
  for (size_t i = 0; i < k; ++i) read_counts(b->gs[i], b->pinned + i * dbbc::kResStride, &out_host[i]);
  return DBBC_OK;
}

int dbbc_batch_count(dbbc_batch* b, dbbc_counts* out_host, void* hip_stream) {
  int rc = dbbc_batch_launch(b, hip_stream);
  if (rc != DBBC_OK) return rc;
  HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
  return dbbc_batch_read(b, out_host);
}

int32_t dbbc_batch_size(const dbbc_batch* b) { return b ? static_cast<int32_t>(b->gs.size()) : 0; }

void dbbc_batch_destroy(dbbc_batch* b) { delete b; }

int dbbc_count_batch(dbbc_graph* const* gs, int32_t k, const dbbc_options* opt, dbbc_counts* out_host,
                     void* hip_stream) {
  g_last_error.clear();
  if (k < 0 || (k > 0 && (!gs || !out_host))) return fail(DBBC_E_INVALID_ARG, "bad batch arguments");
  dbbc_batch* b = nullptr;
  int rc = dbbc_batch_create(gs, k, opt, 0u, hip_stream, &b);
  if (rc != DBBC_OK) return rc;
  rc = dbbc_batch_count(b, out_host, hip_stream);
  dbbc_batch_destroy(b);
  return rc;
}

int dbbc_autotune(dbbc_graph* const* gs, int32_t k, const dbbc_options* start, int32_t reps,
                  void* hip_stream, dbbc_options* best, float* best_ms) {
  g_last_error.clear();
  if (k <= 0 || !gs || !best || reps <= 0) return fail(DBBC_E_INVALID_ARG, "bad autotune arguments");
  if (start && (start->flags & DBBC_OPT_TIME_KERNELS))
    return fail(DBBC_E_INVALID_ARG, "kernel timing cannot be tuned");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  dbbc_options cur;
  if (start) {
    cur = *start;
  } else {
    cur = dbbc_options{-1, -1, -1, -1, -1, -1, 0u};
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  struct Ev {
    hipEvent_t* e;
    ~Ev() {
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } ev_guard{ev};
  // Time one option set: a captured batch, one warm-up replay, reps timed
  // replays.  Options the plan rejects time as +inf.
  auto time_opts = [&](const dbbc_options& o, float& ms) -> int {
    ms = INFINITY;
    dbbc_batch* b = nullptr;
    int rc = dbbc_batch_create(gs, k, &o, DBBC_BATCH_CAPTURE, hip_stream, &b);
    if (rc == DBBC_E_INVALID_ARG) return DBBC_OK;  // not a valid combination
    if (rc != DBBC_OK) return rc;
    std::unique_ptr<dbbc_batch, void (*)(dbbc_batch*)> guard(b, dbbc_batch_destroy);
    HIP_TRY(hipGraphLaunch(b->exec, st));
    HIP_TRY(hipEventRecord(ev[0], st));
    for (int32_t r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(b->exec, st));
    HIP_TRY(hipEventRecord(ev[1], st));
    HIP_TRY(hipEventSynchronize(ev[1]));
    HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
    ms /= static_cast<float>(reps);
    return DBBC_OK;
  };
  float cur_ms = 0.f;
  int rc = time_opts(cur, cur_ms);
  if (rc != DBBC_OK) return rc;
  if (!std::isfinite(cur_ms)) return fail(DBBC_E_INVALID_ARG, "the starting options are not valid");
  // Coordinate search: each knob in turn over its values, keeping the best.
  struct Knob {
    int32_t dbbc_options::*field;
    std::vector<int32_t> values;
  };
  const Knob knobs[] = {
      {&dbbc_options::long_len, {32, 64, 128, 256, 512}},
      {&dbbc_options::small_work, {64, 256, 512}},
      {&dbbc_options::window_L, {512, 2048, 8192, 32768}},
      {&dbbc_options::hub_T, {0, 256, 1024, 4096}},
      {&dbbc_options::part_work, {1 << 20, 1 << 22, 1 << 24}},
  };
  for (const Knob& kn : knobs) {
    for (int32_t v : kn.values) {
      if (cur.*kn.field == v) continue;
      dbbc_options o = cur;
      o.*kn.field = v;
      if (kn.field == &dbbc_options::window_L) o.reverse_L = std::min(v, 4096);
      float ms = 0.f;
      rc = time_opts(o, ms);
      if (rc != DBBC_OK) return rc;
      if (ms < cur_ms) {
        cur = o;
        cur_ms = ms;
      }
    }
  }
  // leave the graphs planned with the winner
  for (int32_t i = 0; i < k; ++i) {
    dbbc::PlanParams p;
    uint32_t long_len = 0;
    rc = params_from(gs[i], &cur, p, long_len);
    if (rc != DBBC_OK) return rc;
    dbbc::AllocScope plan_scope(gs[i]->al, st);
    rc = ensure_plan(gs[i], p, st);
    if (rc != DBBC_OK) return rc;
  }
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return DBBC_OK;
}

int dbbc_last_kernel_times(const dbbc_graph* g, dbbc_kernel_time* out, int32_t cap, int32_t* n_out) {
  if (!g || !n_out || cap < 0 || (cap > 0 && !out)) return fail(DBBC_E_INVALID_ARG, "NULL argument");
  if (!g->timed_valid) return fail(DBBC_E_INVALID_ARG, "no timed count on this handle");
  const int32_t n = static_cast<int32_t>(g->timers_used);
  for (int32_t i = 0; i < n && i < cap; ++i) {
    const KernelRec& t = g->timers[i];
    dbbc_kernel_time kt{};
    std::strncpy(kt.name, t.name.c_str(), sizeof(kt.name) - 1);
    kt.ms = t.ms;
    kt.wedges = t.wedges;
    kt.segments = t.segments;
    kt.items = t.items;
    kt.macs = t.macs;
    out[i] = kt;
  }
  *n_out = n;
  return DBBC_OK;
}

void dbbc_graph_destroy(dbbc_graph* g) { delete g; }

}  // extern "C"
