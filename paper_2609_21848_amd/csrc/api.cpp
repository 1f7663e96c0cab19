// The C ABI of libdbbc (include/dbbc.h): graph handles, plans and the
// stream-ordered launch sequence of a count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

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

// Device memory owned by a handle, freed on destruction.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t n) {
    release();
    if (n == 0) return hipSuccess;
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

template <class T>
hipError_t upload(DevBuf& b, const std::vector<T>& v, hipStream_t st) {
  hipError_t e = b.alloc(v.size() * sizeof(T));
  if (e != hipSuccess || v.empty()) return e;
  return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

// Control block: res[0..7] int64 results, then 8 uint32 work-queue heads.
constexpr size_t kCtlWords = 16;

struct DevPlan {
  dbbc::HostPlan host;
  DevBuf segs, small_segs, small_groups, direct_items, hash_items, reverse_items, reduces, acc;
  DevBuf hub_pairs[2], hub_B[2], hub_Bm[2];
  int32_t hub_K[2] = {0, 0};
  bool valid = false;
  size_t bytes() const {
    size_t b = segs.bytes + small_segs.bytes + small_groups.bytes + direct_items.bytes +
               hash_items.bytes + reverse_items.bytes + reduces.bytes + acc.bytes;
    for (int s = 0; s < 2; ++s) b += hub_pairs[s].bytes + hub_B[s].bytes + hub_Bm[s].bytes;
    return b;
  }
};

}  // namespace

// HIP events around one kernel launch of a timed count.
struct KernelRec {
  std::string name;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int64_t wedges = 0, segments = 0, items = 0, macs = 0;
  float ms = 0.f;
};

struct dbbc_graph {
  dbbc::HostGraph host;
  DeviceInfo dev;
  DevBuf adj[2], off[2];
  DevBuf ctl;
  unsigned long long* pinned = nullptr;  // host mirror of ctl results
  DevPlan plan;
  std::vector<KernelRec> timers;  // events are reused across timed counts
  size_t timers_used = 0;
  bool timed_valid = false;
  ~dbbc_graph() {
    if (pinned) (void)hipHostFree(pinned);
    for (auto& t : timers)
      for (auto& e : t.ev)
        if (e) (void)hipEventDestroy(e);
  }
};

namespace {

int ensure_plan(dbbc_graph* g, const dbbc::PlanParams& p, hipStream_t st) {
  if (g->plan.valid && g->plan.host.p == p) return DBBC_OK;
  g->plan.valid = false;
  std::string err;
  dbbc::HostPlan hp;
  int rc = dbbc::make_plan(g->host, p, hp, err);
  if (rc != DBBC_OK) return fail(rc, err);
  DevPlan& d = g->plan;
  HIP_TRY(upload(d.segs, hp.segs, st));
  HIP_TRY(upload(d.small_segs, hp.small_segs, st));
  HIP_TRY(upload(d.small_groups, hp.small_groups, st));
  HIP_TRY(upload(d.direct_items, hp.direct_items, st));
  HIP_TRY(upload(d.hash_items, hp.hash_items, st));
  HIP_TRY(upload(d.reverse_items, hp.reverse_items, st));
  HIP_TRY(upload(d.reduces, hp.reduces, st));
  HIP_TRY(d.acc.alloc(static_cast<size_t>(hp.acc_slots) * hp.acc_width * sizeof(uint32_t)));
  for (int s = 0; s < 2; ++s) {
    d.hub_pairs[s].release();
    d.hub_B[s].release();
    d.hub_Bm[s].release();
    d.hub_K[s] = 0;
    const int32_t T = hp.T[s], TO = hp.T[1 - s];
    if (T == 0) continue;
    HIP_TRY(d.hub_pairs[s].alloc(static_cast<size_t>(T) * T * sizeof(unsigned long long)));
    // pad the contraction dimension to a multiple of 64
    const int32_t K = (TO + 63) / 64 * 64;
    std::vector<int8_t> B(static_cast<size_t>(T) * K, 0), Bm(static_cast<size_t>(T) * K, 0);
    for (int32_t x = 0; x < T; ++x) {
      std::memcpy(&B[static_cast<size_t>(x) * K], &hp.hub_B[s][static_cast<size_t>(x) * TO], TO);
      std::memcpy(&Bm[static_cast<size_t>(x) * K], &hp.hub_Bm[s][static_cast<size_t>(x) * TO], TO);
    }
    HIP_TRY(upload(d.hub_B[s], B, st));
    HIP_TRY(upload(d.hub_Bm[s], Bm, st));
    d.hub_K[s] = K;
    hp.hub_B[s].clear();
    hp.hub_B[s].shrink_to_fit();
    hp.hub_Bm[s].clear();
    hp.hub_Bm[s].shrink_to_fit();
  }
  HIP_TRY(hipStreamSynchronize(st));
  // the host plan keeps only what later launches need
  hp.segs.clear();
  hp.segs.shrink_to_fit();
  hp.small_segs.clear();
  hp.small_segs.shrink_to_fit();
  hp.small_items.clear();
  hp.small_items.shrink_to_fit();
  d.host = std::move(hp);
  d.valid = true;
  return DBBC_OK;
}

// Runs of at least this many entries are streamed by a whole wavefront.
constexpr int32_t kDefaultLongLen = 256;

int params_from(const dbbc_graph* g, const dbbc_options* opt, dbbc::PlanParams& p, uint32_t& long_len) {
  p = dbbc::default_params(g->host);
  long_len = kDefaultLongLen;
  if (!opt) return DBBC_OK;
  if (opt->flags & ~DBBC_OPT_TIME_KERNELS) return fail(DBBC_E_INVALID_ARG, "unknown dbbc_options flag");
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

// Begin / end one timed launch (no-ops when timing is off).
struct Timing {
  dbbc_graph* g;
  hipStream_t st;
  bool on;
  KernelRec* cur = nullptr;
  int begin(const char* name, int64_t wedges, int64_t segs, int64_t items, int64_t macs) {
    if (!on) return DBBC_OK;
    if (g->timers_used == g->timers.size()) g->timers.emplace_back();
    cur = &g->timers[g->timers_used++];
    for (auto& e : cur->ev)
      if (!e) HIP_TRY(hipEventCreate(&e));
    cur->name = name;
    cur->wedges = wedges;
    cur->segments = segs;
    cur->items = items;
    cur->macs = macs;
    HIP_TRY(hipEventRecord(cur->ev[0], st));
    return DBBC_OK;
  }
  int end() {
    if (!on) return DBBC_OK;
    HIP_TRY(hipEventRecord(cur->ev[1], st));
    return DBBC_OK;
  }
};

#define RC_TRY(expr)            \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != DBBC_OK) return rc_; \
  } while (0)

// Enqueue the whole count on stream st; results land in g->ctl.
int enqueue_count(dbbc_graph* g, hipStream_t st, bool timed, uint32_t long_len) {
  Timing tm{g, st, timed};
  g->timers_used = 0;
  DevPlan& d = g->plan;
  const dbbc::HostPlan& hp = d.host;
  unsigned long long* ctl = g->ctl.as<unsigned long long>();
  uint32_t* queues = reinterpret_cast<uint32_t*>(ctl + 8);
  HIP_TRY(dbbc::launch_fill_u64(ctl, kCtlWords, 0ull, st));
  dbbc::DevSideConst side[2];
  for (int s = 0; s < 2; ++s) {
    side[s].other_adj = g->adj[1 - s].as<uint32_t>();
    side[s].hub_pairs = d.hub_pairs[s].as<unsigned long long>();
    side[s].T = hp.T[s];
    side[s].R = hp.R[s];
    side[s].key_bits = hp.key_bits[s];
    if (hp.T[s] > 0)
      HIP_TRY(dbbc::launch_fill_u64(side[s].hub_pairs, static_cast<size_t>(hp.T[s]) * hp.T[s], 0ull, st));
  }
  const int cus = g->dev.cus;
  {
    dbbc::DirectArgs a{};
    a.items = d.direct_items.as<dbbc::Item>();
    a.segs = d.segs.as<dbbc::Segment>();
    a.side[0] = side[0];
    a.side[1] = side[1];
    a.queue = queues + 0;
    a.acc = d.acc.as<uint32_t>();
    a.res = ctl;
    a.n_items = static_cast<int32_t>(hp.direct_items.size());
    a.acc_width = hp.acc_width;
    a.long_len = long_len;
    RC_TRY(tm.begin("direct", hp.k_wedges[0], hp.k_segs[0], a.n_items, 0));
    HIP_TRY(dbbc::launch_direct(a, std::min<int>(cus, std::max(1, a.n_items)), st));
    RC_TRY(tm.end());
  }
  {
    dbbc::SmallArgs a{};
    a.items = d.reverse_items.as<dbbc::Item>();
    a.segs = d.segs.as<dbbc::Segment>();
    a.side[0] = side[0];
    a.side[1] = side[1];
    a.queue = queues + 3;
    a.acc = d.acc.as<uint32_t>();
    a.acc_width = hp.acc_width;
    a.res = ctl;
    a.n_items = static_cast<int32_t>(hp.reverse_items.size());
    a.long_len = long_len;
    RC_TRY(tm.begin("reverse", hp.k_wedges[3], hp.k_segs[3], a.n_items, 0));
    HIP_TRY(dbbc::launch_reverse(a, std::min<int>(cus, std::max(1, (a.n_items + 15) / 16)), st));
    RC_TRY(tm.end());
  }
  {
    dbbc::SmallArgs a{};
    a.items = d.small_groups.as<dbbc::Item>();
    a.segs = d.small_segs.as<dbbc::Segment>();
    a.side[0] = side[0];
    a.side[1] = side[1];
    a.queue = queues + 1;
    a.res = ctl;
    a.n_items = static_cast<int32_t>(hp.small_groups.size());
    a.long_len = long_len;
    RC_TRY(tm.begin("small", hp.k_wedges[1], hp.k_segs[1], a.n_items, 0));
    HIP_TRY(dbbc::launch_small(a, std::min<int>(4 * cus, std::max(1, (a.n_items + 3) / 4)), st));
    RC_TRY(tm.end());
  }
  {
    dbbc::HashArgs a{};
    a.items = d.hash_items.as<dbbc::Item>();
    a.segs = d.segs.as<dbbc::Segment>();
    a.side[0] = side[0];
    a.side[1] = side[1];
    a.queue = queues + 2;
    a.res = ctl;
    a.n_items = static_cast<int32_t>(hp.hash_items.size());
    a.long_len = long_len;
    RC_TRY(tm.begin("hash", hp.k_wedges[2], hp.k_segs[2], a.n_items, 0));
    HIP_TRY(dbbc::launch_hash(a, std::min<int>(cus, std::max(1, a.n_items)), st));
    RC_TRY(tm.end());
  }
  {
    dbbc::ReduceArgs a{};
    a.reduces = d.reduces.as<dbbc::Reduce>();
    a.side[0] = side[0];
    a.side[1] = side[1];
    a.acc = d.acc.as<uint32_t>();
    a.res = ctl;
    a.n_reduces = static_cast<int32_t>(hp.reduces.size());
    a.acc_width = hp.acc_width;
    RC_TRY(tm.begin("reduce", 0, 0, a.n_reduces, 0));
    HIP_TRY(dbbc::launch_reduce(a, std::min<int>(4 * cus, std::max(1, a.n_reduces)), st));
    RC_TRY(tm.end());
  }
  for (int s = 0; s < 2; ++s) {
    if (hp.T[s] == 0) continue;
    dbbc::HubArgs a{};
    a.Bm = d.hub_Bm[s].as<int8_t>();
    a.B = d.hub_B[s].as<int8_t>();
    a.hub_pairs = side[s].hub_pairs;
    a.res = ctl;
    a.T = hp.T[s];
    a.K = d.hub_K[s];
    // two contractions over K for every tile of the upper triangle
    const int64_t nt = a.T / 128;
    const int64_t macs = 2 * (nt * (nt + 1) / 2) * 128 * 128 * static_cast<int64_t>(a.K);
    RC_TRY(tm.begin(s == 0 ? "hub_u" : "hub_v", 0, 0, nt * (nt + 1) / 2, macs));
    HIP_TRY(dbbc::launch_hub(a, st));
    RC_TRY(tm.end());
  }
  return DBBC_OK;
}

}  // namespace

extern "C" {

const char* dbbc_version(void) { return "0.1.0"; }

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
    default: return "unknown status";
  }
}

int dbbc_graph_create(int32_t n_u, int32_t n_v, int64_t m, const int32_t* u, const int32_t* v,
                      const int8_t* sign, uint32_t flags, void* hip_stream, dbbc_graph** out) {
  g_last_error.clear();
  if (!out) return fail(DBBC_E_INVALID_ARG, "out must not be NULL");
  if (flags & ~(DBBC_INPUT_DEVICE | DBBC_DUP_REJECT)) return fail(DBBC_E_INVALID_ARG, "unknown flag");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  DeviceInfo di;
  int rc;
  if (flags & DBBC_INPUT_DEVICE) {
    rc = current_device(di);
    if (rc != DBBC_OK) return rc;
  }
  std::vector<int32_t> hu, hv;
  std::vector<int8_t> hs;
  if ((flags & DBBC_INPUT_DEVICE) && m > 0) {
    if (!u || !v || !sign) return fail(DBBC_E_INVALID_ARG, "edge arrays must not be NULL");
    hu.resize(static_cast<size_t>(m));
    hv.resize(static_cast<size_t>(m));
    hs.resize(static_cast<size_t>(m));
    HIP_TRY(hipMemcpyAsync(hu.data(), u, m * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hv.data(), v, m * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hs.data(), sign, m * sizeof(int8_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    u = hu.data();
    v = hv.data();
    sign = hs.data();
  }
  std::unique_ptr<dbbc_graph> g(new (std::nothrow) dbbc_graph());
  if (!g) return fail(DBBC_E_OOM, "host allocation failed");
  std::string err;
  try {
    rc = dbbc::build_host_graph(n_u, n_v, m, u, v, sign, flags, g->host, err);
  } catch (const std::bad_alloc&) {
    return fail(DBBC_E_OOM, "host allocation failed while building the graph");
  }
  if (rc != DBBC_OK) return fail(rc, err);
  if (!di.ok) {
    rc = current_device(di);
    if (rc != DBBC_OK) return rc;
  }
  g->dev = di;
  for (int s = 0; s < 2; ++s) {
    std::vector<uint32_t>& adj = g->host.side[s].adj;
    const size_t m_side = adj.size();
    adj.resize(m_side + dbbc::kAdjPad, 0u);  // padding for 16-byte loads
    hipError_t e = upload(g->adj[s], adj, st);
    adj.resize(m_side);
    HIP_TRY(e);
    HIP_TRY(upload(g->off[s], g->host.side[s].off, st));
  }
  HIP_TRY(g->ctl.alloc(kCtlWords * sizeof(unsigned long long)));
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&g->pinned), kCtlWords * sizeof(unsigned long long),
                        hipHostMallocDefault));
  HIP_TRY(hipStreamSynchronize(st));
  *out = g.release();
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
  size_t b = g->ctl.bytes + g->plan.bytes();
  for (int k = 0; k < 2; ++k) b += g->adj[k].bytes + g->off[k].bytes;
  s.device_bytes = static_cast<int64_t>(b);
  s.wedges_vp = g->host.wedges_vp;
  s.pivots_active = g->host.pivots_active;
  *out = s;
  return DBBC_OK;
}

int dbbc_count(dbbc_graph* g, const dbbc_options* opt, dbbc_counts* out_host, void* hip_stream) {
  g_last_error.clear();
  if (!g || !out_host) return fail(DBBC_E_INVALID_ARG, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  dbbc::PlanParams p;
  uint32_t long_len = 0;
  int rc = params_from(g, opt, p, long_len);
  if (rc != DBBC_OK) return rc;
  rc = ensure_plan(g, p, st);
  if (rc != DBBC_OK) return rc;
  const bool timed = opt && (opt->flags & DBBC_OPT_TIME_KERNELS);
  g->timed_valid = false;
  rc = enqueue_count(g, st, timed, long_len);
  if (rc != DBBC_OK) return rc;
  HIP_TRY(hipMemcpyAsync(g->pinned, g->ctl.p, kCtlWords * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (g->pinned[dbbc::kResError] != 0)
    return fail(DBBC_E_DEVICE, "a kernel reported an internal overflow (error bits " +
                                   std::to_string(g->pinned[dbbc::kResError]) + ")");
  if (timed) {
    for (size_t i = 0; i < g->timers_used; ++i) {
      KernelRec& t = g->timers[i];
      HIP_TRY(hipEventElapsedTime(&t.ms, t.ev[0], t.ev[1]));
    }
    g->timed_valid = true;
  }
  out_host->balanced = static_cast<int64_t>(g->pinned[0]);
  out_host->unbalanced = static_cast<int64_t>(g->pinned[1]);
  out_host->total = static_cast<int64_t>(g->pinned[2]);
  out_host->wedges = g->host.wedges_vp;
  return DBBC_OK;
}

int dbbc_count_per_vertex(dbbc_graph* g, int64_t* bal_u, int64_t* bal_v, int64_t* unb_u,
                          int64_t* unb_v, dbbc_counts* out_host, void* hip_stream) {
  (void)g; (void)bal_u; (void)bal_v; (void)unb_u; (void)unb_v; (void)out_host; (void)hip_stream;
  return fail(DBBC_E_INVALID_ARG, "per-vertex counts are not available in this build");
}

int dbbc_count_batch(dbbc_graph* const* gs, int32_t k, const dbbc_options* opt,
                     dbbc_counts* out_host, void* hip_stream) {
  g_last_error.clear();
  if (k < 0 || (k > 0 && (!gs || !out_host))) return fail(DBBC_E_INVALID_ARG, "bad batch arguments");
  for (int32_t i = 0; i < k; ++i) {
    int rc = dbbc_count(gs[i], opt, &out_host[i], hip_stream);
    if (rc != DBBC_OK) return rc;
  }
  return DBBC_OK;
}

int dbbc_last_kernel_times(const dbbc_graph* g, dbbc_kernel_time* out, int32_t cap, int32_t* n_out) {
  if (!g || !n_out || cap < 0 || (cap > 0 && !out)) return fail(DBBC_E_INVALID_ARG, "NULL argument");
  if (!g->timed_valid) return fail(DBBC_E_INVALID_ARG, "no timed count on this handle");
  const int32_t n = static_cast<int32_t>(g->timers_used);
  for (int32_t i = 0; i < n && i < cap; ++i) {
    const KernelRec& t = g->timers[i];
    dbbc_kernel_time k{};
    std::strncpy(k.name, t.name.c_str(), sizeof(k.name) - 1);
    k.ms = t.ms;
    k.wedges = t.wedges;
    k.segments = t.segments;
    k.items = t.items;
    k.macs = t.macs;
    out[i] = k;
  }
  *n_out = n;
  return DBBC_OK;
}

void dbbc_graph_destroy(dbbc_graph* g) { delete g; }

}  // extern "C"
