// Request server of libdbbc: count queries on device-resident graphs of mixed
// sizes, with continuous batching (include/dbbc.h, dbbc_server_*).
//
// Built on the public entry points only.  One scheduler thread owns the
// launch slots (a HIP stream, an event and a reusable batch each).  Whenever
// a slot is free it takes the oldest waiting requests: a graph with at least
// solo_wedges vertex-priority wedges is counted alone (it fills the device
// by itself); smaller ones are packed, oldest first, into one batch of up to
// max_batch graphs and batch_wedges wedges.  Requests that arrive while
// launches run join the next free slot, so work of several launches
// overlaps on the device.  Several requests for one graph share its count
// (the count is a pure function of the graph) unless the server was made
// with DBBC_SERVER_NO_MERGE.  An uploader thread builds
// newly uploaded graphs, admitted against an HBM budget: idle uploaded
// graphs are evicted oldest first to make room, and an upload that cannot
// fit is rejected.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dbbc.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  int64_t ticket = 0;
  int32_t gid = -1;
  bool done = false;
  dbbc_counts res{};
  dbbc_request_info info{};
};

struct Upload {
  int64_t ticket;
  int32_t n_u, n_v;
  std::vector<int32_t> u, v;
  std::vector<int8_t> s;
};

struct GraphRec {
  dbbc_graph* g = nullptr;
  int64_t bytes = 0, wedges = 0, last_use = 0;
  int32_t pending = 0;  // waiting requests
  bool uploaded = false, busy = false;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  dbbc_batch* b = nullptr;
  bool busy = false, lone = false;
  dbbc_graph* lone_g = nullptr;  // the graph of a lone launch
  std::vector<int32_t> gids;
  std::vector<std::vector<int64_t>> tickets;  // per graph of the launch
};

}  // namespace

struct dbbc_server {
  dbbc_server_config cfg{};
  dbbc_options opt{};
  bool has_opt = false;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_up, cv_done;
  std::deque<int64_t> pending;
  std::deque<Upload> uploads;
  std::unordered_map<int64_t, Req> reqs;
  std::vector<GraphRec> graphs;
  std::vector<Slot> slots;
  int64_t next_ticket = 1;
  int64_t resident = 0;
  int32_t uploading = 0;
  dbbc_server_stats st{};
  bool stop = false;
  std::thread sched, up;

  const dbbc_options* o() const { return has_opt ? &opt : nullptr; }
  void run_scheduler();
  void run_uploader();
  void finish(int64_t ticket, int status, const dbbc_counts* c, int64_t t);
};

namespace {

thread_local std::string g_server_error;

int sfail(int status, const std::string& msg) {
  g_server_error = msg;
  return status;
}

// Build and plan a graph on a stream of its own.
int make_graph(const dbbc_options* opt, int32_t n_u, int32_t n_v, int64_t m, const int32_t* u,
               const int32_t* v, const int8_t* s, dbbc_graph** out, dbbc_stats* stats) {
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
    return sfail(DBBC_E_DEVICE, "hipStreamCreate failed");
  dbbc_graph* g = nullptr;
  int rc = dbbc_graph_create(n_u, n_v, m, u, v, s, 0u, nullptr, st, &g);
  if (rc == DBBC_OK) rc = dbbc_graph_plan(g, opt, st);
  if (rc == DBBC_OK) rc = dbbc_graph_stats(g, stats);
  if (rc != DBBC_OK) {
    g_server_error = dbbc_last_error();
    dbbc_graph_destroy(g);
    g = nullptr;
  }
  (void)hipStreamDestroy(st);
  *out = g;
  return rc;
}

}  // namespace

void dbbc_server::finish(int64_t ticket, int status, const dbbc_counts* c, int64_t t) {
  Req& r = reqs[ticket];
  r.done = true;
  r.info.status = status;
  r.info.t_done_ns = t;
  if (c) r.res = *c;
  if (status == DBBC_OK) {
    ++st.completed;
  } else {
    ++st.failed;
  }
}

void dbbc_server::run_scheduler() {
  (void)hipSetDevice(device);
  std::vector<dbbc_counts> out;
  std::vector<dbbc_graph*> gs;
  for (;;) {
    bool progress = false;
    // 1. completions
    for (Slot& sl : slots) {
      if (!sl.busy || hipEventQuery(sl.ev) != hipSuccess) continue;
      out.assign(sl.gids.size(), dbbc_counts{});
      int rc = sl.lone ? dbbc_count_read(sl.lone_g, out.data()) : dbbc_batch_read(sl.b, out.data());
      const int64_t t = now_ns();
      {
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < sl.gids.size(); ++i) {
          GraphRec& gr = graphs[sl.gids[i]];
          gr.busy = false;
          gr.last_use = t;
          for (int64_t tk : sl.tickets[i]) finish(tk, rc, &out[i], t);
        }
      }
      cv_done.notify_all();
      cv_up.notify_all();
      sl.busy = false;
      progress = true;
    }
    // 2. launches into free slots
    std::unique_lock<std::mutex> lk(mu);
    bool any_busy = false;
    for (Slot& sl : slots) any_busy |= sl.busy;
    if (stop && pending.empty() && uploads.empty() && uploading == 0 && !any_busy) break;
    for (Slot& sl : slots) {
      if (sl.busy || pending.empty()) continue;
      // choose the graphs of this launch, oldest request first
      sl.gids.clear();
      sl.tickets.clear();
      std::unordered_map<int32_t, size_t> pos;
      int64_t wedges = 0;
      bool lone = false;
      std::deque<int64_t> keep;
      for (int64_t tk : pending) {
        const int32_t gid = reqs[tk].gid;
        GraphRec& gr = graphs[gid];
        auto it = pos.find(gid);
        if (it != pos.end()) {
          if (cfg.flags & DBBC_SERVER_NO_MERGE) {  // its own count, in a later launch
            keep.push_back(tk);
          } else {  // shares a count already chosen
            sl.tickets[it->second].push_back(tk);
          }
          continue;
        }
        const bool big = gr.wedges >= cfg.solo_wedges;
        const bool fits = !gr.busy && !lone &&
                          (sl.gids.empty() ||
                           (!big && static_cast<int32_t>(sl.gids.size()) < cfg.max_batch &&
                            wedges + gr.wedges <= cfg.batch_wedges));
        if (!fits) {
          keep.push_back(tk);
          continue;
        }
        lone = big;
        pos[gid] = sl.gids.size();
        sl.gids.push_back(gid);
        sl.tickets.push_back({tk});
        wedges += gr.wedges;
      }
      if (sl.gids.empty()) break;  // everything waiting is on busy graphs
      pending.swap(keep);
      gs.clear();
      for (int32_t gid : sl.gids) {
        GraphRec& gr = graphs[gid];
        gr.busy = true;
        gr.pending -= static_cast<int32_t>(sl.tickets[gs.size()].size());
        gs.push_back(gr.g);
      }
      sl.lone = lone;
      sl.lone_g = lone ? gs[0] : nullptr;
      const int64_t t = now_ns();
      for (size_t i = 0; i < sl.gids.size(); ++i)
        for (int64_t tk : sl.tickets[i]) {
          reqs[tk].info.t_launch_ns = t;
          reqs[tk].info.batch_size = static_cast<int32_t>(sl.gids.size());
        }
      ++st.launches;
      st.batched_graphs += static_cast<int64_t>(sl.gids.size());
      lk.unlock();
      int rc;
      if (lone) {
        rc = dbbc_count_async(gs[0], o(), sl.st);
      } else {
        rc = dbbc_batch_reset(sl.b, gs.data(), static_cast<int32_t>(gs.size()), o(), 0u, sl.st);
        if (rc == DBBC_OK) rc = dbbc_batch_launch(sl.b, sl.st);
      }
      if (rc == DBBC_OK && hipEventRecord(sl.ev, sl.st) != hipSuccess) rc = DBBC_E_DEVICE;
      lk.lock();
      if (rc != DBBC_OK) {  // the launch failed: fail its requests
        const int64_t t2 = now_ns();
        for (size_t i = 0; i < sl.gids.size(); ++i) {
          graphs[sl.gids[i]].busy = false;
          for (int64_t tk : sl.tickets[i]) finish(tk, rc, nullptr, t2);
        }
        cv_done.notify_all();
        continue;
      }
      sl.busy = true;
      progress = true;
    }
    if (!progress) {
      // poll the busy slots every few microseconds; else sleep until work
      if (any_busy) {
        cv_work.wait_for(lk, std::chrono::microseconds(20));
      } else {
        cv_work.wait_for(lk, std::chrono::milliseconds(5));
      }
    }
  }
}

void dbbc_server::run_uploader() {
  (void)hipSetDevice(device);
  for (;;) {
    std::unique_lock<std::mutex> lk(mu);
    cv_up.wait(lk, [&] { return stop || !uploads.empty(); });
    if (uploads.empty()) {
      if (stop) break;
      continue;
    }
    Upload u = std::move(uploads.front());
    uploads.pop_front();
    // admission by footprint: an estimate first, the exact size after
    const int64_t m = static_cast<int64_t>(u.u.size());
    const int64_t estimate = 64 * m + (int64_t{1} << 20);
    std::vector<dbbc_graph*> evict;
    while (resident + estimate > cfg.hbm_budget) {
      int32_t lru = -1;
      for (int32_t i = 0; i < static_cast<int32_t>(graphs.size()); ++i) {
        const GraphRec& gr = graphs[i];
        if (gr.g && gr.uploaded && !gr.busy && gr.pending == 0 &&
            (lru < 0 || gr.last_use < graphs[lru].last_use))
          lru = i;
      }
      if (lru < 0) break;
      evict.push_back(graphs[lru].g);
      resident -= graphs[lru].bytes;
      graphs[lru] = GraphRec{};
      ++st.evicted;
    }
    if (resident + estimate > cfg.hbm_budget) {
      ++st.rejected;
      finish(u.ticket, DBBC_E_OOM, nullptr, now_ns());
      lk.unlock();
      cv_done.notify_all();
      for (dbbc_graph* g : evict) dbbc_graph_destroy(g);
      continue;
    }
    resident += estimate;
    ++uploading;
    lk.unlock();
    for (dbbc_graph* g : evict) dbbc_graph_destroy(g);
    dbbc_graph* g = nullptr;
    dbbc_stats s{};
    const int rc = make_graph(o(), u.n_u, u.n_v, m, u.u.data(), u.v.data(), u.s.data(), &g, &s);
    lk.lock();
    --uploading;
    resident -= estimate;
    if (rc != DBBC_OK) {
      finish(u.ticket, rc, nullptr, now_ns());
      lk.unlock();
      cv_done.notify_all();
      continue;
    }
    GraphRec gr;
    gr.g = g;
    gr.bytes = s.device_bytes;
    gr.wedges = s.wedges_vp;
    gr.uploaded = true;
    gr.pending = 1;
    gr.last_use = now_ns();
    resident += gr.bytes;
    graphs.push_back(gr);
    Req& r = reqs[u.ticket];
    r.gid = static_cast<int32_t>(graphs.size()) - 1;
    r.info.graph_id = r.gid;
    pending.push_back(u.ticket);
    lk.unlock();
    cv_work.notify_one();
  }
}

extern "C" {

int64_t dbbc_now_ns(void) { return now_ns(); }

const char* dbbc_server_last_error(void) { return g_server_error.c_str(); }

int dbbc_server_create(const dbbc_server_config* cfg, const dbbc_options* opt, dbbc_server** out) {
  g_server_error.clear();
  if (!out) return sfail(DBBC_E_INVALID_ARG, "out must not be NULL");
  if (opt && (opt->flags & DBBC_OPT_TIME_KERNELS))
    return sfail(DBBC_E_INVALID_ARG, "kernel timing is not available in the server");
  std::unique_ptr<dbbc_server> s(new (std::nothrow) dbbc_server());
  if (!s) return sfail(DBBC_E_OOM, "host allocation failed");
  if (cfg) s->cfg = *cfg;
  if (s->cfg.flags & ~DBBC_SERVER_NO_MERGE) return sfail(DBBC_E_INVALID_ARG, "unknown server flag");
  if (hipGetDevice(&s->device) != hipSuccess) return sfail(DBBC_E_NO_DEVICE, "no HIP device");
  if (s->cfg.slots <= 0) s->cfg.slots = 4;
  if (s->cfg.slots > 16) return sfail(DBBC_E_INVALID_ARG, "at most 16 slots");
  if (s->cfg.max_batch <= 0) s->cfg.max_batch = 512;
  if (s->cfg.solo_wedges <= 0) s->cfg.solo_wedges = int64_t{1} << 26;
  if (s->cfg.batch_wedges <= 0) s->cfg.batch_wedges = int64_t{1} << 28;
  if (s->cfg.hbm_budget <= 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return sfail(DBBC_E_DEVICE, "hipMemGetInfo failed");
    s->cfg.hbm_budget = static_cast<int64_t>(static_cast<double>(free_b) * 0.85);
  }
  if (opt) {
    s->opt = *opt;
    s->has_opt = true;
  }
  s->slots.resize(static_cast<size_t>(s->cfg.slots));
  for (Slot& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess)
      return sfail(DBBC_E_DEVICE, "stream or event creation failed");
    int rc = dbbc_batch_create(nullptr, 0, nullptr, 0u, sl.st, &sl.b);
    if (rc != DBBC_OK) return sfail(rc, dbbc_last_error());
  }
  dbbc_server* raw = s.get();
  raw->sched = std::thread([raw] { raw->run_scheduler(); });
  raw->up = std::thread([raw] { raw->run_uploader(); });
  *out = s.release();
  return DBBC_OK;
}

int dbbc_server_add_graph(dbbc_server* s, int32_t n_u, int32_t n_v, int64_t m, const int32_t* u,
                          const int32_t* v, const int8_t* sign, int32_t* graph_id) {
  g_server_error.clear();
  if (!s || !graph_id) return sfail(DBBC_E_INVALID_ARG, "NULL argument");
  dbbc_graph* g = nullptr;
  dbbc_stats st{};
  const int rc = make_graph(s->o(), n_u, n_v, m, u, v, sign, &g, &st);
  if (rc != DBBC_OK) return rc;
  std::lock_guard<std::mutex> lk(s->mu);
  GraphRec gr;
  gr.g = g;
  gr.bytes = st.device_bytes;
  gr.wedges = st.wedges_vp;
  gr.last_use = now_ns();
  s->resident += gr.bytes;
  s->graphs.push_back(gr);
  *graph_id = static_cast<int32_t>(s->graphs.size()) - 1;
  return DBBC_OK;
}

int dbbc_server_submit(dbbc_server* s, int32_t graph_id, int64_t* ticket) {
  g_server_error.clear();
  if (!s || !ticket) return sfail(DBBC_E_INVALID_ARG, "NULL argument");
  const int64_t t = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return sfail(DBBC_E_INVALID_ARG, "the server is stopping");
    if (graph_id < 0 || graph_id >= static_cast<int32_t>(s->graphs.size()) || !s->graphs[graph_id].g)
      return sfail(DBBC_E_INVALID_ARG, "no resident graph with this id");
    Req r;
    r.ticket = s->next_ticket++;
    r.gid = graph_id;
    r.info.graph_id = graph_id;
    r.info.t_submit_ns = t;
    r.info.queued_ahead = static_cast<int32_t>(s->pending.size());
    s->graphs[graph_id].pending++;
    s->pending.push_back(r.ticket);
    *ticket = r.ticket;
    s->reqs.emplace(r.ticket, r);
    ++s->st.submitted;
    s->st.max_queue = std::max<int64_t>(s->st.max_queue, static_cast<int64_t>(s->pending.size()));
  }
  s->cv_work.notify_one();
  return DBBC_OK;
}

int dbbc_server_submit_upload(dbbc_server* s, int32_t n_u, int32_t n_v, int64_t m, const int32_t* u,
                              const int32_t* v, const int8_t* sign, int64_t* ticket) {
  g_server_error.clear();
  if (!s || !ticket || m < 0 || (m > 0 && (!u || !v || !sign)))
    return sfail(DBBC_E_INVALID_ARG, "bad upload arguments");
  const int64_t t = now_ns();
  Upload up;
  up.n_u = n_u;
  up.n_v = n_v;
  up.u.assign(u, u + m);
  up.v.assign(v, v + m);
  up.s.assign(sign, sign + m);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return sfail(DBBC_E_INVALID_ARG, "the server is stopping");
    Req r;
    r.ticket = s->next_ticket++;
    r.info.graph_id = -1;
    r.info.t_submit_ns = t;
    r.info.queued_ahead = static_cast<int32_t>(s->pending.size());
    up.ticket = r.ticket;
    *ticket = r.ticket;
    s->reqs.emplace(r.ticket, r);
    s->uploads.push_back(std::move(up));
    ++s->st.submitted;
    ++s->st.uploads;
  }
  s->cv_up.notify_one();
  return DBBC_OK;
}

int dbbc_server_wait(dbbc_server* s, int64_t ticket, dbbc_counts* out, dbbc_request_info* info) {
  g_server_error.clear();
  if (!s) return sfail(DBBC_E_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return sfail(DBBC_E_INVALID_ARG, "unknown ticket");
  s->cv_done.wait(lk, [&] { return s->reqs[ticket].done; });
  const Req r = s->reqs[ticket];
  s->reqs.erase(ticket);
  if (out) *out = r.res;
  if (info) *info = r.info;
  return r.info.status;
}

int dbbc_server_get_stats(dbbc_server* s, dbbc_server_stats* out) {
  if (!s || !out) return sfail(DBBC_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  int64_t n = 0;
  for (const GraphRec& gr : s->graphs) n += gr.g != nullptr;
  out->resident_graphs = n;
  out->resident_bytes = s->resident;
  out->queued = static_cast<int64_t>(s->pending.size());
  return DBBC_OK;
}

void dbbc_server_destroy(dbbc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_up.notify_all();
  if (s->up.joinable()) s->up.join();
  if (s->sched.joinable()) s->sched.join();
  for (Slot& sl : s->slots) {
    dbbc_batch_destroy(sl.b);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
  }
  for (GraphRec& gr : s->graphs) dbbc_graph_destroy(gr.g);
  delete s;
}

}  // extern "C"
