// Counting plan: splits the vertex-priority wedges of Algorithm 1 (Phase 5)
// into work items whose counters fit on chip, and lays out the dense hub
// block for the matrix-core path.
//
// Every VP wedge x - y - w (y and w of lower priority than x, w on x's side)
// belongs to exactly one same-side pair (x, w), and Lemma 1 needs all wedges
// of a pair in one place before C(., 2) is taken.  Per side, with a window
// of the L highest-priority vertices and a reverse window of the R <= L
// highest, each pair (sr(x) < sr(w)) is owned by exactly one item:
//   forward-window  sr(w) < L              : at pivot x, keys w in (x, L)
//   reverse         sr(x) < R, sr(w) >= L  : at endpoint w, keys x in [0, R);
//                                            the same wedges walked from w:
//                                            for each neighbour y of w, the
//                                            entries of row y that rank above
//                                            both R and y
//   reverse-mid     R <= sr(x) < L <= sr(w): at endpoint w, keys x in [R, L)
//   forward-tail    sr(x) >= L             : at pivot x, keys w in (x, n)
// Inside the window, the pairs of the hub block (x, w < T, mid y < T on the
// other side) are counted by the dense path; forward items skip those wedges
// and leave their other hub-pair wedges in a pair buffer that the dense path
// adds before taking C(., 2).
#include <algorithm>
#include <atomic>
#include <climits>
#include <string>
#include <thread>

#include "internal.h"

namespace dbbc {

// Density of the top T x T block of the bi-adjacency matrix (rows and
// columns in priority order).
double hub_density(const HostGraph& g, int32_t T) {
  for (int k = 0; k < 3; ++k)
    if ((4096 >> k) == T && g.hub_nnz[k] >= 0) return static_cast<double>(g.hub_nnz[k]) / (static_cast<double>(T) * T);
  const HostSide& S = g.side[0];
  int64_t nnz = 0;
  for (int32_t x = 0; x < T; ++x) {
    const uint32_t* b = S.adj.data() + S.off[x];
    const uint32_t* e = S.adj.data() + S.off[x + 1];
    nnz += std::lower_bound(b, e, static_cast<uint32_t>(T) << 1) - b;
  }
  return static_cast<double>(nnz) / (static_cast<double>(T) * T);
}

PlanParams default_params(const HostGraph& g, int32_t hub_slots) {
  PlanParams p;
  p.window_L = 32768;
  p.reverse_L = 4096;
  // The dense path costs T^3 MACs whatever the block holds, and saves the
  // sparse wedges inside it: take the largest T whose block is at least
  // 15% full (both sides need 2T vertices).
  p.hub_T = 0;
  for (int32_t T : {4096, 2048, 1024}) {
    if (g.side[0].n < 2 * T || g.side[1].n < 2 * T) continue;
    if (hub_density(g, T) >= 0.15) {
      p.hub_T = T;
      break;
    }
  }
  // A tile round past the device's slots would run a few tiles alone for a
  // whole tile time: trim the block to the largest one whose nt (nt + 1) / 2
  // tiles fit (4096 -> 3968 with 512 slots).
  int32_t nt = p.hub_T / 128;
  while (nt > 1 && nt * (nt + 1) / 2 > hub_slots) --nt;
  if (p.hub_T > 0) p.hub_T = nt * 128;
  p.small_work = static_cast<int32_t>(kSmallGroupWork);
  p.part_work = 1 << 24;
  return p;
}

namespace {

int64_t item_work(const HostPlan& plan, const Item& it) {
  int64_t w = 0;
  for (uint32_t k = 0; k < it.seg_count; ++k) w += plan.segs[it.seg_begin + k].len_g >> 1;
  return w;
}

// Pack the small items, in plan order, into groups of at most
// kSmallGroupWork wedges that one wavefront counts in one hash table.  A
// group's hash key is (index of the item in the group << key_bits) | key, so
// the group may hold at most 2^(32 - key_bits) - 1 items (the all-ones word
// marks an empty slot).  Items whose hub-pair counts go to the dense path
// stay alone in their group (the group's owner and flags are theirs).
int planner_threads() {
  const unsigned hw = std::thread::hardware_concurrency();
  return static_cast<int>(std::max(1u, std::min(hw == 0 ? 1u : hw, 16u)));
}

// f(i) for i in [0, n), in blocks of 4096 taken in turn by a pool of threads.
template <class F>
void parallel_for(size_t n, F f) {
  const size_t blocks = (n + 4095) / 4096;
  std::atomic<size_t> next{0};
  auto worker = [&]() {
    for (size_t b; (b = next.fetch_add(1)) < blocks;)
      for (size_t i = b * 4096; i < std::min(n, b * 4096 + 4096); ++i) f(i);
  };
  std::vector<std::thread> pool;
  const int nt = planner_threads();
  for (int t = 1; t < nt && static_cast<size_t>(t) < blocks; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
}

void pack_small_groups(const HostGraph& g, HostPlan& plan) {
  for (int s = 0; s < 2; ++s) {
    int32_t kb = 1;
    while ((int64_t{1} << kb) < g.side[s].n) ++kb;
    plan.key_bits[s] = kb;
  }
  const bool pv = plan.p.per_vertex;
  plan.small_groups.clear();
  plan.small_segs.clear();
  // the grouping (sequential: a group closes when the next item does not
  // fit), then each item's runs copied to its place in the groups' runs
  const size_t ni = plan.small_items.size();
  std::vector<uint32_t> dest(ni), local_of(ni);
  Item grp{};
  bool open = false;
  uint32_t local = 0, nsegs = 0;
  auto close = [&]() {
    if (!open) return;
    grp.seg_count = nsegs - grp.seg_begin;
    grp.key_hi = static_cast<int32_t>(local);  // items in the group
    plan.small_groups.push_back(grp);
    open = false;
  };
  for (size_t i = 0; i < ni; ++i) {
    const Item& it = plan.small_items[i];
    const uint32_t max_items =
        std::min<uint32_t>(kSmallMaxItems, (1u << (32 - plan.key_bits[it.side])) - 1u);
    const bool hub = (it.flags & kItemHubPairs) != 0;
    if (open && (hub || (grp.flags & kItemHubPairs) || grp.side != it.side ||
                 grp.work + it.work > kSmallGroupWork || local >= max_items))
      close();
    if (!open) {
      grp = Item{};
      grp.seg_begin = nsegs;
      grp.owner = it.owner;
      grp.acc_slot = pv ? static_cast<int32_t>(i) : -1;  // owners are listed per item
      grp.flags = it.flags & kItemHubPairs;
      grp.side = it.side;
      local = 0;
      open = true;
    }
    dest[i] = nsegs;
    local_of[i] = local;
    nsegs += it.seg_count;
    grp.work += it.work;
    ++local;
  }
  close();
  plan.small_segs.resize(nsegs);
  if (pv) {
    plan.small_seg_mid.resize(nsegs);
    plan.small_seg_edge.resize(nsegs);
    plan.small_owner.resize(ni);
  }
  parallel_for(ni, [&](size_t i) {
    const Item& it = plan.small_items[i];
    for (uint32_t k = 0; k < it.seg_count; ++k) {
      const Segment sg = plan.segs[it.seg_begin + k];
      plan.small_segs[dest[i] + k] = Segment{sg.start, (local_of[i] << 16) | sg.len_g};
      if (pv) {
        plan.small_seg_mid[dest[i] + k] = plan.seg_mid[it.seg_begin + k];
        plan.small_seg_edge[dest[i] + k] = plan.seg_edge[it.seg_begin + k];
      }
    }
    if (pv) plan.small_owner[i] = it.owner;
  });
}

// Drop the segments of the small items (copied into the groups) from segs.
// Consecutive items with the same runs (key windows of one item) keep
// sharing them.  New places first (in list order), then parallel copies.
void compact_segments(HostPlan& plan) {
  const bool pv = plan.p.per_vertex;
  std::vector<Item*> items;
  std::vector<uint32_t> from;  // old seg_begin of the items that copy
  size_t n = 0;
  for (auto* v : {&plan.direct_items, &plan.hash_items, &plan.reverse_items}) {
    uint32_t last_begin = 0xffffffffu, last_count = 0, last_new = 0;
    for (Item& it : *v) {
      if (it.seg_begin == last_begin && it.seg_count == last_count) {
        it.seg_begin = last_new;
        continue;
      }
      last_begin = it.seg_begin;
      last_count = it.seg_count;
      last_new = static_cast<uint32_t>(n);
      items.push_back(&it);
      from.push_back(it.seg_begin);
      it.seg_begin = last_new;
      n += it.seg_count;
    }
  }
  std::vector<Segment> out(n);
  std::vector<uint32_t> out_mid(pv ? n : 0), out_edge(pv ? n : 0);
  parallel_for(items.size(), [&](size_t i) {
    const Item& it = *items[i];
    std::copy(plan.segs.begin() + from[i], plan.segs.begin() + from[i] + it.seg_count, out.begin() + it.seg_begin);
    if (pv) {
      std::copy(plan.seg_mid.begin() + from[i], plan.seg_mid.begin() + from[i] + it.seg_count,
                out_mid.begin() + it.seg_begin);
      std::copy(plan.seg_edge.begin() + from[i], plan.seg_edge.begin() + from[i] + it.seg_count,
                out_edge.begin() + it.seg_begin);
    }
  });
  plan.segs = std::move(out);
  plan.seg_mid = std::move(out_mid);
  plan.seg_edge = std::move(out_edge);
}

// The runs and items of a range of owners of one side, built apart (one
// range per task) and appended to the plan in owner order, so the plan does
// not depend on how the owners were shared among threads.
struct Piece {
  std::vector<Segment> segs;
  std::vector<uint32_t> seg_mid, seg_edge;
  std::vector<Item> small_items, hash_items, reverse_items, big_direct;
  std::vector<Reduce> reduces;  // acc_slot relative to the piece
  int32_t acc_slots = 0;
  int64_t w_sparse = 0, w_skipped = 0;
};

// Split rows [r0, r1) of a CSR with offsets off into about 64 ranges per
// thread of equal entry counts and run f(lo, hi, range index) on a pool of
// threads taking ranges in turn.  Returns the number of ranges.
template <class F>
size_t parallel_ranges(const std::vector<uint32_t>& off, int32_t r0, int32_t r1, F f) {
  if (r1 <= r0) return 0;
  const int nt = planner_threads();
  const uint64_t total = static_cast<uint64_t>(off[r1] - off[r0]) + static_cast<uint64_t>(r1 - r0);
  const size_t want = static_cast<size_t>(nt) * 64;
  std::vector<int32_t> cuts{r0};
  for (size_t k = 1; k < want; ++k) {
    // first row whose (entries + rows) prefix reaches k / want of the total
    const uint64_t goal = total * k / want;
    int32_t lo = cuts.back(), hi = r1;
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo) / 2;
      if (static_cast<uint64_t>(off[mid] - off[r0]) + static_cast<uint64_t>(mid - r0) < goal)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo > cuts.back() && lo < r1) cuts.push_back(lo);
  }
  cuts.push_back(r1);
  const size_t n = cuts.size() - 1;
  std::atomic<size_t> next{0};
  auto worker = [&]() {
    for (size_t i; (i = next.fetch_add(1)) < n;) f(cuts[i], cuts[i + 1], i);
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt && static_cast<size_t>(t) < n; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  return n;
}

// One Piece per range of owners in [r0, r1), each owner handled by f(P, owner).
template <class F>
std::vector<Piece> build_pieces(const std::vector<uint32_t>& off, int32_t r0, int32_t r1, F f) {
  std::vector<Piece> pieces(static_cast<size_t>(planner_threads()) * 64 + 2);
  const size_t n = parallel_ranges(off, r0, r1, [&](int32_t lo, int32_t hi, size_t i) {
    for (int32_t x = lo; x < hi; ++x) f(pieces[i], x);
  });
  pieces.resize(n);
  return pieces;
}

int merge_pieces(HostPlan& plan, std::vector<Piece>& pieces, std::vector<Item>& big_direct, std::string& err) {
  // every piece's place in each list, then the copies in parallel
  const size_t n = pieces.size();
  struct At {
    size_t seg, mid, small, hash, rev, big, red;
    int64_t slot;
  };
  std::vector<At> at(n + 1);
  at[0] = At{plan.segs.size(), plan.seg_mid.size(), plan.small_items.size(), plan.hash_items.size(),
             plan.reverse_items.size(), big_direct.size(), plan.reduces.size(), plan.acc_slots};
  for (size_t i = 0; i < n; ++i) {
    const Piece& P = pieces[i];
    at[i + 1] = At{at[i].seg + P.segs.size(), at[i].mid + P.seg_mid.size(), at[i].small + P.small_items.size(),
                   at[i].hash + P.hash_items.size(), at[i].rev + P.reverse_items.size(),
                   at[i].big + P.big_direct.size(), at[i].red + P.reduces.size(), at[i].slot + P.acc_slots};
    plan.w_sparse += P.w_sparse;
    plan.w_skipped += P.w_skipped;
  }
  // runs are addressed by 32-bit indices and items by 32-bit counts: check
  // before any index is narrowed
  PlanSizes z{};
  z.runs = at[n].seg;
  z.items = std::max({at[n].small, at[n].hash, at[n].rev, at[n].big});
  z.reduces = at[n].red;
  z.acc_slots = static_cast<uint64_t>(at[n].slot);
  const int rc = check_plan_sizes(z, err);
  if (rc != DBBC_OK) return rc;
  plan.segs.resize(at[n].seg);
  plan.seg_mid.resize(at[n].mid);
  plan.seg_edge.resize(at[n].mid);
  plan.small_items.resize(at[n].small);
  plan.hash_items.resize(at[n].hash);
  plan.reverse_items.resize(at[n].rev);
  big_direct.resize(at[n].big);
  plan.reduces.resize(at[n].red);
  plan.acc_slots = static_cast<int32_t>(at[n].slot);
  std::atomic<size_t> next{0};
  auto worker = [&]() {
    for (size_t i; (i = next.fetch_add(1)) < n;) {
      Piece& P = pieces[i];
      const uint32_t base = static_cast<uint32_t>(at[i].seg);
      const int32_t slot0 = static_cast<int32_t>(at[i].slot);
      auto shift = [&](const std::vector<Item>& from, std::vector<Item>& to, size_t pos) {
        for (Item it : from) {
          it.seg_begin += base;
          if (it.acc_slot >= 0) it.acc_slot += slot0;
          to[pos++] = it;
        }
      };
      std::copy(P.segs.begin(), P.segs.end(), plan.segs.begin() + at[i].seg);
      std::copy(P.seg_mid.begin(), P.seg_mid.end(), plan.seg_mid.begin() + at[i].mid);
      std::copy(P.seg_edge.begin(), P.seg_edge.end(), plan.seg_edge.begin() + at[i].mid);
      shift(P.small_items, plan.small_items, at[i].small);
      shift(P.hash_items, plan.hash_items, at[i].hash);
      shift(P.reverse_items, plan.reverse_items, at[i].rev);
      shift(P.big_direct, big_direct, at[i].big);
      size_t r = at[i].red;
      for (Reduce red : P.reduces) {
        red.acc_slot += slot0;
        plan.reduces[r++] = red;
      }
      P = Piece();  // free as we go
    }
  };
  std::vector<std::thread> pool;
  const int nt = planner_threads();
  for (int t = 1; t < nt && static_cast<size_t>(t) < n; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  return DBBC_OK;
}

}  // namespace

int check_plan_sizes(const PlanSizes& z, std::string& err) {
  const uint64_t i32max = static_cast<uint64_t>(INT32_MAX);
  if (z.runs > UINT32_MAX) {
    err = "graph too large: the plan has " + std::to_string(z.runs) + " runs (at most 2^32 - 1)";
    return DBBC_E_TOO_LARGE;
  }
  if (z.items > i32max || z.reduces > i32max || z.acc_slots > i32max) {
    err = "graph too large: the plan has " + std::to_string(z.items) + " items of one kind, " +
          std::to_string(z.reduces) + " reduces and " + std::to_string(z.acc_slots) +
          " accumulator slots (each at most 2^31 - 1)";
    return DBBC_E_TOO_LARGE;
  }
  return DBBC_OK;
}

int check_plan_params(const PlanParams& p, std::string& err) {
  if (p.window_L < 256 || p.window_L > 32768 || p.window_L % 256 != 0) {
    err = "window_L must be a multiple of 256 in [256, 32768]";
    return DBBC_E_INVALID_ARG;
  }
  if (p.reverse_L < 64 || p.reverse_L > kMaxReverseL || p.reverse_L % 64 != 0 ||
      p.reverse_L > p.window_L) {
    err = "reverse_L must be a multiple of 64 in [64, 4096], at most window_L";
    return DBBC_E_INVALID_ARG;
  }
  if (p.hub_T < 0 || p.hub_T > 16384 || p.hub_T % 128 != 0) {
    err = "hub_T must be 0 or a multiple of 128 up to 16384";
    return DBBC_E_INVALID_ARG;
  }
  if (p.hub_T > p.window_L) {
    err = "hub_T must not exceed window_L";
    return DBBC_E_INVALID_ARG;
  }
  if (p.small_work < 2 || p.small_work > static_cast<int32_t>(kSmallGroupWork) || p.part_work < 4096) {
    err = "small_work must be in [2, " + std::to_string(kSmallGroupWork) +
          "] and part_work at least 4096";
    return DBBC_E_INVALID_ARG;
  }
  return DBBC_OK;
}

void plan_windows(const int32_t n[2], const PlanParams& p, HostPlan& plan) {
  const bool pv = p.per_vertex;
  for (int s = 0; s < 2; ++s) {
    plan.L[s] = std::min<int32_t>(p.window_L, n[s]);
    plan.R[s] = std::min<int32_t>(p.reverse_L, plan.L[s]);
    // the dense block is tiled by 128 rows (at most kMaxPVHubT in the
    // per-vertex pass)
    plan.T[s] = std::min<int32_t>(pv ? std::min(p.hub_T, kMaxPVHubT) : p.hub_T, n[s] / 128 * 128);
  }
  // The dense path needs a block on both sides of the pair.
  if (plan.T[0] == 0 || plan.T[1] == 0) plan.T[0] = plan.T[1] = 0;
  plan.acc_width = std::max(plan.L[0], plan.L[1]);
}

int make_plan(const HostGraph& g, const PlanParams& p, HostPlan& plan, std::string& err) {
  {
    const int rc = check_plan_params(p, err);
    if (rc != DBBC_OK) return rc;
  }
  plan = HostPlan();
  plan.p = p;
  const bool pv = p.per_vertex;
  {
    const int32_t n[2] = {g.side[0].n, g.side[1].n};
    plan_windows(n, p, plan);
  }

  std::vector<Item> big_direct;
  // pieces of both sides in plan order (side 0 forward, side 0 reverse,
  // side 1 forward, side 1 reverse), merged once at the end
  std::vector<Piece> pieces;
  auto keep = [&](std::vector<Piece>&& v) {
    for (Piece& P : v) pieces.push_back(std::move(P));
  };

  for (int s = 0; s < 2; ++s) {
    const HostSide& S = g.side[s];
    const HostSide& O = g.side[1 - s];
    const int32_t L = plan.L[s];
    const int32_t R = plan.R[s];
    const int32_t T = plan.T[s];
    const int32_t TO = plan.T[1 - s];  // hub rows of the other side (mids)
    // Per row y of the other side (its entries are keys of side s): how many
    // entries lie below the window, the reverse window and the hub block.
    std::vector<int32_t> splitL(O.n), splitR(O.n), splitT(O.n);
    parallel_ranges(O.off, 0, O.n, [&](int32_t y0, int32_t y1, size_t) {
      for (int32_t y = y0; y < y1; ++y) {
        const uint32_t* b = O.adj.data() + O.off[y];
        const uint32_t* e = O.adj.data() + O.off[y + 1];
        auto below = [&](int32_t k) {
          return static_cast<int32_t>(std::lower_bound(b, e, static_cast<uint32_t>(k) << 1) - b);
        };
        splitL[y] = below(L);
        splitR[y] = below(R);
        splitT[y] = below(T);
      }
    });

    // A run of entries of row y (the wedges' mid) whose first edge is the
    // entry e of side s's CSR (its negative bit is the run's g).
    auto add_seg = [&](Piece& P, uint32_t start, uint32_t len, uint32_t e) {
      const uint32_t first = S.adj[e];
      P.segs.push_back(Segment{start, (len << 1) | (first & 1u)});
      if (pv) {
        const uint32_t y = first >> 1;
        const uint64_t bound = static_cast<uint64_t>(O.off[y + 1] - O.off[y]) * static_cast<uint64_t>(S.max_deg);
        const bool wide = p.wide_all || bound >= (uint64_t{1} << 32);
        P.seg_mid.push_back(y | (wide ? kMidWide : 0u));
        P.seg_edge.push_back(e);
      }
    };

    auto place = [&](Piece& P, uint32_t seg_begin, int32_t owner, int32_t key_lo, int32_t key_hi,
                     uint32_t flags, ItemKind kind) {
      const uint32_t nseg = static_cast<uint32_t>(P.segs.size() - seg_begin);
      int64_t work = 0;
      for (uint32_t k = 0; k < nseg; ++k) work += P.segs[seg_begin + k].len_g >> 1;
      // With a single segment every pair of the item has at most one wedge
      // and adds nothing -- unless the pair's count is completed by the
      // dense hub block.
      if (nseg == 0 || (nseg < 2 && !(flags & kItemHubPairs))) {
        P.w_skipped += work;
        P.segs.resize(seg_begin);
        if (pv) {
          P.seg_mid.resize(seg_begin);
          P.seg_edge.resize(seg_begin);
        }
        return;
      }
      P.w_sparse += work;
      if (kind == kReverseTail) {
        // rows are sorted by rank, so a run's last entry is its largest key:
        // the item's counters (and its parts' and reduce's) need only the
        // keys up to the largest one
        int32_t mx = key_lo;
        for (uint32_t k = 0; k < nseg; ++k) {
          const Segment sg = P.segs[seg_begin + k];
          mx = std::max(mx, static_cast<int32_t>(O.adj[sg.start + (sg.len_g >> 1) - 1] >> 1));
        }
        key_hi = std::min(key_hi, mx + 1);
      }
      Item it{};
      it.seg_begin = seg_begin;
      it.seg_count = nseg;
      it.owner = owner;
      it.key_lo = key_lo;
      it.key_hi = key_hi;
      it.acc_slot = -1;
      it.flags = flags;
      it.side = static_cast<uint32_t>(s);
      it.work = static_cast<uint32_t>(std::min<int64_t>(work, 0xffffffffll));
      if (kind == kReverseTail && pv && nseg > kReverseMaxSegs) {
        P.big_direct.push_back(it);  // per-vertex counts: one direct item
      } else if (kind == kReverseTail) {
        // parts of at most kReverseMaxSegs segments (8-bit counters; signed
        // 8-bit in a count plan)
        const uint32_t max_segs = pv ? kReverseMaxSegs : kReverseCountMaxSegs;
        if (nseg <= max_segs) {
          P.reverse_items.push_back(it);
          return;
        }
        const int32_t first_slot = P.acc_slots;
        for (uint32_t k = 0; k < nseg; k += max_segs) {
          Item part = it;
          part.seg_begin = seg_begin + k;
          part.seg_count = std::min(max_segs, nseg - k);
          part.flags |= kItemMultiPart;
          part.acc_slot = P.acc_slots++;
          int64_t pw = 0;
          for (uint32_t j = 0; j < part.seg_count; ++j) pw += P.segs[part.seg_begin + j].len_g >> 1;
          part.work = static_cast<uint32_t>(std::min<int64_t>(pw, 0xffffffffll));
          P.reverse_items.push_back(part);
        }
        Reduce r{};
        r.acc_slot = first_slot;
        r.n_parts = P.acc_slots - first_slot;
        r.owner = owner;
        r.key_lo = key_lo;
        r.key_hi = key_hi;
        r.flags = flags;
        r.side = static_cast<uint32_t>(s);
        P.reduces.push_back(r);
      } else if (work <= p.small_work) {
        P.small_items.push_back(it);
      } else if (kind == kForwardTail) {
        P.hash_items.push_back(it);
      } else {
        P.big_direct.push_back(it);
      }
    };

    // Forward items: pivots x of side s, split at the window boundary.
    std::vector<Piece> fwd = build_pieces(S.off, 0, S.n, [&](Piece& P, int32_t x) {
      const bool hub = x < T;
      const uint32_t e0 = S.off[x] + S.cut[x], e1 = S.off[x + 1];
      if (x < L) {  // keys (x, L)
        const uint32_t seg_begin = static_cast<uint32_t>(P.segs.size());
        for (uint32_t e = e0; e < e1; ++e) {
          const uint32_t y = S.adj[e] >> 1;
          uint32_t start = O.off[y] + static_cast<uint32_t>(S.rev[e]) + 1;
          const uint32_t end = O.off[y] + static_cast<uint32_t>(splitL[y]);
          if (hub && static_cast<int32_t>(y) < TO)
            start = std::max(start, O.off[y] + static_cast<uint32_t>(splitT[y]));
          if (end > start)
            add_seg(P, start, end - start, e);
        }
        place(P, seg_begin, x, x + 1, L, hub ? kItemHubPairs : 0u, kForwardWindow);
      }
      if (x >= L) {  // keys (x, n): every endpoint is below the window
        const uint32_t seg_begin = static_cast<uint32_t>(P.segs.size());
        for (uint32_t e = e0; e < e1; ++e) {
          const uint32_t y = S.adj[e] >> 1;
          const uint32_t start = O.off[y] + static_cast<uint32_t>(S.rev[e]) + 1;
          const uint32_t end = O.off[y + 1];
          if (end > start)
            add_seg(P, start, end - start, e);
        }
        place(P, seg_begin, x, x + 1, S.n, 0u, kForwardTail);
      }
    });
    keep(std::move(fwd));
    // Reverse items: endpoints w of side s below the window; keys x < R
    // (reverse), then keys x in [R, L) (reverse-mid).  Within row y the keys
    // above y form the prefix [0, cut[y]).
    std::vector<Piece> rev = build_pieces(S.off, L, S.n, [&](Piece& P, int32_t w) {
      uint32_t seg_begin = static_cast<uint32_t>(P.segs.size());
      for (uint32_t e = S.off[w]; e < S.off[w + 1]; ++e) {
        const uint32_t y = S.adj[e] >> 1;
        const int32_t len = std::min(splitR[y], O.cut[y]);
        if (len > 0)
          add_seg(P, O.off[y], static_cast<uint32_t>(len), e);
      }
      place(P, seg_begin, w, 0, R, 0u, kReverseTail);
      if (R == L) return;
      seg_begin = static_cast<uint32_t>(P.segs.size());
      for (uint32_t e = S.off[w]; e < S.off[w + 1]; ++e) {
        const uint32_t y = S.adj[e] >> 1;
        const int32_t end = std::min(splitL[y], O.cut[y]);
        if (end > splitR[y])
          add_seg(P, O.off[y] + static_cast<uint32_t>(splitR[y]), static_cast<uint32_t>(end - splitR[y]), e);
      }
      place(P, seg_begin, w, R, L, 0u, kReverseMid);
    });
    keep(std::move(rev));

    // Per-vertex plans: the sparse wedges of every hub pivot toward hub
    // endpoints, as runs of their own (the prefix below T of each of the
    // pivot's runs through a non-hub mid).
    if (pv && T > 0) {
      std::vector<uint32_t> nrun(static_cast<size_t>(T) + 1, 0);
      auto hub_runs = [&](int32_t x, auto&& emit) {
        for (uint32_t e = S.off[x] + S.cut[x]; e < S.off[x + 1]; ++e) {
          const uint32_t y = S.adj[e] >> 1;
          if (static_cast<int32_t>(y) < TO) continue;  // dense wedges
          const uint32_t start = O.off[y] + static_cast<uint32_t>(S.rev[e]) + 1;
          const uint32_t end = O.off[y] + static_cast<uint32_t>(splitT[y]);
          if (end > start) emit(start, end - start, e);
        }
      };
      parallel_for(static_cast<size_t>(T), [&](size_t x) {
        uint32_t c = 0;
        hub_runs(static_cast<int32_t>(x), [&](uint32_t, uint32_t, uint32_t) { ++c; });
        nrun[x + 1] = c;
      });
      for (int32_t x = 0; x < T; ++x) nrun[x + 1] += nrun[x];
      const size_t base = plan.hub_segs.size();
      if (base + nrun[T] > UINT32_MAX) {
        err = "graph too large: the dense block's sparse runs exceed 2^32 - 1";
        return DBBC_E_TOO_LARGE;
      }
      plan.hub_segs.resize(base + nrun[T]);
      std::vector<Item> its(static_cast<size_t>(T));
      parallel_for(static_cast<size_t>(T), [&](size_t x) {
        size_t k = base + nrun[x];
        int64_t work = 0;
        hub_runs(static_cast<int32_t>(x), [&](uint32_t start, uint32_t len, uint32_t e) {
          plan.hub_segs[k++] = Segment{start, (len << 1) | (S.adj[e] & 1u)};
          work += len;
        });
        Item& it = its[x];
        it = Item{};
        it.seg_begin = static_cast<uint32_t>(base + nrun[x]);
        it.seg_count = nrun[x + 1] - nrun[x];
        it.owner = static_cast<int32_t>(x);
        it.key_lo = static_cast<int32_t>(x) + 1;
        it.key_hi = T;
        it.acc_slot = -1;
        it.flags = kItemHubPairs;
        it.side = static_cast<uint32_t>(s);
        it.work = static_cast<uint32_t>(std::min<int64_t>(work, 0xffffffffll));
      });
      // heavy pivots in parts of about kHubTallyPartWork wedges (the tally
      // adds each part's counts into the pivot's row), so that one pivot
      // does not hold the tally's last workgroup alone
      for (const Item& it : its) {
        if (!it.seg_count) continue;
        uint32_t k = it.seg_begin;
        const uint32_t end = it.seg_begin + it.seg_count;
        while (k < end) {
          Item part = it;
          part.seg_begin = k;
          int64_t w = 0;
          do {
            w += plan.hub_segs[k].len_g >> 1;
            ++k;
          } while (k < end && w + (plan.hub_segs[k].len_g >> 1) <= kHubTallyPartWork);
          part.seg_count = k - part.seg_begin;
          part.work = static_cast<uint32_t>(w);
          plan.hub_items.push_back(part);
        }
      }
      if (s == 0) plan.n_hub_side0 = static_cast<int32_t>(plan.hub_items.size());
    }

    // Dense hub block of this side: B[x][y] for x < T, y < TO.
    if (T > 0) {
      auto& Bs = plan.hub_B[s];
      auto& Bm = plan.hub_Bm[s];
      Bs.assign(static_cast<size_t>(T) * TO, 0);
      Bm.assign(static_cast<size_t>(T) * TO, 0);
      for (int32_t x = 0; x < T; ++x) {
        for (uint32_t e = S.off[x]; e < S.off[x + 1]; ++e) {
          const int32_t y = static_cast<int32_t>(S.adj[e] >> 1);
          if (y >= TO) break;  // row sorted by y
          const int8_t sg = (S.adj[e] & 1u) ? int8_t(-1) : int8_t(1);
          Bs[static_cast<size_t>(x) * TO + y] = sg;
          if (O.grank[y] > S.grank[x]) Bm[static_cast<size_t>(x) * TO + y] = sg;
        }
      }
    }
  }

  {
    const int rc = merge_pieces(plan, pieces, big_direct, err);
    if (rc != DBBC_OK) return rc;
  }
  pieces.clear();
  pieces.shrink_to_fit();

  // Split heavy direct items into parts (work budget, and fewer than 2^16
  // segments so that per-part counts fit 16 bits), heaviest first.
  std::vector<std::pair<int64_t, size_t>> order;
  order.reserve(big_direct.size());
  for (size_t i = 0; i < big_direct.size(); ++i) order.push_back({item_work(plan, big_direct[i]), i});
  std::sort(order.begin(), order.end(), [](auto& a, auto& b) { return a.first > b.first; });
  std::vector<Item> parts, singles;
  for (auto& [work, i] : order) {
    const Item& it = big_direct[i];
    if (pv) {  // whole items, key windows of at most kPVWindow(Packed) keys
      const HostSide& S = g.side[it.side];
      const int32_t T = plan.T[it.side];
      const int64_t deg_T = T < S.n ? static_cast<int64_t>(S.off[T + 1] - S.off[T]) : 0;
      const bool packed = pv_packed(it.seg_count, (it.flags & kItemHubPairs) != 0, deg_T);
      const int32_t win = packed ? kPVWindowPacked : kPVWindow;
      for (int32_t lo = it.key_lo; lo < it.key_hi; lo += win) {
        Item w = it;
        w.key_lo = lo;
        w.key_hi = std::min(it.key_hi, lo + win);
        if (packed) w.flags |= kItemPacked;
        singles.push_back(w);
      }
      continue;
    }
    if (work <= p.part_work && it.seg_count < 65536) {
      singles.push_back(it);
      continue;
    }
    if (plan.acc_slots > INT32_MAX - static_cast<int32_t>(std::min<uint32_t>(it.seg_count, INT32_MAX))) {
      err = "graph too large: more than 2^31 - 1 accumulator slots";
      return DBBC_E_TOO_LARGE;
    }
    const int32_t first_slot = plan.acc_slots;
    uint32_t k = 0;
    while (k < it.seg_count) {
      Item part = it;
      part.seg_begin = it.seg_begin + k;
      int64_t pw = 0;
      uint32_t c = 0;
      while (k + c < it.seg_count && c < 65535) {
        const int64_t l = plan.segs[it.seg_begin + k + c].len_g >> 1;
        if (c > 0 && pw + l > p.part_work) break;
        pw += l;
        ++c;
      }
      part.seg_count = c;
      part.work = static_cast<uint32_t>(std::min<int64_t>(pw, 0xffffffffll));
      part.flags = it.flags | kItemMultiPart;
      part.acc_slot = plan.acc_slots++;
      parts.push_back(part);
      k += c;
    }
    Reduce r{};
    r.acc_slot = first_slot;
    r.n_parts = plan.acc_slots - first_slot;
    r.owner = it.owner;
    r.key_lo = it.key_lo;
    r.key_hi = it.key_hi;
    r.flags = it.flags;
    r.side = it.side;
    plan.reduces.push_back(r);
  }
  {
    PlanSizes z{};
    z.runs = plan.segs.size();
    z.items = parts.size() + singles.size();
    z.reduces = plan.reduces.size();
    z.acc_slots = static_cast<uint64_t>(plan.acc_slots);
    const int rc = check_plan_sizes(z, err);
    if (rc != DBBC_OK) return rc;
  }
  // parts first (they are the heaviest), then the single-part items
  plan.direct_items = std::move(parts);
  plan.direct_items.insert(plan.direct_items.end(), singles.begin(), singles.end());
  if (pv) {  // the per-vertex pass launches each side's direct items apart
    std::stable_partition(plan.direct_items.begin(), plan.direct_items.end(),
                          [](const Item& it) { return it.side == 0; });
    for (const Item& it : plan.direct_items) plan.n_direct_side0 += it.side == 0;
  }
  // heavy tail pivots first as well
  std::stable_sort(plan.hash_items.begin(), plan.hash_items.end(),
                   [&](const Item& a, const Item& b) { return item_work(plan, a) > item_work(plan, b); });
  pack_small_groups(g, plan);
  compact_segments(plan);
  auto tally = [&](int k, const std::vector<Item>& v) {
    for (const Item& it : v) {
      plan.k_wedges[k] += item_work(plan, it);
      plan.k_segs[k] += it.seg_count;
    }
  };
  for (const Item& it : plan.reverse_items) plan.n_reverse_side0 += it.side == 0;
  tally(0, plan.direct_items);
  tally(2, plan.hash_items);
  tally(3, plan.reverse_items);
  for (const Item& grp : plan.small_groups) {  // group work never saturates
    plan.k_wedges[1] += grp.work;
    plan.k_segs[1] += grp.seg_count;
  }
  // the counting kernel's reverse sweep (signed 8-bit products) needs every
  // reverse item, or part, to have at most kReverseCountMaxSegs runs
  const uint32_t max_segs = p.per_vertex ? kReverseMaxSegs : kReverseCountMaxSegs;
  for (const Item& it : plan.reverse_items) {
    if (it.seg_count > max_segs) {
      err = "internal: a reverse item has " + std::to_string(it.seg_count) + " runs";
      return DBBC_E_DEVICE;
    }
  }
  return DBBC_OK;
}

}  // namespace dbbc
