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
#include <string>

#include "internal.h"

namespace dbbc {

// Density of the top T x T block of the bi-adjacency matrix (rows and
// columns in priority order).
double hub_density(const HostGraph& g, int32_t T) {
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
void pack_small_groups(const HostGraph& g, HostPlan& plan) {
  for (int s = 0; s < 2; ++s) {
    int32_t kb = 1;
    while ((int64_t{1} << kb) < g.side[s].n) ++kb;
    plan.key_bits[s] = kb;
  }
  plan.small_groups.clear();
  plan.small_segs.clear();
  Item grp{};
  bool open = false;
  uint32_t local = 0;
  auto close = [&]() {
    if (!open) return;
    grp.seg_count = static_cast<uint32_t>(plan.small_segs.size()) - grp.seg_begin;
    grp.key_hi = static_cast<int32_t>(local);  // items in the group
    plan.small_groups.push_back(grp);
    open = false;
  };
  for (const Item& it : plan.small_items) {
    const uint32_t max_items =
        std::min<uint32_t>(kSmallMaxItems, (1u << (32 - plan.key_bits[it.side])) - 1u);
    const bool hub = (it.flags & kItemHubPairs) != 0;
    if (open && (hub || (grp.flags & kItemHubPairs) || grp.side != it.side ||
                 grp.work + it.work > kSmallGroupWork || local >= max_items))
      close();
    if (!open) {
      grp = Item{};
      grp.seg_begin = static_cast<uint32_t>(plan.small_segs.size());
      grp.owner = it.owner;
      grp.acc_slot = plan.p.per_vertex ? static_cast<int32_t>(plan.small_owner.size()) : -1;
      grp.flags = it.flags & kItemHubPairs;
      grp.side = it.side;
      local = 0;
      open = true;
    }
    for (uint32_t k = 0; k < it.seg_count; ++k) {
      const Segment sg = plan.segs[it.seg_begin + k];
      plan.small_segs.push_back(Segment{sg.start, (local << 16) | sg.len_g});
      if (plan.p.per_vertex) {
        plan.small_seg_mid.push_back(plan.seg_mid[it.seg_begin + k]);
        plan.small_seg_edge.push_back(plan.seg_edge[it.seg_begin + k]);
      }
    }
    if (plan.p.per_vertex) plan.small_owner.push_back(it.owner);
    grp.work += it.work;
    ++local;
  }
  close();
}

// Drop the segments of the small items (copied into the groups) from segs.
// Consecutive items with the same runs (key windows of one item) keep
// sharing them.
void compact_segments(HostPlan& plan) {
  const bool pv = plan.p.per_vertex;
  std::vector<Segment> out;
  std::vector<uint32_t> out_mid, out_edge;
  size_t n = 0;
  for (auto* v : {&plan.direct_items, &plan.hash_items, &plan.reverse_items})
    for (const Item& it : *v) n += it.seg_count;
  out.reserve(n);
  if (pv) {
    out_mid.reserve(n);
    out_edge.reserve(n);
  }
  for (auto* v : {&plan.direct_items, &plan.hash_items, &plan.reverse_items}) {
    uint32_t last_begin = 0xffffffffu, last_count = 0, last_new = 0;
    for (Item& it : *v) {
      if (it.seg_begin == last_begin && it.seg_count == last_count) {
        it.seg_begin = last_new;
        continue;
      }
      last_begin = it.seg_begin;
      last_count = it.seg_count;
      last_new = static_cast<uint32_t>(out.size());
      out.insert(out.end(), plan.segs.begin() + it.seg_begin, plan.segs.begin() + it.seg_begin + it.seg_count);
      if (pv) {
        out_mid.insert(out_mid.end(), plan.seg_mid.begin() + it.seg_begin,
                       plan.seg_mid.begin() + it.seg_begin + it.seg_count);
        out_edge.insert(out_edge.end(), plan.seg_edge.begin() + it.seg_begin,
                        plan.seg_edge.begin() + it.seg_begin + it.seg_count);
      }
      it.seg_begin = last_new;
    }
  }
  plan.segs = std::move(out);
  plan.seg_mid = std::move(out_mid);
  plan.seg_edge = std::move(out_edge);
}

}  // namespace

int make_plan(const HostGraph& g, const PlanParams& p, HostPlan& plan, std::string& err) {
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
  plan = HostPlan();
  plan.p = p;
  const bool pv = p.per_vertex;
  for (int s = 0; s < 2; ++s) {
    plan.L[s] = std::min<int32_t>(p.window_L, g.side[s].n);
    plan.R[s] = std::min<int32_t>(p.reverse_L, plan.L[s]);
    // the dense block is tiled by 128 rows; the per-vertex pass has none
    plan.T[s] = pv ? 0 : std::min<int32_t>(p.hub_T, g.side[s].n / 128 * 128);
  }
  // The dense path needs a block on both sides of the pair.
  if (plan.T[0] == 0 || plan.T[1] == 0) plan.T[0] = plan.T[1] = 0;

  std::vector<Item> big_direct;

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
    for (int32_t y = 0; y < O.n; ++y) {
      const uint32_t* b = O.adj.data() + O.off[y];
      const uint32_t* e = O.adj.data() + O.off[y + 1];
      auto below = [&](int32_t k) {
        return static_cast<int32_t>(std::lower_bound(b, e, static_cast<uint32_t>(k) << 1) - b);
      };
      splitL[y] = below(L);
      splitR[y] = below(R);
      splitT[y] = below(T);
    }

    // A run of entries of row y (the wedges' mid) whose first edge is the
    // entry e of side s's CSR (its negative bit is the run's g).
    auto add_seg = [&](uint32_t start, uint32_t len, uint32_t e) {
      const uint32_t first = S.adj[e];
      plan.segs.push_back(Segment{start, (len << 1) | (first & 1u)});
      if (pv) {
        const uint32_t y = first >> 1;
        const uint64_t bound = static_cast<uint64_t>(O.off[y + 1] - O.off[y]) * static_cast<uint64_t>(S.max_deg);
        const bool wide = p.wide_all || bound >= (uint64_t{1} << 32);
        plan.seg_mid.push_back(y | (wide ? kMidWide : 0u));
        plan.seg_edge.push_back(e);
      }
    };

    auto place = [&](uint32_t seg_begin, int32_t owner, int32_t key_lo, int32_t key_hi,
                     uint32_t flags, ItemKind kind) {
      const uint32_t nseg = static_cast<uint32_t>(plan.segs.size() - seg_begin);
      int64_t work = 0;
      for (uint32_t k = 0; k < nseg; ++k) work += plan.segs[seg_begin + k].len_g >> 1;
      // With a single segment every pair of the item has at most one wedge
      // and adds nothing -- unless the pair's count is completed by the
      // dense hub block.
      if (nseg == 0 || (nseg < 2 && !(flags & kItemHubPairs))) {
        plan.w_skipped += work;
        plan.segs.resize(seg_begin);
        if (pv) {
          plan.seg_mid.resize(seg_begin);
          plan.seg_edge.resize(seg_begin);
        }
        return;
      }
      plan.w_sparse += work;
      if (kind == kReverseTail) {
        // rows are sorted by rank, so a run's last entry is its largest key:
        // the item's counters (and its parts' and reduce's) need only the
        // keys up to the largest one
        int32_t mx = key_lo;
        for (uint32_t k = 0; k < nseg; ++k) {
          const Segment sg = plan.segs[seg_begin + k];
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
        big_direct.push_back(it);  // per-vertex counts: one direct item
      } else if (kind == kReverseTail) {
        // parts of at most kReverseMaxSegs segments (8-bit counters)
        if (nseg <= kReverseMaxSegs) {
          plan.reverse_items.push_back(it);
          return;
        }
        const int32_t first_slot = plan.acc_slots;
        for (uint32_t k = 0; k < nseg; k += kReverseMaxSegs) {
          Item part = it;
          part.seg_begin = seg_begin + k;
          part.seg_count = std::min(kReverseMaxSegs, nseg - k);
          part.flags |= kItemMultiPart;
          part.acc_slot = plan.acc_slots++;
          part.work = static_cast<uint32_t>(std::min<int64_t>(item_work(plan, part), 0xffffffffll));
          plan.reverse_items.push_back(part);
        }
        Reduce r{};
        r.acc_slot = first_slot;
        r.n_parts = plan.acc_slots - first_slot;
        r.owner = owner;
        r.key_lo = key_lo;
        r.key_hi = key_hi;
        r.flags = flags;
        r.side = static_cast<uint32_t>(s);
        plan.reduces.push_back(r);
      } else if (work <= p.small_work) {
        plan.small_items.push_back(it);
      } else if (kind == kForwardTail) {
        plan.hash_items.push_back(it);
      } else {
        big_direct.push_back(it);
      }
    };

    // Forward items: pivots x of side s, split at the window boundary.
    for (int32_t x = 0; x < S.n; ++x) {
      const bool hub = x < T;
      const uint32_t e0 = S.off[x] + S.cut[x], e1 = S.off[x + 1];
      if (x < L) {  // keys (x, L)
        const uint32_t seg_begin = static_cast<uint32_t>(plan.segs.size());
        for (uint32_t e = e0; e < e1; ++e) {
          const uint32_t y = S.adj[e] >> 1;
          uint32_t start = O.off[y] + static_cast<uint32_t>(S.rev[e]) + 1;
          const uint32_t end = O.off[y] + static_cast<uint32_t>(splitL[y]);
          if (hub && static_cast<int32_t>(y) < TO)
            start = std::max(start, O.off[y] + static_cast<uint32_t>(splitT[y]));
          if (end > start)
            add_seg(start, end - start, e);
        }
        place(seg_begin, x, x + 1, L, hub ? kItemHubPairs : 0u, kForwardWindow);
      }
      if (x >= L) {  // keys (x, n): every endpoint is below the window
        const uint32_t seg_begin = static_cast<uint32_t>(plan.segs.size());
        for (uint32_t e = e0; e < e1; ++e) {
          const uint32_t y = S.adj[e] >> 1;
          const uint32_t start = O.off[y] + static_cast<uint32_t>(S.rev[e]) + 1;
          const uint32_t end = O.off[y + 1];
          if (end > start)
            add_seg(start, end - start, e);
        }
        place(seg_begin, x, x + 1, S.n, 0u, kForwardTail);
      }
    }
    // Reverse items: endpoints w of side s below the window; keys x < R
    // (reverse), then keys x in [R, L) (reverse-mid).  Within row y the keys
    // above y form the prefix [0, cut[y]).
    for (int32_t w = L; w < S.n; ++w) {
      uint32_t seg_begin = static_cast<uint32_t>(plan.segs.size());
      for (uint32_t e = S.off[w]; e < S.off[w + 1]; ++e) {
        const uint32_t y = S.adj[e] >> 1;
        const int32_t len = std::min(splitR[y], O.cut[y]);
        if (len > 0)
          add_seg(O.off[y], static_cast<uint32_t>(len), e);
      }
      place(seg_begin, w, 0, R, 0u, kReverseTail);
      if (R == L) continue;
      seg_begin = static_cast<uint32_t>(plan.segs.size());
      for (uint32_t e = S.off[w]; e < S.off[w + 1]; ++e) {
        const uint32_t y = S.adj[e] >> 1;
        const int32_t end = std::min(splitL[y], O.cut[y]);
        if (end > splitR[y])
          add_seg(O.off[y] + static_cast<uint32_t>(splitR[y]), static_cast<uint32_t>(end - splitR[y]), e);
      }
      place(seg_begin, w, R, L, 0u, kReverseMid);
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

  // Split heavy direct items into parts (work budget, and fewer than 2^16
  // segments so that per-part counts fit 16 bits), heaviest first.
  std::vector<std::pair<int64_t, size_t>> order;
  order.reserve(big_direct.size());
  for (size_t i = 0; i < big_direct.size(); ++i) order.push_back({item_work(plan, big_direct[i]), i});
  std::sort(order.begin(), order.end(), [](auto& a, auto& b) { return a.first > b.first; });
  int32_t width = 0;
  for (int s = 0; s < 2; ++s) width = std::max(width, plan.L[s]);
  plan.acc_width = width;
  std::vector<Item> parts, singles;
  for (auto& [work, i] : order) {
    const Item& it = big_direct[i];
    if (pv) {  // whole items, key windows of at most kPVWindow keys
      for (int32_t lo = it.key_lo; lo < it.key_hi; lo += kPVWindow) {
        Item w = it;
        w.key_lo = lo;
        w.key_hi = std::min(it.key_hi, lo + kPVWindow);
        singles.push_back(w);
      }
      continue;
    }
    if (work <= p.part_work && it.seg_count < 65536) {
      singles.push_back(it);
      continue;
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
  return DBBC_OK;
}

}  // namespace dbbc
