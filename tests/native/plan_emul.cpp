// Test harness (CPU only): builds the library's host graph and counting plan
// and walks every planned item the way the kernels do, in plain loops, so the
// split of the vertex-priority wedges into items can be checked on the CPU.
#include <climits>
#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "host_build.h"

using namespace dbbc;

namespace {
struct Acc {
  int64_t bal = 0, unb = 0, tot = 0;
  void add(int64_t p, int64_t n) {
    bal += p * (p - 1) / 2 + n * (n - 1) / 2;
    unb += p * n;
    tot += (p + n) * (p + n - 1) / 2;
  }
};
}  // namespace

extern "C" int plan_emulate(int32_t n_u, int32_t n_v, int64_t m, const int32_t* u, const int32_t* v,
                            const int8_t* sign, int32_t hub_T, int32_t window_L, int32_t reverse_L,
                            int32_t small_work, int32_t part_work, int64_t* out /* 13 */) {
  HostGraph g;
  std::string err;
  int rc = build_host_graph(n_u, n_v, m, u, v, sign, 0, g, err);
  if (rc) return rc;
  PlanParams p = default_params(g);
  if (hub_T >= 0) p.hub_T = hub_T;
  if (window_L >= 0) p.window_L = window_L;
  if (reverse_L >= 0) p.reverse_L = reverse_L;
  if (small_work >= 0) p.small_work = small_work;
  if (part_work >= 0) p.part_work = part_work;
  HostPlan plan;
  rc = make_plan(g, p, plan, err);
  if (rc) {
    fprintf(stderr, "make_plan: %s\n", err.c_str());
    return rc;
  }
  Acc acc;
  // hub pair partials: (side, x, w) -> (p, n)
  std::map<std::tuple<int, int, int>, std::pair<int64_t, int64_t>> hub;
  std::map<int32_t, std::vector<std::pair<int64_t, int64_t>>> parts;  // acc slot -> per key
  int64_t walked = 0;
  auto run = [&](const Item& it, int64_t limit) {
    const HostSide& O = g.side[1 - it.side];
    std::unordered_map<uint32_t, std::pair<int64_t, int64_t>> cnt;
    for (uint32_t k = 0; k < it.seg_count; ++k) {
      const Segment s = plan.segs[it.seg_begin + k];
      const uint32_t len = s.len_g >> 1, gb = s.len_g & 1;
      for (uint32_t t = 0; t < len; ++t) {
        uint32_t e = O.adj[s.start + t];
        uint32_t key = e >> 1;
        if ((int32_t)key < it.key_lo || (int32_t)key >= it.key_hi) return -100;  // key outside the item's window
        if (((e ^ gb) & 1u) == 0) cnt[key].first++; else cnt[key].second++;
        ++walked;
      }
    }
    for (auto& [key, pn] : cnt) {
      if (pn.first > limit || pn.second > limit) return -101;  // packed counter overflow
      if (it.flags & kItemMultiPart) {
        auto& vec = parts[it.acc_slot];
        if (vec.empty()) vec.assign(plan.acc_width, {0, 0});
        vec[key].first += pn.first;
        vec[key].second += pn.second;
      } else if ((it.flags & kItemHubPairs) && (int32_t)key < plan.T[it.side]) {
        auto& h = hub[{(int)it.side, it.owner, (int)key}];
        h.first += pn.first;
        h.second += pn.second;
      } else {
        acc.add(pn.first, pn.second);
      }
    }
    return 0;
  };
  for (auto* list : {&plan.direct_items, &plan.hash_items})
    for (const Item& it : *list) {
      if ((rc = run(it, 65535))) return rc;
    }
  // small-item groups: tagged runs, one hash per group keyed by
  // (index in group << key_bits) | key, as the kernel keys it
  for (const Item& grp : plan.small_groups) {
    const HostSide& O = g.side[1 - grp.side];
    const uint32_t kb = (uint32_t)plan.key_bits[grp.side];
    if (grp.work > kSmallGroupWork) return -105;
    if ((grp.flags & kItemHubPairs) && grp.key_hi != 1) return -106;  // hub items stay alone
    std::unordered_map<uint32_t, std::pair<int64_t, int64_t>> cnt;
    int64_t w = 0;
    for (uint32_t k = 0; k < grp.seg_count; ++k) {
      const Segment s = plan.small_segs[grp.seg_begin + k];
      const uint32_t local = s.len_g >> 16, len = (s.len_g & 0xffffu) >> 1, gb = s.len_g & 1u;
      if ((int32_t)local >= grp.key_hi) return -107;
      for (uint32_t t = 0; t < len; ++t) {
        const uint32_t e = O.adj[s.start + t];
        const uint32_t key = e >> 1;
        if ((key >> kb) != 0) return -108;
        const uint32_t hk = (local << kb) | key;
        if (hk == 0xffffffffu) return -109;  // would collide with the empty marker
        if (((e ^ gb) & 1u) == 0) cnt[hk].first++; else cnt[hk].second++;
        ++walked;
        ++w;
      }
    }
    if (w != grp.work) return -110;
    for (auto& [hk, pn] : cnt) {
      const int32_t key = (int32_t)(hk & ((1u << kb) - 1u));
      if ((grp.flags & kItemHubPairs) && key < plan.T[grp.side]) {
        auto& h = hub[{(int)grp.side, grp.owner, key}];
        h.first += pn.first;
        h.second += pn.second;
      } else {
        acc.add(pn.first, pn.second);
      }
    }
  }
  for (const Item& it : plan.reverse_items)
    if ((rc = run(it, kReverseCountMaxSegs))) return rc;
  for (const Reduce& r : plan.reduces) {
    for (int32_t key = r.key_lo; key < r.key_hi; ++key) {
      int64_t P = 0, N = 0;
      for (int32_t j = 0; j < r.n_parts; ++j) {
        auto f = parts.find(r.acc_slot + j);
        if (f == parts.end()) continue;
        P += f->second[key].first;
        N += f->second[key].second;
      }
      if (!(P | N)) continue;
      if ((r.flags & kItemHubPairs) && key < plan.T[r.side]) {
        auto& h = hub[{(int)r.side, r.owner, key}];
        h.first += P;
        h.second += N;
      } else {
        acc.add(P, N);
      }
    }
  }
  // dense block, in the matrix form: X = |Bm| |B|^T, Y = Bm B^T
  int64_t wdense = 0;
  for (int s = 0; s < 2; ++s) {
    const int32_t T = plan.T[s], K = plan.T[1 - s];
    if (!T) continue;
    const auto& B = plan.hub_B[s];
    const auto& Bm = plan.hub_Bm[s];
    for (int32_t x = 0; x < T; ++x)
      for (int32_t w = x + 1; w < T; ++w) {
        int64_t X = 0, Y = 0;
        for (int32_t y = 0; y < K; ++y) {
          int a = Bm[(size_t)x * K + y], b = B[(size_t)w * K + y];
          X += (a != 0) * (b != 0);
          Y += a * b;
        }
        int64_t P = (X + Y) / 2, N = (X - Y) / 2;
        auto f = hub.find({s, x, w});
        if (f != hub.end()) {
          P += f->second.first;
          N += f->second.second;
          hub.erase(f);
        }
        acc.add(P, N);
        wdense += X;
      }
  }
  if (!hub.empty()) return -102;  // a hub partial found no dense pair
  out[0] = acc.bal;
  out[1] = acc.unb;
  out[2] = acc.tot;
  out[3] = g.wedges_vp;
  out[4] = plan.w_sparse;
  out[5] = plan.w_skipped;
  out[6] = wdense;
  out[7] = walked;
  out[8] = (int64_t)plan.small_groups.size();
  out[9] = (int64_t)plan.direct_items.size();
  out[10] = (int64_t)plan.hash_items.size();
  out[11] = (int64_t)plan.reduces.size();
  out[12] = (int64_t)plan.reverse_items.size();
  return 0;
}

// The per-vertex pass as the kernels take it: every item of the per-vertex
// plan (no parts) is tallied, then its wedges are walked again to credit
// each mid with p - 1 (symmetric wedge) or n - 1 balanced and n or p
// unbalanced butterflies of the pair, and each pair's C(p,2) + C(n,2) and
// p n go to its key vertex and, summed, to the owner.  With a dense block
// (hub_T > 0): the hub items' runs are tallied first into the hub pairs'
// sparse counts, the block's wedges (hub mids) complete them, the hub
// pairs' key and owner credits and every credit of a block wedge are taken
// from the completed counts (in plain loops here, by matrix products on the
// device), and the hub items' own walks read the completed counts for hub
// keys and leave their key credits out.
// Outputs are per input id: bal / unb of size n_u + n_v (U first).
extern "C" int plan_emulate_pv(int32_t n_u, int32_t n_v, int64_t m, const int32_t* u, const int32_t* v,
                               const int8_t* sign, int32_t hub_T, int32_t window_L, int32_t reverse_L,
                               int32_t small_work, int64_t* bal, int64_t* unb, int64_t* bal_e, int64_t* unb_e,
                               int64_t* out /* 5 */) {
  HostGraph g;
  std::string err;
  int rc = build_host_graph(n_u, n_v, m, u, v, sign, 0, g, err);
  if (rc) return rc;
  PlanParams p = default_params(g);
  if (hub_T >= 0) p.hub_T = hub_T;
  if (window_L >= 0) p.window_L = window_L;
  if (reverse_L >= 0) p.reverse_L = reverse_L;
  if (small_work >= 0) p.small_work = small_work;
  p.per_vertex = true;
  HostPlan plan;
  rc = make_plan(g, p, plan, err);
  if (rc) {
    fprintf(stderr, "make_plan: %s\n", err.c_str());
    return rc;
  }
  if (!plan.reduces.empty() || plan.acc_slots != 0) return -120;  // no parts in this plan
  if (plan.seg_mid.size() != plan.segs.size() || plan.small_seg_mid.size() != plan.small_segs.size())
    return -121;
  if (plan.seg_edge.size() != plan.segs.size() || plan.small_seg_edge.size() != plan.small_segs.size())
    return -125;
  // input record of the entry at position q of side s's CSR (V entries map
  // to their U entry through the reverse positions)
  auto rec = [&](int s, uint32_t q) -> int64_t {
    if (s == 0) return g.side[0].rec[q];
    const uint32_t x = g.side[1].adj[q] >> 1;
    return g.side[0].rec[g.side[0].off[x] + static_cast<uint32_t>(g.side[1].rev[q])];
  };
  const int64_t base[2] = {0, n_u};
  Acc acc;
  auto id = [&](int s, uint32_t sr) { return base[s] + g.side[s].orig[sr]; };
  // position of the edge (x, y) in side s's CSR (x of side s, y of the other)
  auto pos_of = [&](int s, uint32_t x, uint32_t y) -> uint32_t {
    const HostSide& S = g.side[s];
    for (uint32_t q = S.off[x]; q < S.off[x + 1]; ++q)
      if ((S.adj[q] >> 1) == y) return q;
    return 0xffffffffu;
  };
  // Dense block: hub pairs' counts (sparse tally of the hub runs, then the
  // block's wedges), their key and owner credits, and the credits of every
  // block wedge (mid, pivot-mid edge, end-mid edge).
  std::map<std::tuple<int, int, int>, std::pair<int64_t, int64_t>> hubpn;  // (side, x, w) -> (P, N)
  for (const Item& it : plan.hub_items) {
    if (!(it.flags & kItemHubPairs) || it.owner >= plan.T[it.side]) return -130;
    const HostSide& O = g.side[1 - it.side];
    for (uint32_t k = it.seg_begin; k < it.seg_begin + it.seg_count; ++k) {
      const Segment sg = plan.hub_segs[k];
      for (uint32_t t = 0; t < (sg.len_g >> 1); ++t) {
        const uint32_t e = O.adj[sg.start + t];
        const int32_t key = (int32_t)(e >> 1);
        if (key <= it.owner || key >= plan.T[it.side]) return -131;  // hub runs hold hub keys only
        auto& pn = hubpn[{(int)it.side, it.owner, key}];
        (((e ^ sg.len_g) & 1u) == 0 ? pn.first : pn.second)++;
      }
    }
  }
  for (int s = 0; s < 2 && plan.T[0] > 0; ++s) {
    const int32_t T = plan.T[s], TO = plan.T[1 - s];
    const std::vector<int8_t>& B = plan.hub_B[s];
    const std::vector<int8_t>& Bm = plan.hub_Bm[s];
    for (int32_t x = 0; x < T; ++x)
      for (int32_t w = x + 1; w < T; ++w)
        for (int32_t y = 0; y < TO; ++y) {
          const int8_t a = Bm[(size_t)x * TO + y], b = B[(size_t)w * TO + y];
          if (a && b) (a == b ? hubpn[{s, x, w}].first : hubpn[{s, x, w}].second)++;
        }
    for (int32_t x = 0; x < T; ++x)
      for (int32_t w = x + 1; w < T; ++w) {
        auto f = hubpn.find({s, x, w});
        if (f == hubpn.end()) continue;
        const int64_t P = f->second.first, N = f->second.second;
        const int64_t cb = P * (P - 1) / 2 + N * (N - 1) / 2, cu = P * N;
        acc.add(P, N);
        bal[id(s, x)] += cb;
        unb[id(s, x)] += cu;
        bal[id(s, w)] += cb;
        unb[id(s, w)] += cu;
        for (int32_t y = 0; y < TO; ++y) {
          const int8_t a = Bm[(size_t)x * TO + y], b = B[(size_t)w * TO + y];
          if (!a || !b) continue;
          const bool sym = a == b;
          const int64_t wb = sym ? P - 1 : N - 1, wu = sym ? N : P;
          bal[id(1 - s, y)] += wb;
          unb[id(1 - s, y)] += wu;
          if (bal_e) {
            const int64_t r0 = rec(s, pos_of(s, x, y)), r1 = rec(s, pos_of(s, w, y));
            bal_e[r0] += wb;
            unb_e[r0] += wu;
            bal_e[r1] += wb;
            unb_e[r1] += wu;
          }
        }
      }
  }
  // the completed counts of a hub pair (x, key) of side `side`
  auto hub_lookup = [&](int side, int32_t x, int32_t key, int64_t& P, int64_t& N) {
    auto f = hubpn.find({side, x, key});
    P = f == hubpn.end() ? 0 : f->second.first;
    N = f == hubpn.end() ? 0 : f->second.second;
  };
  // one item: runs [b, b + c) of segs / mids, key filter, owner lookup
  auto run = [&](int side, const Segment* segs, const uint32_t* mids, const uint32_t* edges, uint32_t b,
                 uint32_t c, int32_t lo, int32_t hi, bool tagged, const int32_t* owners, int32_t owner,
                 int32_t maxcnt, bool hub_item) -> int {
    const HostSide& O = g.side[1 - side];
    std::map<std::pair<uint32_t, uint32_t>, std::pair<int64_t, int64_t>> cnt;  // (local, key)
    for (int pass = 0; pass < 2; ++pass) {
      for (uint32_t k = b; k < b + c; ++k) {
        const Segment sg = segs[k];
        const uint32_t local = tagged ? sg.len_g >> 16 : 0;
        const uint32_t len = tagged ? (sg.len_g & 0xffffu) >> 1 : sg.len_g >> 1, gb = sg.len_g & 1u;
        for (uint32_t t = 0; t < len; ++t) {
          const uint32_t e = O.adj[sg.start + t];
          const int32_t key = (int32_t)(e >> 1);
          if (key < lo || key >= hi) {
            if (!tagged && lo == 0 && hi == INT32_MAX) return -122;
            continue;  // another key window of the same runs
          }
          const bool sym = ((e ^ gb) & 1u) == 0;
          // a hub pair's wedge: its counts are the completed ones
          const bool hubkey = hub_item && key < plan.T[side];
          if (hubkey && pass == 0) continue;
          auto& pn = cnt[{local, (uint32_t)key}];
          if (pass == 0) {
            (sym ? pn.first : pn.second)++;
          } else {
            int64_t Pk = pn.first, Nk = pn.second;
            if (hubkey) hub_lookup(side, owners ? owners[local] : owner, key, Pk, Nk);
            const int64_t mid = id(1 - side, mids[k] & ~kMidWide);
            const int64_t cb = sym ? Pk - 1 : Nk - 1, cu = sym ? Nk : Pk;
            bal[mid] += cb;
            unb[mid] += cu;
            if (bal_e) {  // the run's first edge and the walked entry's edge
              const int64_t r0 = rec(side, edges[k]), r1 = rec(1 - side, sg.start + t);
              bal_e[r0] += cb;
              unb_e[r0] += cu;
              bal_e[r1] += cb;
              unb_e[r1] += cu;
            }
          }
        }
      }
    }
    std::map<uint32_t, std::pair<int64_t, int64_t>> own;  // per local: owner sums
    for (auto& [lk, pn] : cnt) {
      if (hub_item && (int32_t)lk.second < plan.T[side]) continue;  // credited by the dense block
      if (pn.first > maxcnt || pn.second > maxcnt) return -123;
      const int64_t P = pn.first, N = pn.second;
      const int64_t cb = P * (P - 1) / 2 + N * (N - 1) / 2, cu = P * N;
      acc.add(P, N);
      bal[id(side, lk.second)] += cb;
      unb[id(side, lk.second)] += cu;
      own[lk.first].first += cb;
      own[lk.first].second += cu;
    }
    for (auto& [local, s] : own) {
      const int32_t ow = owners ? owners[local] : owner;
      bal[id(side, (uint32_t)ow)] += s.first;
      unb[id(side, (uint32_t)ow)] += s.second;
    }
    return 0;
  };
  for (auto* list : {&plan.direct_items, &plan.hash_items, &plan.reverse_items})
    for (const Item& it : *list) {
      const int32_t lim = list == &plan.reverse_items ? (int32_t)kReverseMaxSegs : INT32_MAX;
      if (list == &plan.direct_items &&
          it.key_hi - it.key_lo > ((it.flags & kItemPacked) ? kPVWindowPacked : kPVWindow))
        return -124;
      if (it.flags & kItemPacked) {  // packed counters only where no key can reach 2^16
        const HostSide& S = g.side[it.side];
        const int32_t T = plan.T[it.side];
        const int64_t deg_T = T < S.n ? static_cast<int64_t>(S.off[T + 1] - S.off[T]) : 0;
        if (!pv_packed(it.seg_count, (it.flags & kItemHubPairs) != 0, deg_T)) return -126;
      }
      if ((it.flags & kItemHubPairs) && list != &plan.direct_items) return -132;  // hub items are direct or small
      if ((rc = run(it.side, plan.segs.data(), plan.seg_mid.data(), plan.seg_edge.data(), it.seg_begin,
                    it.seg_count, it.key_lo, it.key_hi, false, nullptr, it.owner, lim,
                    (it.flags & kItemHubPairs) != 0)))
        return rc;
    }
  for (const Item& grp : plan.small_groups) {
    const bool hub = (grp.flags & kItemHubPairs) != 0;
    if (hub && grp.key_hi != 1) return -133;  // a hub item is alone in its group
    if ((rc = run(grp.side, plan.small_segs.data(), plan.small_seg_mid.data(), plan.small_seg_edge.data(),
                  grp.seg_begin, grp.seg_count, 0, INT32_MAX - 1, true, plan.small_owner.data() + grp.acc_slot, 0,
                  65535, hub)))
      return rc;
  }
  out[0] = acc.bal;
  out[1] = acc.unb;
  out[2] = acc.tot;
  out[3] = g.wedges_vp;
  out[4] = plan.T[0];
  return 0;
}

// The planner's size guard (runs addressed by 32-bit indices, int32 item,
// reduce and accumulator-slot counts), called with sizes chosen by the test.
extern "C" int plan_check_sizes(uint64_t runs, uint64_t items, uint64_t reduces, uint64_t acc_slots) {
  PlanSizes z;
  z.runs = runs;
  z.items = items;
  z.reduces = reduces;
  z.acc_slots = acc_slots;
  std::string err;
  return check_plan_sizes(z, err);
}
