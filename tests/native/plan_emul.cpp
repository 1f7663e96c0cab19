// Test harness (CPU only): builds the library's host graph and counting plan
// and walks every planned item the way the kernels do, in plain loops, so the
// split of the vertex-priority wedges into items can be checked on the CPU.
#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../paper_2609_21848_amd/csrc/internal.h"

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
    if ((rc = run(it, kReverseMaxSegs))) return rc;
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
