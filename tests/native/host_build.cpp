// Test harness (CPU only): the library's host graph (the priority-ordered
// CSR pair of Definition 3 with per-entry reverse positions, cut, W_VP and
// the U-entry record map) built in plain loops on the host, so the planner
// can be checked on the CPU.  The library builds the same layout on the
// device (build.hip).
#include <algorithm>
#include <cstring>
#include <numeric>

#include "host_build.h"

namespace dbbc {
namespace {

// Stable counting sort of idx[] by key(idx) in [0, nkeys); writes out[].
template <class Key>
void counting_sort(const std::vector<uint32_t>& idx, std::vector<uint32_t>& out, int64_t nkeys,
                   Key key) {
  std::vector<uint32_t> cnt(static_cast<size_t>(nkeys) + 1, 0);
  for (uint32_t i : idx) cnt[key(i) + 1]++;
  for (int64_t k = 0; k < nkeys; ++k) cnt[k + 1] += cnt[k];
  out.resize(idx.size());
  for (uint32_t i : idx) out[cnt[key(i)]++] = i;
}

// Order of one side by (degree desc, id desc): a counting sort over degrees.
void priority_order(const std::vector<int64_t>& deg, int64_t max_deg, std::vector<int32_t>& order) {
  const int64_t n = static_cast<int64_t>(deg.size());
  std::vector<int64_t> start(static_cast<size_t>(max_deg) + 2, 0);
  for (int64_t x = 0; x < n; ++x) start[max_deg - deg[x] + 1]++;
  for (int64_t k = 0; k <= max_deg; ++k) start[k + 1] += start[k];
  order.assign(static_cast<size_t>(n), 0);
  for (int64_t x = n - 1; x >= 0; --x) order[start[max_deg - deg[x]]++] = static_cast<int32_t>(x);
}

}  // namespace

int build_host_graph(int32_t n_u, int32_t n_v, int64_t m, const int32_t* u, const int32_t* v,
                     const int8_t* sign, uint32_t flags, HostGraph& g, std::string& err) {
  if (n_u <= 0 || n_v <= 0 || m < 0) {
    err = "n_u and n_v must be positive and m non-negative";
    return DBBC_E_INVALID_ARG;
  }
  if (static_cast<int64_t>(n_u) + n_v >= (int64_t(1) << 30) || m >= (int64_t(1) << 31) - 1) {
    err = "graph too large: need n_u + n_v < 2^30 and m < 2^31 - 1";
    return DBBC_E_TOO_LARGE;
  }
  if (m > 0 && (!u || !v || !sign)) {
    err = "edge arrays must not be NULL";
    return DBBC_E_INVALID_ARG;
  }
  for (int64_t i = 0; i < m; ++i) {
    if (u[i] < 0 || u[i] >= n_u || v[i] < 0 || v[i] >= n_v) {
      err = "edge " + std::to_string(i) + " has a vertex id out of range";
      return DBBC_E_ID_RANGE;
    }
    if (sign[i] != 1 && sign[i] != -1) {
      err = "edge " + std::to_string(i) + " has sign " + std::to_string(int(sign[i])) +
            " (must be +1 or -1)";
      return DBBC_E_SIGN;
    }
  }

  // Last-wins dedup: sort input positions by (u, v), stable, keep the last
  // record of each run of equal pairs.
  std::vector<uint32_t> idx(static_cast<size_t>(m)), tmp;
  std::iota(idx.begin(), idx.end(), 0u);
  counting_sort(idx, tmp, n_v, [&](uint32_t i) { return v[i]; });
  counting_sort(tmp, idx, n_u, [&](uint32_t i) { return u[i]; });
  std::vector<uint32_t> keep;
  keep.reserve(static_cast<size_t>(m));
  int64_t dups = 0;
  for (int64_t k = 0; k < m; ++k) {
    uint32_t i = idx[k];
    if (k + 1 < m && u[idx[k + 1]] == u[i] && v[idx[k + 1]] == v[i]) {
      ++dups;
      continue;
    }
    keep.push_back(i);
  }
  if (dups && (flags & DBBC_DUP_REJECT)) {
    err = std::to_string(dups) + " duplicate (u, v) records";
    return DBBC_E_DUPLICATE;
  }
  const int64_t me = static_cast<int64_t>(keep.size());
  g.n_u = n_u;
  g.n_v = n_v;
  g.m = me;
  g.m_in = m;
  g.dups_dropped = dups;

  // Degrees and the priority order of Definition 3 within each side.
  std::vector<int64_t> deg_u(n_u, 0), deg_v(n_v, 0);
  for (uint32_t i : keep) {
    deg_u[u[i]]++;
    deg_v[v[i]]++;
  }
  int64_t md_u = deg_u.empty() ? 0 : *std::max_element(deg_u.begin(), deg_u.end());
  int64_t md_v = deg_v.empty() ? 0 : *std::max_element(deg_v.begin(), deg_v.end());
  std::vector<int32_t> ord_u, ord_v;
  priority_order(deg_u, md_u, ord_u);
  priority_order(deg_v, md_v, ord_v);
  std::vector<int32_t> sr_u(n_u), sr_v(n_v);
  for (int32_t r = 0; r < n_u; ++r) sr_u[ord_u[r]] = r;
  for (int32_t r = 0; r < n_v; ++r) sr_v[ord_v[r]] = r;

  HostSide& U = g.side[0];
  HostSide& V = g.side[1];
  U.n = n_u;
  V.n = n_v;
  U.max_deg = md_u;
  V.max_deg = md_v;
  U.orig = ord_u;
  V.orig = ord_v;

  // Merge the two sides into one priority order (ids: u for U, n_u + v for V).
  U.grank.assign(n_u, 0);
  V.grank.assign(n_v, 0);
  {
    int32_t a = 0, b = 0, r = 0;
    while (a < n_u || b < n_v) {
      bool take_u;
      if (a == n_u) {
        take_u = false;
      } else if (b == n_v) {
        take_u = true;
      } else {
        int64_t du = deg_u[ord_u[a]], dv = deg_v[ord_v[b]];
        int64_t iu = ord_u[a], iv = static_cast<int64_t>(n_u) + ord_v[b];
        take_u = du != dv ? du > dv : iu > iv;
      }
      if (take_u)
        U.grank[a++] = r++;
      else
        V.grank[b++] = r++;
    }
  }

  // CSR of U in rank space, rows sorted by the V neighbour's rank: sort the
  // kept records by (sr_v) then stably by (sr_u).
  counting_sort(keep, tmp, n_v, [&](uint32_t i) { return sr_v[v[i]]; });
  std::vector<uint32_t> by_u;
  counting_sort(tmp, by_u, n_u, [&](uint32_t i) { return sr_u[u[i]]; });
  std::vector<uint32_t> by_v;
  counting_sort(by_u, by_v, n_v, [&](uint32_t i) { return sr_v[v[i]]; });
  keep.clear();
  keep.shrink_to_fit();
  tmp.clear();
  tmp.shrink_to_fit();

  auto fill_side = [&](HostSide& S, const std::vector<uint32_t>& order, bool is_u) {
    S.off.assign(static_cast<size_t>(S.n) + 1, 0);
    S.adj.resize(static_cast<size_t>(me));
    for (int64_t k = 0; k < me; ++k) {
      uint32_t i = order[k];
      int32_t row = is_u ? sr_u[u[i]] : sr_v[v[i]];
      int32_t nbr = is_u ? sr_v[v[i]] : sr_u[u[i]];
      S.off[row + 1]++;
      S.adj[k] = (static_cast<uint32_t>(nbr) << 1) | (sign[i] < 0 ? 1u : 0u);
    }
    for (int32_t r = 0; r < S.n; ++r) S.off[r + 1] += S.off[r];
  };
  fill_side(U, by_u, true);
  fill_side(V, by_v, false);

  // rev: for the entry of edge (x, y) in row x, the index of x inside row y.
  // Position of each input record in the two CSRs, then a scatter.
  {
    std::vector<uint32_t> pos_v(static_cast<size_t>(m), 0);
    for (int64_t k = 0; k < me; ++k) pos_v[by_v[k]] = static_cast<uint32_t>(k);
    U.rev.resize(static_cast<size_t>(me));
    V.rev.resize(static_cast<size_t>(me));
    for (int64_t k = 0; k < me; ++k) {
      uint32_t i = by_u[k];
      uint32_t pv = pos_v[i];
      int32_t ru = sr_u[u[i]], rv = sr_v[v[i]];
      U.rev[k] = static_cast<int32_t>(pv - V.off[rv]);
      V.rev[pv] = static_cast<int32_t>(static_cast<uint32_t>(k) - U.off[ru]);
    }
  }
  // the input record of every U entry (per-edge outputs are by record)
  U.rec = std::move(by_u);

  // cut: neighbours of higher priority form a prefix of each row.
  auto fill_cut = [&](HostSide& S, const HostSide& O) {
    S.cut.assign(S.n, 0);
    for (int32_t x = 0; x < S.n; ++x) {
      const uint32_t* b = S.adj.data() + S.off[x];
      const uint32_t* e = S.adj.data() + S.off[x + 1];
      const int32_t gx = S.grank[x];
      const uint32_t* p = std::partition_point(
          b, e, [&](uint32_t w) { return O.grank[w >> 1] < gx; });
      S.cut[x] = static_cast<int32_t>(p - b);
    }
  };
  fill_cut(U, V);
  fill_cut(V, U);

  // W_VP in closed form: a down-edge (x, y) (y of lower priority) walks the
  // entries of row y after x, all of lower priority than x.
  int64_t w = 0, active = 0;
  for (int s = 0; s < 2; ++s) {
    const HostSide& S = g.side[s];
    const HostSide& O = g.side[1 - s];
    for (int32_t x = 0; x < S.n; ++x) {
      int64_t wx = 0;
      for (uint32_t e = S.off[x] + S.cut[x]; e < S.off[x + 1]; ++e) {
        uint32_t y = S.adj[e] >> 1;
        wx += static_cast<int64_t>(O.off[y + 1] - O.off[y]) - 1 - S.rev[e];
      }
      w += wx;
      active += wx > 0;
    }
  }
  g.wedges_vp = w;
  g.pivots_active = active;
  return DBBC_OK;
}

}  // namespace dbbc
