// Plans built on the device: the work split of make_plan (plan.cpp), for a
// count or for the per-vertex pass, computed from the device CSR with
// kernels, scans and sorts (the binning step of Algorithm 1 that sizes each
// pivot's work, Eq. 1, done per CSR entry instead of per pivot on the host).
//
// Per side s, every CSR entry e of row x, with mid y = adj[e] >> 1, yields at
// most one run of each kind:
//   F  forward: pivot x, the entries of row y below x in priority (from
//      rev[e] + 1 on), for e past x's higher-priority prefix cut[x]; a
//      window pivot (x < L) stops at the window, a hub pivot (x < T) with a
//      hub mid (y < T') starts past the dense block;
//   R  reverse (x >= L): the prefix of row y below both the reverse window
//      R and y's own higher-priority prefix cut[y];
//   M  reverse-mid (x >= L, R < L): the part of that prefix in [R, L);
//   H  per-vertex plans, hub pivots (x < T) through non-hub mids (y >= T'):
//      the part of the forward run below T (the hub pairs' sparse wedges,
//      tallied apart and completed by the dense block).
// Each (row, kind) is one candidate item.  Exclusive scans of the run flags
// and lengths over the entries give every candidate's run count and work as
// a difference of two scan values, and every run's place in its item.  The
// candidates are classified as make_plan classifies its items (skipped,
// small, hash, direct, reverse); one scan of the candidates' list counts
// places every item in its list and every run in segs or small_segs.
//
// Per-vertex plans also record every run's mid (flagged kMidWide where its
// credits may need two words) and first-edge position, and the owner of
// every small item; they have no multi-part items (a direct item is cut into
// key windows that share its runs) and reverse endpoints with more than
// kReverseMaxSegs runs become direct items.
// Where the result differs from make_plan's, both are valid plans of the
// same wedges (the counts are the same):
//   - items and runs are listed in candidate order (row, then kind);
//   - small items are grouped greedily within chunks of kGroupChunk items;
//   - a split direct item starts a new part at every run that holds a
//     multiple of part_work in its wedge range (and every kPartMaxRuns
//     runs), so a part has at most part_work wedges plus its first run; the
//     hub pivots' tally items are cut the same way at kHubTallyPartWork.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include <algorithm>
#include <climits>
#include <string>

#include "kernels.h"
#include "plan_dev.h"

namespace dbbc {
namespace {

constexpr int kThreads = 256;

enum : int { kF = 0, kR = 1, kM = 2, kH = 3 };  // run kinds (kH: per-vertex plans only)
enum : int { kSkip = 0, kSmallC = 1, kHashC = 2, kDirectC = 3, kRevC = 4, kHubC = 5 };  // item classes

constexpr uint32_t kPartMaxRuns = 65535;  // runs of a direct part (16-bit per-part counters)
constexpr int kGroupChunk = 256;          // small items grouped per chunk

struct Fail {
  int status;
  std::string msg;
};

#define PD_TRY(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw Fail{e_ == hipErrorOutOfMemory ? DBBC_E_OOM : DBBC_E_DEVICE,                \
                 std::string(#expr) + ": " + hipGetErrorString(e_)};                    \
  } while (0)

int grid_for(int64_t n) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 1 << 16)));
}

#define GRID_STRIDE(i, n)                                                                    \
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); \
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)

// One side's arrays as the planning kernels see them.
struct PSide {
  const uint32_t* off;   // n + 1
  const uint32_t* adj;   // m
  const int32_t* rev;    // m
  const int32_t* cut;    // n
  const uint32_t* ooff;  // the other side's offsets, entries and prefixes
  const uint32_t* oadj;
  const int32_t* ocut;
  const int32_t* splitL;  // per row y of the other side: entries of rank below L, R, T
  const int32_t* splitR;
  const int32_t* splitT;
  const uint32_t* row;    // row of every entry
  uint32_t* len[4];       // run length per kind and entry (m + 1, the last 0)
  uint32_t* cnt[4];       // exclusive scans of len > 0
  unsigned long long* wsum[4];  // exclusive scans of len
  uint32_t* bnd[3];       // kinds F, M (split direct items) and H: exclusive scans of part-start flags
  int32_t* rmax;          // per row: largest key of its reverse runs
  int32_t n, no, L, R, T, TO;
  int32_t nk;             // run kinds (candidates per row): 3, or 4 in per-vertex plans
  bool pv;                // a per-vertex plan
  bool wide_all;          // per-vertex plans: flag every run kMidWide
  unsigned long long max_deg;  // largest degree of the side (the wide-credit bound)
  int64_t m;
  uint32_t side;
  int64_t cand0;          // index of the side's first candidate (nk per row)
  uint32_t small_work;
  unsigned long long part_work;
};

struct PSides {
  PSide s[2];
};

struct Run {
  uint32_t start, len;
};

// The run of kind k at entry e of row x.
__device__ Run run_at(const PSide& P, int k, int32_t x, uint32_t e) {
  const uint32_t y = P.adj[e] >> 1;
  const uint32_t yb = P.ooff[y];
  if (k == kF) {
    if (e < P.off[x] + static_cast<uint32_t>(P.cut[x])) return Run{0, 0};
    uint32_t start = yb + static_cast<uint32_t>(P.rev[e]) + 1;
    uint32_t end;
    if (x < P.L) {
      end = yb + static_cast<uint32_t>(P.splitL[y]);
      if (x < P.T && static_cast<int32_t>(y) < P.TO) start = max(start, yb + static_cast<uint32_t>(P.splitT[y]));
    } else {
      end = P.ooff[y + 1];
    }
    return Run{start, end > start ? end - start : 0u};
  }
  if (k == kH) {  // hub pivot x through a non-hub mid: the run's keys below T
    if (x >= P.T || static_cast<int32_t>(y) < P.TO || e < P.off[x] + static_cast<uint32_t>(P.cut[x]))
      return Run{0, 0};
    const uint32_t start = yb + static_cast<uint32_t>(P.rev[e]) + 1;
    const uint32_t end = yb + static_cast<uint32_t>(P.splitT[y]);
    return Run{start, end > start ? end - start : 0u};
  }
  if (x < P.L) return Run{0, 0};
  if (k == kR) {
    const int32_t l = min(P.splitR[y], P.ocut[y]);
    return Run{yb, l > 0 ? static_cast<uint32_t>(l) : 0u};
  }
  if (P.R == P.L) return Run{0, 0};
  const int32_t end = min(P.splitL[y], P.ocut[y]);
  const int32_t lo = P.splitR[y];
  return Run{yb + static_cast<uint32_t>(lo), end > lo ? static_cast<uint32_t>(end - lo) : 0u};
}

struct Cand {
  int cls;
  uint32_t nseg;
  unsigned long long work;
  uint32_t nparts;  // reverse: parts (0 = a single item); direct: parts when split
  bool split;       // a direct item cut into parts
  int32_t key_lo, key_hi;
  uint32_t flags;
};

// Classify candidate (x, k) as make_plan's place() does.  With parts set,
// a split direct item's part count is read from the part-start scans.
template <bool kParts>
__device__ Cand classify(const PSide& P, int32_t x, int k) {
  Cand c{};
  c.cls = kSkip;
  if (k == kH) {  // a hub pivot's tally item (per-vertex plans): kept with one run
    if (x >= P.T) return c;
    const uint32_t b = P.off[x], e = P.off[x + 1];
    c.nseg = P.cnt[kH][e] - P.cnt[kH][b];
    if (c.nseg == 0) return c;
    c.work = P.wsum[kH][e] - P.wsum[kH][b];
    c.cls = kHubC;
    c.key_lo = x + 1;
    c.key_hi = P.T;
    c.flags = kItemHubPairs;
    if (kParts) c.nparts = P.bnd[2][e] - P.bnd[2][b];
    return c;
  }
  if (k != kF && (x < P.L || (k == kM && P.R == P.L))) return c;
  const uint32_t b = P.off[x], e = P.off[x + 1];
  c.nseg = P.cnt[k][e] - P.cnt[k][b];
  c.work = P.wsum[k][e] - P.wsum[k][b];
  const bool hub = k == kF && x < P.T;
  c.flags = hub ? kItemHubPairs : 0u;
  // one run: every pair of the item has at most one wedge, and adds nothing
  // unless the dense block completes the pair
  if (c.nseg == 0 || (c.nseg < 2 && !hub)) return c;
  const bool small = c.work <= P.small_work;
  if (k == kF) {
    c.key_lo = x + 1;
    c.key_hi = x < P.L ? P.L : P.n;
    c.cls = small ? kSmallC : (x < P.L ? kDirectC : kHashC);
  } else if (k == kR) {
    // rows are sorted by rank: the keys stop at the largest run end
    c.key_lo = 0;
    c.key_hi = min(P.R, max(P.rmax[x], 0) + 1);
    if (P.pv) {  // no parts: one reverse item, or a direct item past kReverseMaxSegs runs
      c.cls = c.nseg > kReverseMaxSegs ? kDirectC : kRevC;
      return c;
    }
    c.cls = kRevC;
    c.nparts = c.nseg <= kReverseCountMaxSegs ? 0u : (c.nseg + kReverseCountMaxSegs - 1) / kReverseCountMaxSegs;
  } else {
    c.key_lo = P.R;
    c.key_hi = P.L;
    c.cls = small ? kSmallC : kDirectC;
  }
  if (c.cls == kDirectC && !P.pv && (c.work > P.part_work || c.nseg > kPartMaxRuns)) {
    c.split = true;
    if (kParts) {
      const uint32_t* bs = P.bnd[k == kF ? 0 : 1];
      c.nparts = bs[e] - bs[b];
    }
  }
  return c;
}

// ---- kernels ------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  GRID_STRIDE(i, n) p[i] = v;
}

__global__ void k_iota(uint32_t* p, int64_t n) {
  GRID_STRIDE(i, n) p[i] = static_cast<uint32_t>(i);
}

// rows[off[x]] = x for every non-empty row (the rest is zero); an inclusive
// max-scan then gives every entry its row.
__global__ void k_row_marks(const uint32_t* off, int32_t n, uint32_t* rows) {
  GRID_STRIDE(x, n) {
    if (off[x + 1] > off[x]) rows[off[x]] = static_cast<uint32_t>(x);
  }
}

// Per row y of the other side: entries of rank below L, R and T (rows are
// sorted by rank; an entry is (rank << 1) | negative).
__global__ void k_splits(const uint32_t* ooff, const uint32_t* oadj, int32_t no, int32_t L, int32_t R, int32_t T,
                         int32_t* sL, int32_t* sR, int32_t* sT) {
  GRID_STRIDE(y, no) {
    const uint32_t b = ooff[y], e = ooff[y + 1];
    auto below = [&](int32_t k) {
      const uint32_t key = static_cast<uint32_t>(k) << 1;
      uint32_t lo = b, hi = e;
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (oadj[mid] < key)
          lo = mid + 1;
        else
          hi = mid;
      }
      return static_cast<int32_t>(lo - b);
    };
    sL[y] = below(L);
    sR[y] = below(R);
    sT[y] = below(T);
  }
}

// Run lengths of every entry, and each row's largest reverse-run key.
__global__ void k_run_lengths(PSide P) {
  GRID_STRIDE(e64, P.m) {
    const uint32_t e = static_cast<uint32_t>(e64);
    const int32_t x = static_cast<int32_t>(P.row[e]);
    for (int k = 0; k < P.nk; ++k) {
      const Run r = run_at(P, k, x, e);
      P.len[k][e] = r.len;
      if (k == kR && r.len > 0) atomicMax(&P.rmax[x], static_cast<int32_t>(P.oadj[r.start + r.len - 1] >> 1));
    }
  }
}

// Part-start flags of the runs of split direct items (kinds F and M) and of
// the hub pivots' tally items (kind H): the first run, every kPartMaxRuns-th
// run, and every run whose wedge range [pex, pex + len) of the item holds a
// multiple of the part budget (part_work, or kHubTallyPartWork).
__global__ void k_part_flags(PSide P, int k, uint32_t* flag) {
  GRID_STRIDE(e64, P.m) {
    const uint32_t e = static_cast<uint32_t>(e64);
    const uint32_t len = P.len[k][e];
    uint32_t f = 0;
    if (len > 0) {
      const int32_t x = static_cast<int32_t>(P.row[e]);
      const Cand c = classify<false>(P, x, k);
      if (c.split || c.cls == kHubC) {
        const uint32_t b = P.off[x];
        const uint32_t j = P.cnt[k][e] - P.cnt[k][b];
        const unsigned long long pex = P.wsum[k][e] - P.wsum[k][b];
        const unsigned long long pw =
            k == kH ? static_cast<unsigned long long>(kHubTallyPartWork) : P.part_work;
        f = (j % kPartMaxRuns == 0 || (pex + len - 1) / pw != (pex - 1) / pw) ? 1u : 0u;
      }
    }
    flag[e] = f;
  }
}

// What one candidate adds to each list (scanned into list positions).
struct PlanCount {
  unsigned long long big_runs;    // runs in segs (hash, direct and reverse items)
  unsigned long long small_runs;  // runs in small_segs
  unsigned long long hub_runs;    // runs in hub_segs (per-vertex plans)
  uint32_t small_items, hash, direct, direct_parts, direct_split, rev, rev_reduces, rev_acc, hub_parts, pad;
};

struct PlanCountSum {
  __host__ __device__ PlanCount operator()(const PlanCount& a, const PlanCount& b) const {
    PlanCount r;
    r.big_runs = a.big_runs + b.big_runs;
    r.small_runs = a.small_runs + b.small_runs;
    r.hub_runs = a.hub_runs + b.hub_runs;
    r.hub_parts = a.hub_parts + b.hub_parts;
    r.pad = 0;
    r.small_items = a.small_items + b.small_items;
    r.hash = a.hash + b.hash;
    r.direct = a.direct + b.direct;
    r.direct_parts = a.direct_parts + b.direct_parts;
    r.direct_split = a.direct_split + b.direct_split;
    r.rev = a.rev + b.rev;
    r.rev_reduces = a.rev_reduces + b.rev_reduces;
    r.rev_acc = a.rev_acc + b.rev_acc;
    return r;
  }
};

// Plan statistics: wedges and runs per kernel (direct, small, hash,
// reverse), then the sparse and the skipped wedges.
enum : int { kStWedges = 0, kStRuns = 4, kStSparse = 8, kStSkipped = 9, kStWords = 10 };

__device__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Per-vertex plans: the key windows of a direct item (kPVWindowPacked keys
// with packed counters, see pv_packed; else kPVWindow keys).
__device__ bool pv_item_packed(const PSide& P, uint32_t nseg, uint32_t flags) {
  const int64_t deg_T = P.T < P.n ? static_cast<int64_t>(P.off[P.T + 1] - P.off[P.T]) : 0;
  return pv_packed(nseg, (flags & kItemHubPairs) != 0, deg_T);
}
__device__ uint32_t pv_window_count(int32_t key_lo, int32_t key_hi, bool packed) {
  const uint32_t win = static_cast<uint32_t>(packed ? kPVWindowPacked : kPVWindow);
  return (static_cast<uint32_t>(key_hi - key_lo) + win - 1) / win;
}

// Each candidate's list counts; the statistics are summed per thread over
// its candidates, then per wavefront, then once per wavefront into stats.
__global__ void k_count(PSide P, PlanCount* counts, unsigned long long* stats) {
  const int64_t nc = P.nk * static_cast<int64_t>(P.n);
  unsigned long long w[4] = {0, 0, 0, 0}, r[4] = {0, 0, 0, 0}, sparse = 0, skipped = 0;
  GRID_STRIDE(i, nc) {
    const int32_t x = static_cast<int32_t>(i / P.nk);
    const int k = static_cast<int>(i % P.nk);
    const Cand c = classify<true>(P, x, k);
    PlanCount q{};
    int slot = -1;
    uint32_t mult = 1;
    switch (c.cls) {
      case kSmallC:
        q.small_runs = c.nseg;
        q.small_items = 1;
        slot = 1;
        break;
      case kHashC:
        q.big_runs = c.nseg;
        q.hash = 1;
        slot = 2;
        break;
      case kDirectC:
        q.big_runs = c.nseg;
        q.direct = 1;
        if (c.split) {
          q.direct_parts = c.nparts;
          q.direct_split = 1;
        }
        slot = 0;
        if (P.pv)  // the windows share the runs
          mult = pv_window_count(c.key_lo, c.key_hi, pv_item_packed(P, c.nseg, c.flags));
        break;
      case kRevC:
        q.big_runs = c.nseg;
        if (c.nparts) {
          q.rev = c.nparts;
          q.rev_reduces = 1;
          q.rev_acc = c.nparts;
        } else {
          q.rev = 1;
        }
        slot = 3;
        break;
      case kHubC:  // the dense block's sparse wedges: not in the kernels' statistics
        q.hub_runs = c.nseg;
        q.hub_parts = c.nparts;
        break;
      default:
        skipped += c.work;
        break;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      w[j] += j == slot ? c.work * mult : 0ull;
      r[j] += j == slot ? static_cast<unsigned long long>(c.nseg) * mult : 0ull;
    }
    if (slot >= 0) sparse += c.work;
    counts[P.cand0 + i] = q;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    w[j] = wave_sum(w[j]);
    r[j] = wave_sum(r[j]);
  }
  sparse = wave_sum(sparse);
  skipped = wave_sum(skipped);
  if ((threadIdx.x & 63) == 0) {
    for (int j = 0; j < 4; ++j) {
      if (w[j]) atomicAdd(&stats[kStWedges + j], w[j]);
      if (r[j]) atomicAdd(&stats[kStRuns + j], r[j]);
    }
    if (sparse) atomicAdd(&stats[kStSparse], sparse);
    if (skipped) atomicAdd(&stats[kStSkipped], skipped);
  }
}

uint32_t sat32(unsigned long long w) { return w > 0xffffffffull ? 0xffffffffu : static_cast<uint32_t>(w); }
__device__ uint32_t dsat32(unsigned long long w) { return w > 0xffffffffull ? 0xffffffffu : static_cast<uint32_t>(w); }

// A direct item before ordering: its row, kind and parts.
struct DirectMeta {
  int32_t x;
  uint32_t kind_side;   // kind | side << 2
  uint32_t nparts;      // 0: one item
  uint32_t part_base;   // first of its part starts
};

struct ItemOut {
  Item* small;         // small items (grouped later)
  int32_t* small_owner;  // per-vertex plans: the owner of every small item
  Item* hash;          // hash items, unordered
  unsigned long long* hash_key;
  Item* direct;        // direct items, unordered
  unsigned long long* direct_key;
  DirectMeta* direct_meta;
  Item* rev;           // reverse items (final)
  Reduce* reduces;     // reverse reduces first
};

__global__ void k_items(PSide P, const PlanCount* pos, ItemOut o) {
  const int64_t nc = P.nk * static_cast<int64_t>(P.n);
  GRID_STRIDE(i, nc) {
    const int32_t x = static_cast<int32_t>(i / P.nk);
    const int k = static_cast<int>(i % P.nk);
    const Cand c = classify<true>(P, x, k);
    if (c.cls == kSkip || c.cls == kHubC) continue;  // hub tally items: k_hub_parts
    const PlanCount q = pos[P.cand0 + i];
    Item it{};
    it.seg_count = c.nseg;
    it.owner = x;
    it.key_lo = c.key_lo;
    it.key_hi = c.key_hi;
    it.acc_slot = -1;
    it.flags = c.flags;
    it.side = P.side;
    it.work = dsat32(c.work);
    it.graph = 0;
    if (c.cls == kSmallC) {
      it.seg_begin = static_cast<uint32_t>(q.small_runs);
      o.small[q.small_items] = it;
      if (P.pv) o.small_owner[q.small_items] = x;
      continue;
    }
    it.seg_begin = static_cast<uint32_t>(q.big_runs);
    if (c.cls == kHashC) {
      o.hash[q.hash] = it;
      o.hash_key[q.hash] = c.work;
    } else if (c.cls == kDirectC) {
      o.direct[q.direct] = it;
      // per-vertex plans: side 0 first, then heaviest first (ascending keys);
      // count plans: heaviest first (descending keys)
      o.direct_key[q.direct] =
          P.pv ? (static_cast<unsigned long long>(P.side) << 48) | ((1ull << 48) - 1 - min(c.work, (1ull << 48) - 1))
               : c.work;
      o.direct_meta[q.direct] = DirectMeta{x, static_cast<uint32_t>(k) | (P.side << 2), c.split ? c.nparts : 0u,
                                           q.direct_parts};
    } else if (c.nparts == 0) {
      o.rev[q.rev] = it;
    } else {
      // parts of kReverseCountMaxSegs runs (their work is summed once the
      // runs are written), reduced into one accumulator slot each
      for (uint32_t p = 0; p < c.nparts; ++p) {
        Item part = it;
        part.seg_begin = it.seg_begin + p * kReverseCountMaxSegs;
        part.seg_count = min(kReverseCountMaxSegs, c.nseg - p * kReverseCountMaxSegs);
        part.flags |= kItemMultiPart;
        part.acc_slot = static_cast<int32_t>(q.rev_acc + p);
        part.work = 0;
        o.rev[q.rev + p] = part;
      }
      Reduce r{};
      r.acc_slot = static_cast<int32_t>(q.rev_acc);
      r.n_parts = static_cast<int32_t>(c.nparts);
      r.owner = x;
      r.key_lo = c.key_lo;
      r.key_hi = c.key_hi;
      r.flags = c.flags;
      r.side = P.side;
      r.graph = 0;
      o.reduces[q.rev_reduces] = r;
    }
  }
}

// Small items into groups of at most kSmallGroupWork wedges that one
// wavefront counts in one hash table: greedy in list order within each chunk
// of kGroupChunk items.  A group holds items of one side, at most
// min(kSmallMaxItems, 2^(32 - key_bits) - 1) of them (the group's hash key is
// (index in group << key_bits) | key), and an item whose hub-pair counts go
// to the dense path stays alone.  Pass 0 counts each chunk's groups; pass 1
// writes them and each item's index in its group.
template <int kPass>
__global__ void k_group(const Item* small, int64_t n_small, int32_t kb0, int32_t kb1, bool pv, uint32_t* chunk_groups,
                        Item* groups, uint32_t* local_of) {
  const int64_t n_chunks = (n_small + kGroupChunk - 1) / kGroupChunk;
  GRID_STRIDE(ch, n_chunks) {
    const int64_t i0 = ch * kGroupChunk, i1 = min(n_small, i0 + kGroupChunk);
    uint32_t g = kPass ? chunk_groups[ch] : 0u;
    Item grp{};
    bool open = false;
    uint32_t local = 0;
    for (int64_t i = i0; i < i1; ++i) {
      const Item it = small[i];
      const int32_t kb = it.side ? kb1 : kb0;
      const uint32_t max_items = min(kSmallMaxItems, (1u << (32 - kb)) - 1u);
      const bool hub = (it.flags & kItemHubPairs) != 0;
      if (open && (hub || (grp.flags & kItemHubPairs) || grp.side != it.side ||
                   grp.work + it.work > kSmallGroupWork || local >= max_items)) {
        if (kPass) {
          grp.key_hi = static_cast<int32_t>(local);
          groups[g] = grp;
        }
        ++g;
        open = false;
      }
      if (!open) {
        grp = Item{};
        grp.seg_begin = it.seg_begin;
        grp.owner = it.owner;
        grp.acc_slot = pv ? static_cast<int32_t>(i) : -1;  // per-vertex plans: owners are listed per item
        grp.flags = it.flags & kItemHubPairs;
        grp.side = it.side;
        local = 0;
        open = true;
      }
      if (kPass) local_of[i] = local;
      grp.seg_count += it.seg_count;
      grp.work += it.work;
      ++local;
    }
    if (open) {
      if (kPass) {
        grp.key_hi = static_cast<int32_t>(local);
        groups[g] = grp;
      }
      ++g;
    }
    if (!kPass) chunk_groups[ch] = g;
  }
}

struct RunOut {
  Segment* segs;
  Segment* small_segs;
  const uint32_t* local_of;  // small item -> index in its group
  uint32_t* part_start;      // split direct items: the entry of each part's first run
  // per-vertex plans
  uint32_t* seg_mid;         // each run's mid (| kMidWide), and its first edge's position
  uint32_t* seg_edge;
  uint32_t* small_seg_mid;
  uint32_t* small_seg_edge;
  Segment* hub_segs;         // the hub pivots' tally runs
  uint32_t* hub_part_start;  // ... the entry of each tally item's first run
  uint32_t* any_wide;        // set when some run is flagged kMidWide
};

// Every run into its item's place: segs[item's first + j] for the j-th run
// of the item, or small_segs tagged with the item's index in its group.
__global__ void k_runs(PSide P, const PlanCount* pos, RunOut o) {
  GRID_STRIDE(e64, P.m) {
    const uint32_t e = static_cast<uint32_t>(e64);
    const int32_t x = static_cast<int32_t>(P.row[e]);
    const uint32_t b = P.off[x];
    const uint32_t g = P.adj[e] & 1u;
    // per-vertex plans: the run's mid, flagged when its credits may reach
    // 2^32 (the mid's degree times the side's largest degree)
    uint32_t mid = 0;
    if (P.pv) {
      const uint32_t y = P.adj[e] >> 1;
      const unsigned long long dy = P.ooff[y + 1] - P.ooff[y];
      const bool wide = P.wide_all || dy * P.max_deg >= (1ull << 32);
      mid = y | (wide ? kMidWide : 0u);
    }
    for (int k = 0; k < P.nk; ++k) {
      if (P.len[k][e] == 0) continue;
      const Cand c = classify<true>(P, x, k);
      if (c.cls == kSkip) continue;
      const PlanCount q = pos[P.cand0 + P.nk * static_cast<int64_t>(x) + k];
      const Run r = run_at(P, k, x, e);
      const uint32_t j = P.cnt[k][e] - P.cnt[k][b];
      const uint32_t len_g = (r.len << 1) | g;
      if (c.cls == kHubC) {
        o.hub_segs[q.hub_runs + j] = Segment{r.start, len_g};
        const uint32_t* bs = P.bnd[2];
        if (bs[e + 1] != bs[e]) o.hub_part_start[q.hub_parts + (bs[e] - bs[b])] = e;
        continue;
      }
      if (P.pv && (mid & kMidWide) && *reinterpret_cast<volatile uint32_t*>(o.any_wide) == 0)
        atomicOr(o.any_wide, 1u);
      if (c.cls == kSmallC) {
        const size_t at = q.small_runs + j;
        o.small_segs[at] = Segment{r.start, (o.local_of[q.small_items] << 16) | len_g};
        if (P.pv) {
          o.small_seg_mid[at] = mid;
          o.small_seg_edge[at] = e;
        }
      } else {
        const size_t at = q.big_runs + j;
        o.segs[at] = Segment{r.start, len_g};
        if (P.pv) {
          o.seg_mid[at] = mid;
          o.seg_edge[at] = e;
        }
        if (c.split) {
          const uint32_t* bs = P.bnd[k == kF ? 0 : 1];
          if (bs[e + 1] != bs[e]) o.part_start[q.direct_parts + (bs[e] - bs[b])] = e;
        }
      }
    }
  }
}

// The work of every reverse part (at most kReverseCountMaxSegs runs).
__global__ void k_rev_part_work(Item* rev, int64_t n, const Segment* segs) {
  GRID_STRIDE(i, n) {
    Item& it = rev[i];
    if (!(it.flags & kItemMultiPart)) continue;
    uint32_t w = 0;
    for (uint32_t j = 0; j < it.seg_count; ++j) w += segs[it.seg_begin + j].len_g >> 1;
    it.work = w;
  }
}

// The hub pivots' tally items (per-vertex plans), one per part of each
// pivot's hub runs (parts start at the flagged runs).
__global__ void k_hub_parts(PSide P, const PlanCount* pos, const uint32_t* part_start, Item* out) {
  GRID_STRIDE(x64, P.T) {
    const int32_t x = static_cast<int32_t>(x64);
    const Cand c = classify<true>(P, x, kH);
    if (c.cls != kHubC) continue;
    const PlanCount q = pos[P.cand0 + P.nk * static_cast<int64_t>(x) + kH];
    const uint32_t b = P.off[x], end = P.off[x + 1];
    const uint32_t* cnt = P.cnt[kH];
    const unsigned long long* ws = P.wsum[kH];
    for (uint32_t p = 0; p < c.nparts; ++p) {
      const uint32_t es = part_start[q.hub_parts + p];
      const uint32_t en = p + 1 < c.nparts ? part_start[q.hub_parts + p + 1] : end;
      Item it{};
      it.seg_begin = static_cast<uint32_t>(q.hub_runs) + (cnt[es] - cnt[b]);
      it.seg_count = cnt[en] - cnt[es];
      it.owner = x;
      it.key_lo = c.key_lo;
      it.key_hi = c.key_hi;
      it.acc_slot = -1;
      it.flags = c.flags;
      it.side = P.side;
      it.work = dsat32(ws[en] - ws[es]);
      it.graph = 0;
      out[q.hub_parts + p] = it;
    }
  }
}

__global__ void k_gather_items(const Item* in, const uint32_t* perm, int64_t n, Item* out) {
  GRID_STRIDE(i, n) out[i] = in[perm[i]];
}

// Direct items in order of work (heaviest first): the parts of split items,
// then the single items.
struct DirectCount {
  uint32_t parts, single, split;
};

struct DirectCountSum {
  __host__ __device__ DirectCount operator()(const DirectCount& a, const DirectCount& b) const {
    return DirectCount{a.parts + b.parts, a.single + b.single, a.split + b.split};
  }
};

__global__ void k_direct_count(PSides S, const Item* direct, const DirectMeta* meta, const uint32_t* perm, int64_t n,
                               bool pv, DirectCount* out) {
  GRID_STRIDE(i, n) {
    if (pv) {  // every item as its key windows, in order
      const Item& it = direct[perm[i]];
      const bool packed = pv_item_packed(S.s[it.side], it.seg_count, it.flags);
      out[i] = DirectCount{pv_window_count(it.key_lo, it.key_hi, packed), 0u, 0u};
      continue;
    }
    const uint32_t np = meta[perm[i]].nparts;
    out[i] = DirectCount{np, np ? 0u : 1u, np ? 1u : 0u};
  }
}

struct DirectOut {
  Item* items;
  Reduce* reduces;
  uint32_t n_parts;     // parts of all split items (the singles follow)
  uint32_t acc0;        // first accumulator slot of the direct parts
  uint32_t red0;        // first reduce of the split direct items
  bool pv;              // per-vertex plan: key windows
};

__global__ void k_direct_write(PSides S, const Item* direct, const DirectMeta* meta, const uint32_t* perm,
                               const DirectCount* pos, int64_t n, const uint32_t* part_start, DirectOut o) {
  GRID_STRIDE(i, n) {
    const Item it = direct[perm[i]];
    const DirectMeta md = meta[perm[i]];
    const DirectCount q = pos[i];
    if (o.pv) {
      const bool packed = pv_item_packed(S.s[it.side], it.seg_count, it.flags);
      const uint32_t nw = pv_window_count(it.key_lo, it.key_hi, packed);
      const int32_t win = packed ? kPVWindowPacked : kPVWindow;
      for (uint32_t w = 0; w < nw; ++w) {
        Item iw = it;
        iw.key_lo = it.key_lo + static_cast<int32_t>(w) * win;
        iw.key_hi = min(it.key_hi, iw.key_lo + win);
        if (packed) iw.flags |= kItemPacked;
        o.items[q.parts + w] = iw;
      }
      continue;
    }
    if (md.nparts == 0) {
      o.items[o.n_parts + q.single] = it;
      continue;
    }
    const int k = static_cast<int>(md.kind_side & 3u);
    const PSide& P = S.s[md.kind_side >> 2];
    const uint32_t b = P.off[md.x], end = P.off[md.x + 1];
    const uint32_t* cnt = P.cnt[k];
    const unsigned long long* ws = P.wsum[k];
    for (uint32_t p = 0; p < md.nparts; ++p) {
      const uint32_t es = part_start[md.part_base + p];
      const uint32_t en = p + 1 < md.nparts ? part_start[md.part_base + p + 1] : end;
      Item part = it;
      part.seg_begin = it.seg_begin + (cnt[es] - cnt[b]);
      part.seg_count = cnt[en] - cnt[es];
      part.work = dsat32(ws[en] - ws[es]);
      part.flags |= kItemMultiPart;
      part.acc_slot = static_cast<int32_t>(o.acc0 + q.parts + p);
      o.items[q.parts + p] = part;
    }
    Reduce r{};
    r.acc_slot = static_cast<int32_t>(o.acc0 + q.parts);
    r.n_parts = static_cast<int32_t>(md.nparts);
    r.owner = it.owner;
    r.key_lo = it.key_lo;
    r.key_hi = it.key_hi;
    r.flags = it.flags;
    r.side = it.side;
    r.graph = 0;
    o.reduces[o.red0 + q.split] = r;
  }
}

// The dense block's signs: B[x][y] for x < T, y < T' (rows of K bytes), and
// Bm keeps those of mids above x in the global order.
// (pos, per-vertex plans: the CSR position of every hub edge)
__global__ void k_hub_signs(const uint32_t* off, const uint32_t* adj, const uint32_t* rows, const int32_t* grank_s,
                            const int32_t* grank_o, int32_t T, int32_t TO, int32_t K, int8_t* B, int8_t* Bm,
                            int32_t* pos) {
  const int64_t ne = off[T];
  GRID_STRIDE(e, ne) {
    const uint32_t x = rows[e];
    const uint32_t y = adj[e] >> 1;
    if (static_cast<int32_t>(y) >= TO) continue;
    const int8_t sg = (adj[e] & 1u) ? int8_t(-1) : int8_t(1);
    const size_t at = static_cast<size_t>(x) * K + y;
    B[at] = sg;
    if (grank_o[y] > grank_s[x]) Bm[at] = sg;
    if (pos) pos[at] = static_cast<int32_t>(e);
  }
}

// The transposes of B and Bm (K x T): Bt[y][x] = B[x][y].
__global__ void k_hub_transpose(const int8_t* B, const int8_t* Bm, int32_t T, int32_t K, int8_t* Bt, int8_t* Bmt) {
  const int64_t n = static_cast<int64_t>(T) * K;
  GRID_STRIDE(i, n) {  // i = y T + x: coalesced writes
    const int64_t y = i / T, x = i % T;
    Bt[i] = B[x * K + y];
    Bmt[i] = Bm[x * K + y];
  }
}

// Per column y: Zc[x][y] = #{w > x : B[w][y] != 0} and
// Zc'[w][y] = #{x < w : Bm[x][y] != 0} (T x K each), in chunks of
// kColChunk rows: the nonzeros of every (column, chunk), then per (column,
// chunk) the counts of the chunks below (above) it and a walk of its rows.
constexpr int32_t kColChunk = 128;

__global__ void k_hub_chunk_counts(const int8_t* B, const int8_t* Bm, int32_t T, int32_t K, uint32_t* cB,
                                   uint32_t* cBm) {
  const int32_t nch = (T + kColChunk - 1) / kColChunk;
  const int64_t n = static_cast<int64_t>(nch) * K;
  GRID_STRIDE(i, n) {  // i = c K + y: coalesced reads of row x
    const int32_t c = static_cast<int32_t>(i / K), y = static_cast<int32_t>(i % K);
    uint32_t nb = 0, nbm = 0;
    for (int32_t x = c * kColChunk; x < min(T, (c + 1) * kColChunk); ++x) {
      nb += B[static_cast<size_t>(x) * K + y] != 0;
      nbm += Bm[static_cast<size_t>(x) * K + y] != 0;
    }
    cB[i] = nb;
    cBm[i] = nbm;
  }
}

__global__ void k_hub_col_counts(const int8_t* B, const int8_t* Bm, int32_t T, int32_t K, const uint32_t* cB,
                                 const uint32_t* cBm, int32_t* Zc, int32_t* Zcp) {
  const int32_t nch = (T + kColChunk - 1) / kColChunk;
  const int64_t n = static_cast<int64_t>(nch) * K;
  GRID_STRIDE(i, n) {
    const int32_t c = static_cast<int32_t>(i / K), y = static_cast<int32_t>(i % K);
    int32_t below = 0, above = 0;
    for (int32_t d = c + 1; d < nch; ++d) below += static_cast<int32_t>(cB[static_cast<size_t>(d) * K + y]);
    for (int32_t d = 0; d < c; ++d) above += static_cast<int32_t>(cBm[static_cast<size_t>(d) * K + y]);
    const int32_t x0 = c * kColChunk, x1 = min(T, (c + 1) * kColChunk);
    for (int32_t x = x1 - 1; x >= x0; --x) {
      Zc[static_cast<size_t>(x) * K + y] = below;
      below += B[static_cast<size_t>(x) * K + y] != 0;
    }
    for (int32_t w = x0; w < x1; ++w) {
      Zcp[static_cast<size_t>(w) * K + y] = above;
      above += Bm[static_cast<size_t>(w) * K + y] != 0;
    }
  }
}

// U-CSR position k -> V-CSR position of the same edge: row y = adj_u[k] >> 1
// of V, at the entry's reverse position.
__global__ void k_edge_positions(const uint32_t* adj_u, const int32_t* rev_u, const uint32_t* off_v, int64_t m,
                                 uint32_t* out) {
  GRID_STRIDE(k, m) out[k] = off_v[adj_u[k] >> 1] + static_cast<uint32_t>(rev_u[k]);
}

// ---- host side ------------------------------------------------------------------

struct CubTmp {
  DevBuf buf;
  size_t bytes = 0;
  void* get(size_t need) {
    if (need > bytes) {
      PD_TRY(buf.alloc(need));
      bytes = need;
    }
    return buf.p;
  }
};

struct NonZero {
  __host__ __device__ uint32_t operator()(uint32_t v) const { return v ? 1u : 0u; }
};
struct Widen {
  __host__ __device__ unsigned long long operator()(uint32_t v) const { return v; }
};

void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kThreads), 0, st, p, n, v);
  PD_TRY(hipGetLastError());
}

template <class In, class Out>
void exclusive_sum(CubTmp& ct, In in, Out out, int64_t n, hipStream_t st) {
  size_t need = 0;
  PD_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, need, in, out, static_cast<int>(n), st));
  void* t = ct.get(need);
  PD_TRY(hipcub::DeviceScan::ExclusiveSum(t, need, in, out, static_cast<int>(n), st));
}

template <class T, class Op>
void exclusive_scan(CubTmp& ct, const T* in, T* out, Op op, int64_t n, hipStream_t st) {
  size_t need = 0;
  PD_TRY(hipcub::DeviceScan::ExclusiveScan(nullptr, need, in, out, op, T{}, static_cast<int>(n), st));
  void* t = ct.get(need);
  PD_TRY(hipcub::DeviceScan::ExclusiveScan(t, need, in, out, op, T{}, static_cast<int>(n), st));
}

void sort_desc(CubTmp& ct, const unsigned long long* kin, unsigned long long* kout, const uint32_t* vin,
               uint32_t* vout, int64_t n, hipStream_t st) {
  size_t need = 0;
  PD_TRY(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, need, kin, kout, vin, vout, static_cast<int>(n), 0,
                                                      64, st));
  void* t = ct.get(need);
  PD_TRY(hipcub::DeviceRadixSort::SortPairsDescending(t, need, kin, kout, vin, vout, static_cast<int>(n), 0, 64,
                                                      st));
}

void sort_asc(CubTmp& ct, const unsigned long long* kin, unsigned long long* kout, const uint32_t* vin,
              uint32_t* vout, int64_t n, hipStream_t st) {
  size_t need = 0;
  PD_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, need, kin, kout, vin, vout, static_cast<int>(n), 0, 64, st));
  void* t = ct.get(need);
  PD_TRY(hipcub::DeviceRadixSort::SortPairs(t, need, kin, kout, vin, vout, static_cast<int>(n), 0, 64, st));
}

template <class T>
T* alloc_n(DevBuf& b, int64_t n) {
  PD_TRY(b.alloc(static_cast<size_t>(std::max<int64_t>(n, 1)) * sizeof(T)));
  return b.as<T>();
}

// One side's scratch arrays.
struct SideBufs {
  DevBuf rows, rows_tmp, splitL, splitR, splitT, rmax, len[4], cnt[4], wsum[4], bnd[3];
};

void plan(const DevGraphView& g, const PlanParams& p, hipStream_t st, HostPlan& hp, DevPlanLists& out) {
  CubTmp ct;
  SideBufs sb[2];
  PSides S{};
  for (int s = 0; s < 2; ++s) {
    const int o = 1 - s;
    PSide& P = S.s[s];
    SideBufs& B = sb[s];
    const int64_t m = g.m;
    P.off = g.off[s];
    P.adj = g.adj[s];
    P.rev = g.rev[s];
    P.cut = g.cut[s];
    P.ooff = g.off[o];
    P.oadj = g.adj[o];
    P.ocut = g.cut[o];
    P.n = g.n[s];
    P.no = g.n[o];
    P.L = hp.L[s];
    P.R = hp.R[s];
    P.T = hp.T[s];
    P.TO = hp.T[o];
    P.m = m;
    P.side = static_cast<uint32_t>(s);
    P.pv = p.per_vertex;
    P.nk = P.pv ? 4 : 3;
    P.wide_all = p.wide_all;
    P.max_deg = static_cast<unsigned long long>(g.max_deg[s]);
    P.cand0 = s == 0 ? 0 : P.nk * static_cast<int64_t>(g.n[0]);
    P.small_work = static_cast<uint32_t>(p.small_work);
    P.part_work = static_cast<unsigned long long>(p.part_work);
    // the row of every entry
    uint32_t* rows = alloc_n<uint32_t>(B.rows, m);
    uint32_t* marks = alloc_n<uint32_t>(B.rows_tmp, m);
    fill_u32(marks, m, 0u, st);
    hipLaunchKernelGGL(k_row_marks, dim3(grid_for(P.n)), dim3(kThreads), 0, st, P.off, P.n, marks);
    PD_TRY(hipGetLastError());
    if (m > 0) {
      size_t need = 0;
      PD_TRY(hipcub::DeviceScan::InclusiveScan(nullptr, need, marks, rows, hipcub::Max(), static_cast<int>(m), st));
      void* t = ct.get(need);
      PD_TRY(hipcub::DeviceScan::InclusiveScan(t, need, marks, rows, hipcub::Max(), static_cast<int>(m), st));
    }
    B.rows_tmp.release();
    P.row = rows;
    int32_t* sL = alloc_n<int32_t>(B.splitL, P.no);
    int32_t* sR = alloc_n<int32_t>(B.splitR, P.no);
    int32_t* sT = alloc_n<int32_t>(B.splitT, P.no);
    hipLaunchKernelGGL(k_splits, dim3(grid_for(P.no)), dim3(kThreads), 0, st, P.ooff, P.oadj, P.no, P.L, P.R, P.T,
                       sL, sR, sT);
    PD_TRY(hipGetLastError());
    P.splitL = sL;
    P.splitR = sR;
    P.splitT = sT;
    P.rmax = alloc_n<int32_t>(B.rmax, P.n);
    fill_u32(reinterpret_cast<uint32_t*>(P.rmax), P.n, 0u, st);
    for (int k = 0; k < P.nk; ++k) {
      P.len[k] = alloc_n<uint32_t>(B.len[k], m + 1);
      fill_u32(P.len[k] + m, 1, 0u, st);
    }
    if (m > 0) {
      hipLaunchKernelGGL(k_run_lengths, dim3(grid_for(m)), dim3(kThreads), 0, st, P);
      PD_TRY(hipGetLastError());
    }
    for (int k = 0; k < P.nk; ++k) {
      P.cnt[k] = alloc_n<uint32_t>(B.cnt[k], m + 1);
      P.wsum[k] = alloc_n<unsigned long long>(B.wsum[k], m + 1);
      exclusive_sum(ct, rocprim::make_transform_iterator(P.len[k], NonZero{}), P.cnt[k], m + 1, st);
      exclusive_sum(ct, rocprim::make_transform_iterator(P.len[k], Widen{}), P.wsum[k], m + 1, st);
    }
    // part starts of split direct items (kinds F and M; count plans) or of
    // the hub pivots' tally items (kind H; per-vertex plans)
    DevBuf flags;
    uint32_t* fl = alloc_n<uint32_t>(flags, m + 1);
    for (int j = 0; j < 3; ++j) {
      if ((j == 2) != P.pv) continue;
      const int k = j == 0 ? kF : j == 1 ? kM : kH;
      fill_u32(fl + m, 1, 0u, st);
      if (m > 0) {
        hipLaunchKernelGGL(k_part_flags, dim3(grid_for(m)), dim3(kThreads), 0, st, P, k, fl);
        PD_TRY(hipGetLastError());
      }
      P.bnd[j] = alloc_n<uint32_t>(B.bnd[j], m + 1);
      exclusive_sum(ct, fl, P.bnd[j], m + 1, st);
    }
  }

  // candidates of both sides, one scan of their list counts
  const int nk = S.s[0].nk;
  const int64_t nc = nk * (static_cast<int64_t>(g.n[0]) + g.n[1]);
  DevBuf counts_b, pos_b, stats_b;
  PlanCount* counts = alloc_n<PlanCount>(counts_b, nc + 1);
  PlanCount* pos = alloc_n<PlanCount>(pos_b, nc + 1);
  unsigned long long* stats = alloc_n<unsigned long long>(stats_b, kStWords);
  PD_TRY(launch_fill_u64(stats, kStWords, 0ull, st));
  PD_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(counts + nc), sizeof(PlanCount) / 8, 0ull, st));
  for (int s = 0; s < 2; ++s) {
    // a few candidates per thread: the statistics are reduced once per thread
    const int grid = std::min(grid_for(nk * static_cast<int64_t>(g.n[s])), 2048);
    hipLaunchKernelGGL(k_count, dim3(grid), dim3(kThreads), 0, st, S.s[s], counts, stats);
    PD_TRY(hipGetLastError());
  }
  exclusive_scan(ct, counts, pos, PlanCountSum{}, nc + 1, st);
  counts_b.release();
  PlanCount tot{}, at1{};  // the totals, and the positions of side 1's first candidate
  unsigned long long hstats[kStWords];
  PD_TRY(hipMemcpyAsync(&tot, pos + nc, sizeof(tot), hipMemcpyDeviceToHost, st));
  PD_TRY(hipMemcpyAsync(&at1, pos + S.s[1].cand0, sizeof(at1), hipMemcpyDeviceToHost, st));
  PD_TRY(hipMemcpyAsync(hstats, stats, sizeof(hstats), hipMemcpyDeviceToHost, st));
  PD_TRY(hipStreamSynchronize(st));
  {
    PlanSizes z{};
    z.runs = std::max({tot.big_runs, tot.small_runs, tot.hub_runs});
    z.items = std::max<uint64_t>({tot.small_items, tot.hash, tot.rev, tot.hub_parts,
                                  uint64_t{tot.direct_parts} + tot.direct - tot.direct_split});
    z.reduces = uint64_t{tot.rev_reduces} + tot.direct_split;
    z.acc_slots = uint64_t{tot.rev_acc} + tot.direct_parts;
    std::string err;
    const int rc = check_plan_sizes(z, err);
    if (rc != DBBC_OK) throw Fail{rc, err};
  }
  const int64_t n_small = tot.small_items, n_hash = tot.hash, n_direct = tot.direct, n_rev = tot.rev;
  int64_t n_dir_items = int64_t{tot.direct_parts} + tot.direct - tot.direct_split;  // per-vertex: the windows
  const int64_t n_reduces = int64_t{tot.rev_reduces} + tot.direct_split;
  const int64_t acc_slots = int64_t{tot.rev_acc} + tot.direct_parts;

  // items
  DevBuf small_b, hash_tmp_b, hash_key_b, direct_tmp_b, direct_key_b, direct_meta_b, part_start_b;
  ItemOut io{};
  io.small = alloc_n<Item>(small_b, n_small);
  io.hash = alloc_n<Item>(hash_tmp_b, n_hash);
  io.hash_key = alloc_n<unsigned long long>(hash_key_b, n_hash);
  io.direct = alloc_n<Item>(direct_tmp_b, n_direct);
  io.direct_key = alloc_n<unsigned long long>(direct_key_b, n_direct);
  io.direct_meta = alloc_n<DirectMeta>(direct_meta_b, n_direct);
  io.rev = alloc_n<Item>(out.reverse_items, n_rev);
  io.reduces = alloc_n<Reduce>(out.reduces, n_reduces);
  if (p.per_vertex) io.small_owner = alloc_n<int32_t>(out.small_owner, n_small);
  for (int s = 0; s < 2; ++s) {
    hipLaunchKernelGGL(k_items, dim3(grid_for(nk * static_cast<int64_t>(g.n[s]))), dim3(kThreads), 0, st, S.s[s],
                       pos, io);
    PD_TRY(hipGetLastError());
  }

  // small groups
  for (int s = 0; s < 2; ++s) {
    int32_t kb = 1;
    while ((int64_t{1} << kb) < g.n[s]) ++kb;
    hp.key_bits[s] = kb;
  }
  const int64_t n_chunks = (n_small + kGroupChunk - 1) / kGroupChunk;
  DevBuf chunk_b, chunk_pos_b, local_b;
  uint32_t* chunk_cnt = alloc_n<uint32_t>(chunk_b, n_chunks + 1);
  uint32_t* chunk_pos = alloc_n<uint32_t>(chunk_pos_b, n_chunks + 1);
  uint32_t* local_of = alloc_n<uint32_t>(local_b, n_small);
  fill_u32(chunk_cnt + n_chunks, 1, 0u, st);
  if (n_chunks > 0) {
    hipLaunchKernelGGL(k_group<0>, dim3(grid_for(n_chunks)), dim3(kThreads), 0, st, io.small, n_small, hp.key_bits[0],
                       hp.key_bits[1], p.per_vertex, chunk_cnt, nullptr, nullptr);
    PD_TRY(hipGetLastError());
  }
  exclusive_sum(ct, chunk_cnt, chunk_pos, n_chunks + 1, st);
  uint32_t n_groups = 0;
  PD_TRY(hipMemcpyAsync(&n_groups, chunk_pos + n_chunks, sizeof(n_groups), hipMemcpyDeviceToHost, st));
  PD_TRY(hipStreamSynchronize(st));
  Item* groups = alloc_n<Item>(out.small_groups, n_groups);
  if (n_chunks > 0) {
    hipLaunchKernelGGL(k_group<1>, dim3(grid_for(n_chunks)), dim3(kThreads), 0, st, io.small, n_small,
                       hp.key_bits[0], hp.key_bits[1], p.per_vertex, chunk_pos, groups, local_of);
    PD_TRY(hipGetLastError());
  }

  // runs
  RunOut ro{};
  ro.segs = alloc_n<Segment>(out.segs, static_cast<int64_t>(tot.big_runs));
  ro.small_segs = alloc_n<Segment>(out.small_segs, static_cast<int64_t>(tot.small_runs));
  ro.local_of = local_of;
  ro.part_start = alloc_n<uint32_t>(part_start_b, tot.direct_parts);
  DevBuf hub_part_start_b, wide_b;
  if (p.per_vertex) {
    ro.seg_mid = alloc_n<uint32_t>(out.seg_mid, static_cast<int64_t>(tot.big_runs));
    ro.seg_edge = alloc_n<uint32_t>(out.seg_edge, static_cast<int64_t>(tot.big_runs));
    ro.small_seg_mid = alloc_n<uint32_t>(out.small_seg_mid, static_cast<int64_t>(tot.small_runs));
    ro.small_seg_edge = alloc_n<uint32_t>(out.small_seg_edge, static_cast<int64_t>(tot.small_runs));
    ro.hub_segs = alloc_n<Segment>(out.hub_segs, static_cast<int64_t>(tot.hub_runs));
    ro.hub_part_start = alloc_n<uint32_t>(hub_part_start_b, tot.hub_parts);
    ro.any_wide = alloc_n<uint32_t>(wide_b, 1);
    fill_u32(ro.any_wide, 1, 0u, st);
  }
  for (int s = 0; s < 2; ++s) {
    if (g.m == 0) break;
    hipLaunchKernelGGL(k_runs, dim3(grid_for(g.m)), dim3(kThreads), 0, st, S.s[s], pos, ro);
    PD_TRY(hipGetLastError());
  }
  if (n_rev > 0) {
    hipLaunchKernelGGL(k_rev_part_work, dim3(grid_for(n_rev)), dim3(kThreads), 0, st, io.rev, n_rev, ro.segs);
    PD_TRY(hipGetLastError());
  }
  if (p.per_vertex) {  // the hub pivots' tally items, side 0 first
    Item* hub_items = alloc_n<Item>(out.hub_items, tot.hub_parts);
    for (int s = 0; s < 2; ++s) {
      if (S.s[s].T == 0) continue;
      hipLaunchKernelGGL(k_hub_parts, dim3(grid_for(S.s[s].T)), dim3(kThreads), 0, st, S.s[s], pos,
                         ro.hub_part_start, hub_items);
      PD_TRY(hipGetLastError());
    }
  }

  // hash items, heaviest first
  DevBuf kout_b, vin_b, perm_b;
  {
    Item* hash = alloc_n<Item>(out.hash_items, n_hash);
    if (n_hash > 0) {
      unsigned long long* kout = alloc_n<unsigned long long>(kout_b, n_hash);
      uint32_t* vin = alloc_n<uint32_t>(vin_b, n_hash);
      uint32_t* perm = alloc_n<uint32_t>(perm_b, n_hash);
      hipLaunchKernelGGL(k_iota, dim3(grid_for(n_hash)), dim3(kThreads), 0, st, vin, n_hash);
      PD_TRY(hipGetLastError());
      sort_desc(ct, io.hash_key, kout, vin, perm, n_hash, st);
      hipLaunchKernelGGL(k_gather_items, dim3(grid_for(n_hash)), dim3(kThreads), 0, st, io.hash, perm, n_hash, hash);
      PD_TRY(hipGetLastError());
    }
  }
  // direct items, heaviest first: parts of split items, then single items
  {
    DirectOut dout{};
    dout.items = alloc_n<Item>(out.direct_items, n_dir_items);
    dout.reduces = io.reduces;
    dout.n_parts = tot.direct_parts;
    dout.acc0 = tot.rev_acc;
    dout.red0 = tot.rev_reduces;
    dout.pv = p.per_vertex;
    if (n_direct > 0) {
      unsigned long long* kout = alloc_n<unsigned long long>(kout_b, n_direct);
      uint32_t* vin = alloc_n<uint32_t>(vin_b, n_direct);
      uint32_t* perm = alloc_n<uint32_t>(perm_b, n_direct);
      hipLaunchKernelGGL(k_iota, dim3(grid_for(n_direct)), dim3(kThreads), 0, st, vin, n_direct);
      PD_TRY(hipGetLastError());
      if (p.per_vertex)  // side 0 first, heaviest first within a side (ascending keys)
        sort_asc(ct, io.direct_key, kout, vin, perm, n_direct, st);
      else
        sort_desc(ct, io.direct_key, kout, vin, perm, n_direct, st);
      DevBuf dc_b, dpos_b;
      DirectCount* dc = alloc_n<DirectCount>(dc_b, n_direct + 1);
      DirectCount* dpos = alloc_n<DirectCount>(dpos_b, n_direct + 1);
      hipLaunchKernelGGL(k_direct_count, dim3(grid_for(n_direct)), dim3(kThreads), 0, st, S, io.direct,
                         io.direct_meta, perm, n_direct, p.per_vertex, dc);
      PD_TRY(hipGetLastError());
      if (p.per_vertex) {
        // the windows' total sizes the list; side 0's items come first (at1.direct
        // of them), so the windows before side 1's first item are side 0's
        fill_u32(reinterpret_cast<uint32_t*>(dc + n_direct), sizeof(DirectCount) / 4, 0u, st);
        exclusive_scan(ct, dc, dpos, DirectCountSum{}, n_direct + 1, st);
        DirectCount t{}, t0{};
        PD_TRY(hipMemcpyAsync(&t, dpos + n_direct, sizeof(t), hipMemcpyDeviceToHost, st));
        PD_TRY(hipMemcpyAsync(&t0, dpos + at1.direct, sizeof(t0), hipMemcpyDeviceToHost, st));
        PD_TRY(hipStreamSynchronize(st));
        n_dir_items = t.parts;
        hp.n_direct_side0 = static_cast<int32_t>(t0.parts);
        PlanSizes z{};
        z.items = static_cast<uint64_t>(n_dir_items);
        std::string err;
        const int rc = check_plan_sizes(z, err);
        if (rc != DBBC_OK) throw Fail{rc, err};
        dout.items = alloc_n<Item>(out.direct_items, n_dir_items);
      } else {
        exclusive_scan(ct, dc, dpos, DirectCountSum{}, n_direct, st);
      }
      hipLaunchKernelGGL(k_direct_write, dim3(grid_for(n_direct)), dim3(kThreads), 0, st, S, io.direct,
                         io.direct_meta, perm, dpos, n_direct, ro.part_start, dout);
      PD_TRY(hipGetLastError());
      PD_TRY(hipStreamSynchronize(st));  // dc_b, dpos_b leave scope
    }
  }
  PD_TRY(out.acc.alloc(std::max<size_t>(static_cast<size_t>(acc_slots) * hp.acc_width * sizeof(uint32_t), 16)));

  // the dense block's signs
  for (int s = 0; s < 2; ++s) {
    out.hub_K[s] = 0;
    const int32_t T = hp.T[s], TO = hp.T[1 - s];
    if (T == 0) continue;
    const int32_t K = (TO + kHubKPad - 1) / kHubKPad * kHubKPad;
    const size_t TK = static_cast<size_t>(T) * K;
    int8_t* Bs = alloc_n<int8_t>(out.hub_B[s], static_cast<int64_t>(TK));
    int8_t* Bm = alloc_n<int8_t>(out.hub_Bm[s], static_cast<int64_t>(TK));
    PD_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(Bs), TK / 8, 0ull, st));
    PD_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(Bm), TK / 8, 0ull, st));
    int32_t* hpos = nullptr;
    if (p.per_vertex) {  // T K is a multiple of 128 kHubKPad: whole words
      hpos = alloc_n<int32_t>(out.hub_pos[s], static_cast<int64_t>(TK));
      PD_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(hpos), TK / 2, ~0ull, st));
    }
    if (g.m > 0) {
      hipLaunchKernelGGL(k_hub_signs, dim3(grid_for(static_cast<int64_t>(g.m))), dim3(kThreads), 0, st, g.off[s],
                         g.adj[s], S.s[s].row, g.grank[s], g.grank[1 - s], T, TO, K, Bs, Bm, hpos);
      PD_TRY(hipGetLastError());
    }
    if (p.per_vertex) {  // the credit products' constants
      int8_t* Bt = alloc_n<int8_t>(out.hub_Bt[s], static_cast<int64_t>(TK));
      int8_t* Bmt = alloc_n<int8_t>(out.hub_Bmt[s], static_cast<int64_t>(TK));
      int32_t* Zc = alloc_n<int32_t>(out.hub_Zc[s], static_cast<int64_t>(TK));
      int32_t* Zcp = alloc_n<int32_t>(out.hub_Zcp[s], static_cast<int64_t>(TK));
      hipLaunchKernelGGL(k_hub_transpose, dim3(grid_for(static_cast<int64_t>(TK))), dim3(kThreads), 0, st, Bs, Bm,
                         T, K, Bt, Bmt);
      PD_TRY(hipGetLastError());
      const int64_t ncol = static_cast<int64_t>((T + kColChunk - 1) / kColChunk) * K;
      DevBuf cb_b, cbm_b;
      uint32_t* cB = alloc_n<uint32_t>(cb_b, ncol);
      uint32_t* cBm = alloc_n<uint32_t>(cbm_b, ncol);
      hipLaunchKernelGGL(k_hub_chunk_counts, dim3(grid_for(ncol)), dim3(kThreads), 0, st, Bs, Bm, T, K, cB, cBm);
      PD_TRY(hipGetLastError());
      hipLaunchKernelGGL(k_hub_col_counts, dim3(grid_for(ncol)), dim3(kThreads), 0, st, Bs, Bm, T, K, cB, cBm, Zc,
                         Zcp);
      PD_TRY(hipGetLastError());
      PD_TRY(hipStreamSynchronize(st));  // cb_b, cbm_b leave scope
    }
    out.hub_K[s] = K;
  }
  uint32_t wide_h = 0;
  if (p.per_vertex) PD_TRY(hipMemcpyAsync(&wide_h, ro.any_wide, sizeof(wide_h), hipMemcpyDeviceToHost, st));
  PD_TRY(hipStreamSynchronize(st));
  out.any_wide = wide_h != 0;

  hp.acc_slots = static_cast<int32_t>(acc_slots);
  hp.n_reverse_side0 = static_cast<int32_t>(at1.rev);
  if (p.per_vertex) hp.n_hub_side0 = static_cast<int32_t>(at1.hub_parts);
  hp.n_items_kept[0] = static_cast<int32_t>(n_dir_items);
  hp.n_items_kept[1] = static_cast<int32_t>(n_rev);
  hp.n_items_kept[2] = static_cast<int32_t>(n_groups);
  hp.n_items_kept[3] = static_cast<int32_t>(n_hash);
  hp.n_items_kept[4] = static_cast<int32_t>(n_reduces);
  for (int j = 0; j < 4; ++j) {
    hp.k_wedges[j] = static_cast<int64_t>(hstats[kStWedges + j]);
    hp.k_segs[j] = static_cast<int64_t>(hstats[kStRuns + j]);
  }
  hp.w_sparse = static_cast<int64_t>(hstats[kStSparse]);
  hp.w_skipped = static_cast<int64_t>(hstats[kStSkipped]);
}

}  // namespace

int make_plan_device(const DevGraphView& g, const PlanParams& p, hipStream_t st, HostPlan& hp, DevPlanLists& out,
                     std::string& err) {
  int rc = check_plan_params(p, err);
  if (rc != DBBC_OK) return rc;
  // hipCUB takes int sizes: candidates and entries (plus one) must fit
  if ((p.per_vertex ? 4 : 3) * (static_cast<int64_t>(g.n[0]) + g.n[1]) + 1 > INT32_MAX || g.m + 1 > INT32_MAX) {
    err = "graph too large for the device planner";
    return DBBC_E_TOO_LARGE;
  }
  hp = HostPlan();
  hp.p = p;
  plan_windows(g.n, p, hp);
  try {
    plan(g, p, st, hp, out);
  } catch (const Fail& f) {
    err = f.msg;
    (void)hipStreamSynchronize(st);
    return f.status;
  } catch (const std::bad_alloc&) {
    err = "host allocation failed while planning";
    (void)hipStreamSynchronize(st);
    return DBBC_E_OOM;
  }
  return DBBC_OK;
}

}  // namespace dbbc

namespace dbbc {

int edge_positions_device(const DevGraphView& g, uint32_t* out, hipStream_t st, std::string& err) {
  if (g.m == 0) return DBBC_OK;
  hipLaunchKernelGGL(k_edge_positions, dim3(grid_for(g.m)), dim3(kThreads), 0, st, g.adj[0], g.rev[0], g.off[1], g.m,
                     out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("edge positions: ") + hipGetErrorString(e);
    return DBBC_E_DEVICE;
  }
  return DBBC_OK;
}

}  // namespace dbbc
