// Counting plan built on the device: the work split of make_plan (plan.cpp)
// for a count, computed from the device CSR with kernels, scans and sorts
// (the binning step of Algorithm 1 that sizes each pivot's work, Eq. 1,
// done per CSR entry instead of per pivot on the host).
//
// Per side s, every CSR entry e of row x, with mid y = adj[e] >> 1, yields at
// most one run of each kind:
//   F  forward: pivot x, the entries of row y below x in priority (from
//      rev[e] + 1 on), for e past x's higher-priority prefix cut[x]; a
//      window pivot (x < L) stops at the window, a hub pivot (x < T) with a
//      hub mid (y < T') starts past the dense block;
//   R  reverse (x >= L): the prefix of row y below both the reverse window
//      R and y's own higher-priority prefix cut[y];
//   M  reverse-mid (x >= L, R < L): the part of that prefix in [R, L).
// Each (row, kind) is one candidate item.  Exclusive scans of the run flags
// and lengths over the entries give every candidate's run count and work as
// a difference of two scan values, and every run's place in its item.  The
// candidates are classified as make_plan classifies its items (skipped,
// small, hash, direct, reverse); one scan of the candidates' list counts
// places every item in its list and every run in segs or small_segs.
//
// Where the result differs from make_plan's, both are valid plans of the
// same wedges (the counts are the same):
//   - items and runs are listed in candidate order (row, then kind);
//   - small items are grouped greedily within chunks of kGroupChunk items;
//   - a split direct item starts a new part at every run that holds a
//     multiple of part_work in its wedge range (and every kPartMaxRuns
//     runs), so a part has at most part_work wedges plus its first run.
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

enum : int { kF = 0, kR = 1, kM = 2 };                                 // run kinds
enum : int { kSkip = 0, kSmallC = 1, kHashC = 2, kDirectC = 3, kRevC = 4 };  // item classes

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
  uint32_t* len[3];       // run length per kind and entry (m + 1, the last 0)
  uint32_t* cnt[3];       // exclusive scans of len > 0
  unsigned long long* wsum[3];  // exclusive scans of len
  uint32_t* bnd[2];       // kinds F and M: exclusive scans of part-start flags
  int32_t* rmax;          // per row: largest key of its reverse runs
  int32_t n, no, L, R, T, TO;
  int64_t m;
  uint32_t side;
  int64_t cand0;          // index of the side's first candidate (3 per row)
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
    c.cls = kRevC;
    c.nparts = c.nseg <= kReverseCountMaxSegs ? 0u : (c.nseg + kReverseCountMaxSegs - 1) / kReverseCountMaxSegs;
  } else {
    c.key_lo = P.R;
    c.key_hi = P.L;
    c.cls = small ? kSmallC : kDirectC;
  }
  if (c.cls == kDirectC && (c.work > P.part_work || c.nseg > kPartMaxRuns)) {
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
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const Run r = run_at(P, k, x, e);
      P.len[k][e] = r.len;
      if (k == kR && r.len > 0) atomicMax(&P.rmax[x], static_cast<int32_t>(P.oadj[r.start + r.len - 1] >> 1));
    }
  }
}

// Part-start flags of the runs of split direct items (kinds F and M): the
// first run, every kPartMaxRuns-th run, and every run whose wedge range
// [pex, pex + len) of the item holds a multiple of part_work.
__global__ void k_part_flags(PSide P, int k, uint32_t* flag) {
  GRID_STRIDE(e64, P.m) {
    const uint32_t e = static_cast<uint32_t>(e64);
    const uint32_t len = P.len[k][e];
    uint32_t f = 0;
    if (len > 0) {
      const int32_t x = static_cast<int32_t>(P.row[e]);
      const Cand c = classify<false>(P, x, k);
      if (c.split) {
        const uint32_t b = P.off[x];
        const uint32_t j = P.cnt[k][e] - P.cnt[k][b];
        const unsigned long long pex = P.wsum[k][e] - P.wsum[k][b];
        const unsigned long long pw = P.part_work;
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
  uint32_t small_items, hash, direct, direct_parts, direct_split, rev, rev_reduces, rev_acc;
};

struct PlanCountSum {
  __host__ __device__ PlanCount operator()(const PlanCount& a, const PlanCount& b) const {
    PlanCount r;
    r.big_runs = a.big_runs + b.big_runs;
    r.small_runs = a.small_runs + b.small_runs;
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

// Each candidate's list counts; the statistics are summed per thread over
// its candidates, then per wavefront, then once per wavefront into stats.
__global__ void k_count(PSide P, PlanCount* counts, unsigned long long* stats) {
  const int64_t nc = 3 * static_cast<int64_t>(P.n);
  unsigned long long w[4] = {0, 0, 0, 0}, r[4] = {0, 0, 0, 0}, sparse = 0, skipped = 0;
  GRID_STRIDE(i, nc) {
    const int32_t x = static_cast<int32_t>(i / 3);
    const int k = static_cast<int>(i % 3);
    const Cand c = classify<true>(P, x, k);
    PlanCount q{};
    int slot = -1;
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
      default:
        skipped += c.work;
        break;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      w[j] += j == slot ? c.work : 0ull;
      r[j] += j == slot ? c.nseg : 0u;
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
  Item* hash;          // hash items, unordered
  unsigned long long* hash_key;
  Item* direct;        // direct items, unordered
  unsigned long long* direct_key;
  DirectMeta* direct_meta;
  Item* rev;           // reverse items (final)
  Reduce* reduces;     // reverse reduces first
};

__global__ void k_items(PSide P, const PlanCount* pos, ItemOut o) {
  const int64_t nc = 3 * static_cast<int64_t>(P.n);
  GRID_STRIDE(i, nc) {
    const int32_t x = static_cast<int32_t>(i / 3);
    const int k = static_cast<int>(i % 3);
    const Cand c = classify<true>(P, x, k);
    if (c.cls == kSkip) continue;
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
      continue;
    }
    it.seg_begin = static_cast<uint32_t>(q.big_runs);
    if (c.cls == kHashC) {
      o.hash[q.hash] = it;
      o.hash_key[q.hash] = c.work;
    } else if (c.cls == kDirectC) {
      o.direct[q.direct] = it;
      o.direct_key[q.direct] = c.work;
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
__global__ void k_group(const Item* small, int64_t n_small, int32_t kb0, int32_t kb1, uint32_t* chunk_groups,
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
        grp.acc_slot = -1;
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
};

// Every run into its item's place: segs[item's first + j] for the j-th run
// of the item, or small_segs tagged with the item's index in its group.
__global__ void k_runs(PSide P, const PlanCount* pos, RunOut o) {
  GRID_STRIDE(e64, P.m) {
    const uint32_t e = static_cast<uint32_t>(e64);
    const int32_t x = static_cast<int32_t>(P.row[e]);
    const uint32_t b = P.off[x];
    const uint32_t g = P.adj[e] & 1u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (P.len[k][e] == 0) continue;
      const Cand c = classify<true>(P, x, k);
      if (c.cls == kSkip) continue;
      const PlanCount q = pos[P.cand0 + 3 * static_cast<int64_t>(x) + k];
      const Run r = run_at(P, k, x, e);
      const uint32_t j = P.cnt[k][e] - P.cnt[k][b];
      const uint32_t len_g = (r.len << 1) | g;
      if (c.cls == kSmallC) {
        o.small_segs[q.small_runs + j] = Segment{r.start, (o.local_of[q.small_items] << 16) | len_g};
      } else {
        o.segs[q.big_runs + j] = Segment{r.start, len_g};
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

__global__ void k_direct_count(const DirectMeta* meta, const uint32_t* perm, int64_t n, DirectCount* out) {
  GRID_STRIDE(i, n) {
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
};

__global__ void k_direct_write(PSides S, const Item* direct, const DirectMeta* meta, const uint32_t* perm,
                               const DirectCount* pos, int64_t n, const uint32_t* part_start, DirectOut o) {
  GRID_STRIDE(i, n) {
    const Item it = direct[perm[i]];
    const DirectMeta md = meta[perm[i]];
    const DirectCount q = pos[i];
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
__global__ void k_hub_signs(const uint32_t* off, const uint32_t* adj, const uint32_t* rows, const int32_t* grank_s,
                            const int32_t* grank_o, int32_t T, int32_t TO, int32_t K, int8_t* B, int8_t* Bm) {
  const int64_t ne = off[T];
  GRID_STRIDE(e, ne) {
    const uint32_t x = rows[e];
    const uint32_t y = adj[e] >> 1;
    if (static_cast<int32_t>(y) >= TO) continue;
    const int8_t sg = (adj[e] & 1u) ? int8_t(-1) : int8_t(1);
    const size_t at = static_cast<size_t>(x) * K + y;
    B[at] = sg;
    if (grank_o[y] > grank_s[x]) Bm[at] = sg;
  }
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

template <class T>
T* alloc_n(DevBuf& b, int64_t n) {
  PD_TRY(b.alloc(static_cast<size_t>(std::max<int64_t>(n, 1)) * sizeof(T)));
  return b.as<T>();
}

// One side's scratch arrays.
struct SideBufs {
  DevBuf rows, rows_tmp, splitL, splitR, splitT, rmax, len[3], cnt[3], wsum[3], bnd[2];
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
    P.cand0 = s == 0 ? 0 : 3 * static_cast<int64_t>(g.n[0]);
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
    for (int k = 0; k < 3; ++k) {
      P.len[k] = alloc_n<uint32_t>(B.len[k], m + 1);
      fill_u32(P.len[k] + m, 1, 0u, st);
    }
    if (m > 0) {
      hipLaunchKernelGGL(k_run_lengths, dim3(grid_for(m)), dim3(kThreads), 0, st, P);
      PD_TRY(hipGetLastError());
    }
    for (int k = 0; k < 3; ++k) {
      P.cnt[k] = alloc_n<uint32_t>(B.cnt[k], m + 1);
      P.wsum[k] = alloc_n<unsigned long long>(B.wsum[k], m + 1);
      exclusive_sum(ct, rocprim::make_transform_iterator(P.len[k], NonZero{}), P.cnt[k], m + 1, st);
      exclusive_sum(ct, rocprim::make_transform_iterator(P.len[k], Widen{}), P.wsum[k], m + 1, st);
    }
    // part starts of split direct items (kinds F and M); the flags borrow
    // the row scratch of the other kind's scan
    DevBuf flags;
    uint32_t* fl = alloc_n<uint32_t>(flags, m + 1);
    for (int j = 0; j < 2; ++j) {
      const int k = j == 0 ? kF : kM;
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
  const int64_t nc = 3 * (static_cast<int64_t>(g.n[0]) + g.n[1]);
  DevBuf counts_b, pos_b, stats_b;
  PlanCount* counts = alloc_n<PlanCount>(counts_b, nc + 1);
  PlanCount* pos = alloc_n<PlanCount>(pos_b, nc + 1);
  unsigned long long* stats = alloc_n<unsigned long long>(stats_b, kStWords);
  PD_TRY(launch_fill_u64(stats, kStWords, 0ull, st));
  PD_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(counts + nc), sizeof(PlanCount) / 8, 0ull, st));
  for (int s = 0; s < 2; ++s) {
    // a few candidates per thread: the statistics are reduced once per thread
    const int grid = std::min(grid_for(3 * static_cast<int64_t>(g.n[s])), 2048);
    hipLaunchKernelGGL(k_count, dim3(grid), dim3(kThreads), 0, st, S.s[s], counts, stats);
    PD_TRY(hipGetLastError());
  }
  exclusive_scan(ct, counts, pos, PlanCountSum{}, nc + 1, st);
  counts_b.release();
  PlanCount tot{};
  unsigned long long hstats[kStWords];
  PD_TRY(hipMemcpyAsync(&tot, pos + nc, sizeof(tot), hipMemcpyDeviceToHost, st));
  PD_TRY(hipMemcpyAsync(hstats, stats, sizeof(hstats), hipMemcpyDeviceToHost, st));
  PD_TRY(hipStreamSynchronize(st));
  {
    PlanSizes z{};
    z.runs = std::max(tot.big_runs, tot.small_runs);
    z.items = std::max<uint64_t>({tot.small_items, tot.hash, tot.rev,
                                  uint64_t{tot.direct_parts} + tot.direct - tot.direct_split});
    z.reduces = uint64_t{tot.rev_reduces} + tot.direct_split;
    z.acc_slots = uint64_t{tot.rev_acc} + tot.direct_parts;
    std::string err;
    const int rc = check_plan_sizes(z, err);
    if (rc != DBBC_OK) throw Fail{rc, err};
  }
  const int64_t n_small = tot.small_items, n_hash = tot.hash, n_direct = tot.direct, n_rev = tot.rev;
  const int64_t n_dir_items = int64_t{tot.direct_parts} + tot.direct - tot.direct_split;
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
  for (int s = 0; s < 2; ++s) {
    hipLaunchKernelGGL(k_items, dim3(grid_for(3 * static_cast<int64_t>(g.n[s]))), dim3(kThreads), 0, st, S.s[s],
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
                       hp.key_bits[1], chunk_cnt, nullptr, nullptr);
    PD_TRY(hipGetLastError());
  }
  exclusive_sum(ct, chunk_cnt, chunk_pos, n_chunks + 1, st);
  uint32_t n_groups = 0;
  PD_TRY(hipMemcpyAsync(&n_groups, chunk_pos + n_chunks, sizeof(n_groups), hipMemcpyDeviceToHost, st));
  PD_TRY(hipStreamSynchronize(st));
  Item* groups = alloc_n<Item>(out.small_groups, n_groups);
  if (n_chunks > 0) {
    hipLaunchKernelGGL(k_group<1>, dim3(grid_for(n_chunks)), dim3(kThreads), 0, st, io.small, n_small,
                       hp.key_bits[0], hp.key_bits[1], chunk_pos, groups, local_of);
    PD_TRY(hipGetLastError());
  }

  // runs
  RunOut ro{};
  ro.segs = alloc_n<Segment>(out.segs, static_cast<int64_t>(tot.big_runs));
  ro.small_segs = alloc_n<Segment>(out.small_segs, static_cast<int64_t>(tot.small_runs));
  ro.local_of = local_of;
  ro.part_start = alloc_n<uint32_t>(part_start_b, tot.direct_parts);
  for (int s = 0; s < 2; ++s) {
    if (g.m == 0) break;
    hipLaunchKernelGGL(k_runs, dim3(grid_for(g.m)), dim3(kThreads), 0, st, S.s[s], pos, ro);
    PD_TRY(hipGetLastError());
  }
  if (n_rev > 0) {
    hipLaunchKernelGGL(k_rev_part_work, dim3(grid_for(n_rev)), dim3(kThreads), 0, st, io.rev, n_rev, ro.segs);
    PD_TRY(hipGetLastError());
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
    if (n_direct > 0) {
      unsigned long long* kout = alloc_n<unsigned long long>(kout_b, n_direct);
      uint32_t* vin = alloc_n<uint32_t>(vin_b, n_direct);
      uint32_t* perm = alloc_n<uint32_t>(perm_b, n_direct);
      hipLaunchKernelGGL(k_iota, dim3(grid_for(n_direct)), dim3(kThreads), 0, st, vin, n_direct);
      PD_TRY(hipGetLastError());
      sort_desc(ct, io.direct_key, kout, vin, perm, n_direct, st);
      DevBuf dc_b, dpos_b;
      DirectCount* dc = alloc_n<DirectCount>(dc_b, n_direct + 1);
      DirectCount* dpos = alloc_n<DirectCount>(dpos_b, n_direct + 1);
      hipLaunchKernelGGL(k_direct_count, dim3(grid_for(n_direct)), dim3(kThreads), 0, st, io.direct_meta, perm,
                         n_direct, dc);
      PD_TRY(hipGetLastError());
      exclusive_scan(ct, dc, dpos, DirectCountSum{}, n_direct, st);
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
    hipLaunchKernelGGL(k_hub_signs, dim3(grid_for(static_cast<int64_t>(g.m))), dim3(kThreads), 0, st, g.off[s],
                       g.adj[s], S.s[s].row, g.grank[s], g.grank[1 - s], T, TO, K, Bs, Bm);
    PD_TRY(hipGetLastError());
    out.hub_K[s] = K;
  }
  PD_TRY(hipStreamSynchronize(st));

  hp.acc_slots = static_cast<int32_t>(acc_slots);
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
  if (p.per_vertex) {
    err = "internal: the device planner makes count plans only";
    return DBBC_E_INVALID_ARG;
  }
  int rc = check_plan_params(p, err);
  if (rc != DBBC_OK) return rc;
  // hipCUB takes int sizes: candidates and entries (plus one) must fit
  if (3 * (static_cast<int64_t>(g.n[0]) + g.n[1]) + 1 > INT32_MAX || g.m + 1 > INT32_MAX) {
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
