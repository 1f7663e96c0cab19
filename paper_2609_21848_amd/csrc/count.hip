// HIP kernels (gfx950) for the vertex-priority wedge tally and the pair
// reduction of Algorithm 1, Phase 5, with Lemma 1's per-endpoint
// C(B1,2) + C(B2,2) (and the unbalanced B1 * B2, the total C(B1 + B2, 2)).
//
// Work arrives as items (see plan.cpp): each item owns a set of same-side
// vertex pairs and lists the CSR runs ("segments") whose entries end its
// wedges.  A wedge is tallied into a per-key counter packed as
// (asymmetric << 16) | symmetric; an item never has more than 65535
// segments, and a key gains at most one wedge per segment, so neither half
// overflows.  After an item's walk its counters are swept: every pair's
// counts are turned into the three int64 sums, written to a part buffer
// (items split for load balance), or handed to the dense hub path.
//
// Memory layout: CSR entries are 32-bit words (neighbour side rank << 1 |
// negative bit), rows in priority order, so each segment is a coalesced run.
// The entry arrays are padded by kAdjPad words so that 16-byte loads at the
// end of a run stay inside the allocation.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"

namespace dbbc {
namespace dev {

constexpr int kWave = 64;
constexpr uint32_t kChunk = 256;   // entries per wavefront 16-byte load (64 lanes x 4)
constexpr uint32_t kGather = 256;  // positions per staging round of short runs
constexpr uint32_t kEmpty = 0xffffffffu;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t readlane(uint32_t v, int j) {
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), j));
}

// DPP move of v within the wavefront (lanes without a source read 0).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(v), kCtrl, kRowMask, 0xf, false));
}

// Exclusive prefix sum over the wavefront with DPP: an inclusive scan inside
// each row of 16 lanes (row_shr 1, 2, 4, 8), then row_bcast:15 and
// row_bcast:31 carry the row totals upward.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t* total) {
  uint32_t v = x;
  v += dpp<0x111, 0xf>(v);  // row_shr:1
  v += dpp<0x112, 0xf>(v);  // row_shr:2
  v += dpp<0x114, 0xf>(v);  // row_shr:4
  v += dpp<0x118, 0xf>(v);  // row_shr:8
  v += dpp<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  *total = readlane(v, kWave - 1);
  return v - x;
}

// Order this wavefront's LDS accesses (not its global loads, which may stay
// in flight, e.g. prefetches of the next item).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
}

// One lane's run of a batch (len 0 = none).  Bit 0 of tag is the sign bit g
// of the run's first wedge edge; the runs of a small-item group also carry
// the item's index in the group above it (tag = index << 1 | g).
struct SegReg {
  uint32_t start, len, tag;
};

template <bool kTagged>
__device__ __forceinline__ SegReg load_seg(const Segment* __restrict__ segs, uint32_t k0, uint32_t k1) {
  const uint32_t k = k0 + lane_id();
  SegReg r{0, 0, 0};
  if (k < k1) {
    const Segment s = segs[k];
    r.start = s.start;
    if (kTagged) {
      r.len = (s.len_g & 0xffffu) >> 1;
      r.tag = (s.len_g & 1u) | ((s.len_g >> 16) << 1);
    } else {
      r.len = s.len_g >> 1;
      r.tag = s.len_g & 1u;
    }
  }
  return r;
}

// v of lane src (all lanes must be active).
__device__ __forceinline__ uint32_t bpermute(uint32_t v, uint32_t src) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_ds_bpermute(static_cast<int>(src << 2), static_cast<int>(v)));
}

// Short runs of a batch are laid end to end: flat position t (0 <= t <
// total) is entry base + t of its run's row, with base = start - excl of
// the run.  A staging round covers positions [done, done + kGather), dealt
// to lanes as t = done + 64 u + lane (coalesced loads).  Every run that
// starts in the round, or continues into it, writes its base and its tag
// (with bit 31 set as a presence flag) at its first position of the round
// into the wavefront's marks buffers; a position's run is then the last
// mark at or before it: a ballot per block of 64 positions, carried across
// blocks.  Each lane clears the presence words it read, so they are all
// zero between rounds.
constexpr int kStageU = kGather / kWave;

// TagT holds a run's tag plus the presence bit (its top bit): 8 bits for
// plain runs (tag = g), 32 bits for small-item groups.
template <class TagT>
struct Marks {
  uint32_t* base;  // kGather words
  TagT* tag;       // kGather entries, zero when no run starts there
  static constexpr uint32_t kBit = 1u << (8 * sizeof(TagT) - 1);
};

struct Staged {
  uint32_t e[kStageU], tag[kStageU];
  bool valid[kStageU];
};

template <class M>
__device__ __forceinline__ void stage_round(Staged& s, M mk, uint32_t excl, uint32_t slen,
                                            uint32_t base, uint32_t tag, uint32_t total, uint32_t done,
                                            const uint32_t* __restrict__ adj) {
  const int lane = lane_id();
  wave_sync_lds();
  if (slen != 0 && excl < done + kGather && excl + slen > done) {
    const uint32_t pos = excl > done ? excl - done : 0u;
    mk.base[pos] = base;
    mk.tag[pos] = static_cast<decltype(+mk.tag[0])>(tag | M::kBit);
  }
  wave_sync_lds();
  const uint64_t upto = (2ull << lane) - 1ull;  // lanes 0 .. lane
  uint32_t cb = 0, ct = 0;
#pragma unroll
  for (int u = 0; u < kStageU; ++u) {
    const uint32_t mt = static_cast<uint32_t>(mk.tag[u * kWave + lane]);
    const uint32_t mb = mk.base[u * kWave + lane];
    mk.tag[u * kWave + lane] = 0;
    const uint64_t below = __ballot(mt != 0) & upto;
    const uint32_t src = below ? 63u - static_cast<uint32_t>(__clzll(below)) : 0u;
    const uint32_t pb = bpermute(mb, src), pt = bpermute(mt, src);
    // positions past the end may have no run: masked below
    const uint32_t b = below ? pb : cb;
    const uint32_t tg = below ? pt : ct;
    cb = readlane(b, kWave - 1);
    ct = readlane(tg, kWave - 1);
    s.tag[u] = tg & ~M::kBit;
    const uint32_t t = done + static_cast<uint32_t>(u * kWave + lane);
    s.valid[u] = t < total;
    s.e[u] = adj[s.valid[u] ? b + t : 0u];
  }
}

// Walk a batch of up to 64 runs (one per lane, in registers) with one
// wavefront, calling f.add(entry, tag, valid) once per wedge slot.
//  - Runs of at least long_len entries are consumed as a stream of
//    256-entry chunks: every lane loads 4 aligned entries (16 bytes) per
//    chunk, U chunks are in flight per lane, and a chunk's out-of-run words
//    are masked.  The chunk loop is wavefront-uniform.
//  - Shorter runs are staged (stage_round) so that every lane holds wedges;
//    the loads of the first round are issued before the long stream and the
//    next round's loads before the current round is tallied.
template <int U, class M, class F>
__device__ __forceinline__ void walk_regs(SegReg sr, const uint32_t* __restrict__ adj, M marks,
                                          uint32_t long_len, F&& f) {
  const int lane = lane_id();
  const uint32_t start = sr.start, tag = sr.tag, len = sr.len;
  uint64_t longm = __ballot(len >= long_len);
  const uint32_t slen = len >= long_len ? 0u : len;
  uint32_t total;
  const uint32_t excl = wave_excl_scan(slen, &total);
  const uint32_t base = start - excl;
  Staged cur;
  if (total) stage_round(cur, marks, excl, slen, base, tag, total, 0, adj);
  uint32_t cur_st = 0, cur_end = 0, cur_g = 0, cur_pos = 0;
  bool have = false;
  while (longm || have) {
    uint4 v[U];
    uint32_t vst[U], vend[U], vg[U], vp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!have && longm) {
        const int j = __ffsll(static_cast<unsigned long long>(longm)) - 1;
        longm &= longm - 1;
        cur_st = readlane(start, j);
        cur_end = cur_st + readlane(len, j);
        cur_g = readlane(tag, j);
        cur_pos = cur_st & ~3u;
        have = true;
      }
      // The load is unconditional (no wait on registers of a skipped load):
      // lanes past the run's end and empty slots read the first entries of
      // the array, and their words fail the index test below.
      const bool h = have;
      const uint32_t p = cur_pos + 4 * lane;
      vst[u] = cur_st;
      vg[u] = cur_g;
      vp[u] = p;
      vend[u] = h ? cur_end : 0u;
      v[u] = *reinterpret_cast<const uint4*>(adj + ((h && p < cur_end) ? p : 0u));
      if (h) {
        cur_pos += kChunk;
        if (cur_pos >= cur_end) have = false;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t e4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t idx = vp[u] + q;
        f.add(e4[q], vg[u], idx >= vst[u] && idx < vend[u]);
      }
    }
  }
  for (uint32_t done = 0; done < total; done += kGather) {
    const bool more = done + kGather < total;
    Staged nxt;
    if (more) stage_round(nxt, marks, excl, slen, base, tag, total, done + kGather, adj);
#pragma unroll
    for (int u = 0; u < kStageU; ++u) f.add(cur.e[u], cur.tag[u], cur.valid[u]);
    if (!more) break;
    cur = nxt;
  }
}

template <int U, bool kTagged = false, class M, class F>
__device__ __forceinline__ void walk_batch(const Segment* __restrict__ segs, uint32_t k0, uint32_t k1,
                                           const uint32_t* __restrict__ adj, M marks,
                                           uint32_t long_len, F&& f) {
  walk_regs<U>(load_seg<kTagged>(segs, k0, k1), adj, marks, long_len, f);
}

// Walk every run of an item with one wavefront; the first batch of 64 runs
// was loaded beforehand (first).
template <int U, bool kTagged = false, class M, class F>
__device__ __forceinline__ void walk_item(const Item& it, SegReg first, const Segment* __restrict__ segs,
                                          const uint32_t* __restrict__ adj, M marks,
                                          uint32_t long_len, F&& f) {
  const uint32_t seg_end = it.seg_begin + it.seg_count;
  walk_regs<U>(first, adj, marks, long_len, f);
  for (uint32_t k0 = it.seg_begin + kWave; k0 < seg_end; k0 += kWave) {
    const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
    walk_regs<U>(load_seg<kTagged>(segs, k0, k1), adj, marks, long_len, f);
  }
}

template <bool kTagged = false>
__device__ __forceinline__ SegReg first_batch(const Item& it, const Segment* __restrict__ segs) {
  const uint32_t seg_end = it.seg_begin + it.seg_count;
  return load_seg<kTagged>(segs, it.seg_begin,
                           it.seg_begin + kWave < seg_end ? it.seg_begin + kWave : seg_end);
}

// Packed counter increment of one wedge: +1 symmetric or +2^16 asymmetric.
__device__ __forceinline__ uint32_t wedge_inc(uint32_t e, uint32_t g) {
  return ((e ^ g) & 1u) ? 0x10000u : 1u;
}

// Tally functors for walk_regs: add(entry, g, valid) counts a valid
// entry's wedge in the counter of its key (a non-returning LDS atomic, so a
// wavefront never waits on its own counter updates).
struct DirectTally {  // 16 | 16-bit counters, one 32-bit word per key
  uint32_t* cnt;
  __device__ __forceinline__ void add(uint32_t e, uint32_t g, bool valid) const {
    if (valid) atomicAdd(&cnt[e >> 1], wedge_inc(e, g));
  }
};

struct PairTally {  // 8 | 8-bit counters, two keys per 32-bit word
  uint32_t* cnt;
  __device__ __forceinline__ void add(uint32_t e, uint32_t g, bool valid) const {
    // the entry's low bits select the byte: bit 0 (negative) ^ g picks the
    // symmetric / asymmetric byte, bit 1 (key parity) the 16-bit half
    if (valid) atomicAdd(&cnt[e >> 2], 1u << (((e ^ (g & 1u)) & 3u) << 3));
  }
};

// Hash tallies do all their work in add (a probe loop).
template <class G>
struct HashTally {
  G g;
  __device__ __forceinline__ void add(uint32_t e, uint32_t gb, bool valid) const {
    if (valid) g(e, gb);
  }
};
template <class G>
__device__ __forceinline__ HashTally<G> hash_tally(G g) {
  return HashTally<G>{g};
}

struct Sums {
  int64_t bal = 0, unb = 0, tot = 0;
  __device__ __forceinline__ void add(uint32_t p, uint32_t n) {
    const int64_t P = p, N = n;
    bal += P * (P - 1) / 2 + N * (N - 1) / 2;
    unb += P * N;
    tot += (P + N) * (P + N - 1) / 2;
  }
};

// The sums of a wavefront (or workgroup) belong to one graph at a time:
// items of a graph are contiguous in every list, and the running sums are
// flushed to the graph's result slot when an item of another graph comes.
constexpr uint32_t kNoGraph = 0xffffffffu;

__device__ __forceinline__ int64_t wave_sum64(int64_t x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

// Add the wavefront's sums to a graph's results (one atomic per wavefront
// and value).
__device__ __forceinline__ void flush_sums(const Sums& s, unsigned long long* res) {
  const int64_t b = wave_sum64(s.bal), u = wave_sum64(s.unb), t = wave_sum64(s.tot);
  if (lane_id() == 0) {
    if (b) atomicAdd(res + kResBalanced, static_cast<unsigned long long>(b));
    if (u) atomicAdd(res + kResUnbalanced, static_cast<unsigned long long>(u));
    if (t) atomicAdd(res + kResTotal, static_cast<unsigned long long>(t));
  }
}

// Final fate of one pair count of an item.
__device__ __forceinline__ void emit(const Item& it, uint32_t key, uint32_t p, uint32_t n,
                                     const DevSideConst& sc, Sums& s) {
  if ((it.flags & kItemHubPairs) && static_cast<int32_t>(key) < sc.T) {
    sc.hub_pairs[static_cast<size_t>(it.owner) * sc.T + key] =
        (static_cast<unsigned long long>(n) << 32) | p;
  } else {
    s.add(p, n);
  }
}

// ---------------------------------------------------------------------------
// Window items: one workgroup per item (or item part), counters for keys
// [0, L) in LDS; the sweep reads the item's whole key window.
constexpr int kDirectThreads = 1024;
constexpr int kDirectWaves = kDirectThreads / kWave;
constexpr int kDirectKeys = 32768;

__global__ __launch_bounds__(kDirectThreads) void k_direct(DirectArgs a) {
  __shared__ uint32_t cnt[kDirectKeys];
  __shared__ uint32_t mbase[kDirectWaves][kGather];
  __shared__ uint8_t mtag[kDirectWaves][kGather];
  __shared__ int32_t item_sh;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  for (int i = tid; i < kDirectKeys; i += kDirectThreads) cnt[i] = 0;
  for (int i = tid; i < kDirectWaves * static_cast<int>(kGather); i += kDirectThreads) (&mtag[0][0])[i] = 0;
  Sums sums;
  uint32_t graph = kNoGraph;
  for (;;) {
    if (tid == 0) item_sh = static_cast<int32_t>(atomicAdd(a.queue, 1u));
    __syncthreads();
    const int32_t i = item_sh;
    if (i >= a.n_items) break;
    const Item it = a.items[i];
    if (it.graph != graph) {
      if (graph != kNoGraph) flush_sums(sums, a.res + static_cast<size_t>(graph) * kResStride);
      sums = Sums{};
      graph = it.graph;
    }
    const DevSideConst sc = a.sides[2 * it.graph + it.side];
    const uint32_t* __restrict__ adj = sc.other_adj;
    const uint32_t seg_end = it.seg_begin + it.seg_count;
    for (uint32_t k0 = it.seg_begin + wave * kWave; k0 < seg_end; k0 += kDirectThreads) {
      const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
      walk_batch<4>(sc.segs, k0, k1, adj, Marks<uint8_t>{mbase[wave], mtag[wave]}, a.long_len, DirectTally{cnt});
    }
    __syncthreads();
    if (it.flags & kItemMultiPart) {
      // write the part's counters for the whole key window (zeros included)
      uint32_t* __restrict__ dst = sc.acc + static_cast<size_t>(it.acc_slot) * sc.acc_width;
      for (uint32_t key = it.key_lo + tid; key < static_cast<uint32_t>(it.key_hi); key += kDirectThreads) {
        dst[key] = cnt[key];
        cnt[key] = 0;
      }
    } else {
      const uint32_t lo = static_cast<uint32_t>(it.key_lo) & ~3u;
      const uint32_t hi = static_cast<uint32_t>(it.key_hi);
      for (uint32_t key = lo + 4 * tid; key < hi; key += 4 * kDirectThreads) {
        const uint4 c4 = *reinterpret_cast<uint4*>(&cnt[key]);
        if ((c4.x | c4.y | c4.z | c4.w) == 0) continue;
        const uint32_t cv[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (cv[j]) emit(it, key + j, cv[j] & 0xffffu, cv[j] >> 16, sc, sums);
        *reinterpret_cast<uint4*>(&cnt[key]) = make_uint4(0, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (graph != kNoGraph) flush_sums(sums, a.res + static_cast<size_t>(graph) * kResStride);
}

// ---------------------------------------------------------------------------
// Reverse items: one wavefront per item, a private LDS direct array over the
// reverse window [0, R) (R <= kMaxReverseL).  Counters are 8-bit
// (symmetric | asymmetric << 8) in 16-bit halves, two keys per 32-bit word:
// an item (or part) has at most kReverseMaxSegs segments, so no byte
// overflows.  Items are dealt to wavefronts in a fixed stride; the next
// item's first segments and the descriptor of the one after are loaded while
// the current item is walked.  The sweep reads the whole window with 16-byte
// LDS loads.
constexpr int kReverseThreads = 1024;
constexpr int kReverseWaves = kReverseThreads / kWave;
constexpr int kReverseWords = kMaxReverseL / 2;

// Per-key sums of squares: with W the wedges of the swept keys (sum of
// p + n), sum C(p,2) + C(n,2) = (sum p^2 + n^2 - W) / 2 and the unbalanced
// sum is sum p * n.  24-bit multiply-adds on 32-bit per-item accumulators:
// the callers bound p and n so that an item's sums stay below 2^32.
struct SqSums {
  uint32_t sq = 0, pn = 0, w = 0;
  __device__ __forceinline__ void add(uint32_t p, uint32_t n) {
    sq += __umul24(p, p);
    sq += __umul24(n, n);
    pn += __umul24(p, n);
    w += p + n;
  }
  __device__ __forceinline__ void add_word(uint32_t c2) {  // two 8|8-bit keys
    add(c2 & 0xffu, (c2 >> 8) & 0xffu);
    add((c2 >> 16) & 0xffu, c2 >> 24);
  }
};

// Running per-lane totals of SqSums, flushed once per wavefront.
struct SqTotals {
  uint64_t sq = 0, pn = 0, w = 0;
  __device__ __forceinline__ void add(const SqSums& s) {
    sq += s.sq;
    pn += s.pn;
    w += s.w;
  }
  __device__ __forceinline__ void flush(unsigned long long* res) const {
    const int64_t q = wave_sum64(static_cast<int64_t>(sq));
    const int64_t x = wave_sum64(static_cast<int64_t>(pn));
    const int64_t ww = wave_sum64(static_cast<int64_t>(w));
    if (lane_id() == 0) {
      const int64_t bal = (q - ww) / 2;
      if (bal) atomicAdd(res + kResBalanced, static_cast<unsigned long long>(bal));
      if (x) atomicAdd(res + kResUnbalanced, static_cast<unsigned long long>(x));
      if (bal + x) atomicAdd(res + kResTotal, static_cast<unsigned long long>(bal + x));
    }
  }
};

__global__ __launch_bounds__(kReverseThreads) void k_reverse(SmallArgs a) {
  __shared__ uint32_t cnt[kReverseWaves][kReverseWords];
  __shared__ uint32_t mbase[kReverseWaves][kGather];
  __shared__ uint8_t mtag[kReverseWaves][kGather];
  const int wave = threadIdx.x / kWave;
  const int lane = lane_id();
  uint32_t* C = cnt[wave];
  for (int i = lane; i < kReverseWords; i += kWave) C[i] = 0;
  for (int i = lane; i < static_cast<int>(kGather); i += kWave) mtag[wave][i] = 0;
  wave_sync_lds();
  SqTotals tot;
  const int32_t n = a.n_items;
  const int32_t stride = static_cast<int32_t>(gridDim.x) * kReverseWaves;
  int32_t i = static_cast<int32_t>(blockIdx.x) * kReverseWaves + wave;
  Item cur{}, nxt{};
  SegReg cfirst{0, 0, 0};
  if (i < n) {
    cur = a.items[i];
    cfirst = first_batch(cur, a.sides[2 * cur.graph + cur.side].segs);
  }
  if (i + stride < n) nxt = a.items[i + stride];
  uint32_t graph = kNoGraph;
  for (; i < n; i += stride) {
    const Item it = cur;
    const SegReg first = cfirst;
    const int32_t j = i + stride, j2 = j + stride;
    if (it.graph != graph) {
      if (graph != kNoGraph) tot.flush(a.res + static_cast<size_t>(graph) * kResStride);
      tot = SqTotals{};
      graph = it.graph;
    }
    SegReg nfirst{0, 0, 0};
    if (j < n) nfirst = first_batch(nxt, a.sides[2 * nxt.graph + nxt.side].segs);
    Item nxt2{};
    if (j2 < n) nxt2 = a.items[j2];
    const DevSideConst sc = a.sides[2 * it.graph + it.side];
    walk_item<8>(it, first, sc.segs, sc.other_adj, Marks<uint8_t>{mbase[wave], mtag[wave]}, a.long_len,
                 PairTally{C});
    wave_sync_lds();
    const int32_t w_hi = (it.key_hi + 1) >> 1;  // counter words of the item's keys
    if (it.flags & kItemMultiPart) {
      uint32_t* __restrict__ dst = sc.acc + static_cast<size_t>(it.acc_slot) * sc.acc_width;
      for (int32_t wd = lane; wd < w_hi; wd += kWave) {
        const uint32_t c2 = C[wd];
        C[wd] = 0;
        dst[2 * wd] = (c2 & 0xffu) | (((c2 >> 8) & 0xffu) << 16);
        if (2 * wd + 1 < it.key_hi) dst[2 * wd + 1] = ((c2 >> 16) & 0xffu) | ((c2 >> 24) << 16);
      }
    } else {
      // p, n <= 255 and at most 2 * kReverseWords / 64 = 64 keys per lane
      SqSums ss;
      for (int32_t wd = 4 * lane; wd < w_hi; wd += 4 * kWave) {
        const uint4 c4 = *reinterpret_cast<uint4*>(&C[wd]);
        if ((c4.x | c4.y | c4.z | c4.w) == 0) continue;
        *reinterpret_cast<uint4*>(&C[wd]) = make_uint4(0, 0, 0, 0);
        ss.add_word(c4.x);
        ss.add_word(c4.y);
        ss.add_word(c4.z);
        ss.add_word(c4.w);
      }
      tot.add(ss);
    }
    wave_sync_lds();
    cur = nxt;
    cfirst = nfirst;
    nxt = nxt2;
  }
  if (graph != kNoGraph) tot.flush(a.res + static_cast<size_t>(graph) * kResStride);
}

// ---------------------------------------------------------------------------
// Small items, packed into groups (see plan.cpp): one wavefront per group,
// an open-addressing hash in LDS keyed by (item index in the group <<
// key_bits) | key, with 16 | 16-bit counts (a group has at most
// kSmallGroupWork wedges).  The table is sized to the group (a power of two
// at least twice its wedges), so the sweep reads only that many slots.
constexpr int kSmallThreads = 256;
constexpr int kSmallWaves = kSmallThreads / kWave;
constexpr int kSmallSlots = 2 * kSmallGroupWork;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(kSmallThreads) void k_small(SmallArgs a) {
  __shared__ uint32_t keys[kSmallWaves][kSmallSlots];
  __shared__ uint32_t vals[kSmallWaves][kSmallSlots];
  __shared__ uint32_t marks[kSmallWaves][2][kGather];
  const int wave = threadIdx.x / kWave;
  const int lane = lane_id();
  uint32_t* K = keys[wave];
  uint32_t* Vv = vals[wave];
  for (int i = lane; i < kSmallSlots; i += kWave) {
    K[i] = kEmpty;
    Vv[i] = 0;
  }
  for (int i = lane; i < 2 * static_cast<int>(kGather); i += kWave) (&marks[wave][0][0])[i] = 0;
  wave_sync_lds();
  SqTotals tot;
  const int32_t stride = static_cast<int32_t>(gridDim.x) * kSmallWaves;
  int32_t i = static_cast<int32_t>(blockIdx.x) * kSmallWaves + wave;
  Item nxt{};
  SegReg nfirst{0, 0, 0};
  if (i < a.n_items) {
    nxt = a.items[i];
    nfirst = first_batch<true>(nxt, a.sides[2 * nxt.graph + nxt.side].small_segs);
  }
  uint32_t graph = kNoGraph;
  for (; i < a.n_items; i += stride) {
    const Item it = nxt;
    const SegReg first = nfirst;
    const int32_t j = i + stride;
    if (j < a.n_items) nxt = a.items[j];
    if (it.graph != graph) {
      if (graph != kNoGraph) tot.flush(a.res + static_cast<size_t>(graph) * kResStride);
      tot = SqTotals{};
      graph = it.graph;
    }
    const DevSideConst sc = a.sides[2 * it.graph + it.side];
    const uint32_t kb = static_cast<uint32_t>(sc.key_bits);
    // table size: a power of two >= 2 * work, at least 64
    uint32_t size = 64;
    while (size < 2 * it.work) size <<= 1;
    const uint32_t mask = size - 1;
    walk_item<4, true>(it, first, sc.small_segs, sc.other_adj, Marks<uint32_t>{marks[wave][0], marks[wave][1]},
                       a.long_len,
                       hash_tally([&](uint32_t e, uint32_t tag) {
                         const uint32_t key = ((tag >> 1) << kb) | (e >> 1);
                         const uint32_t inc = wedge_inc(e, tag);
                         uint32_t h = mix32(key) & mask;
                         for (uint32_t probe = 0;; ++probe) {
                           if (probe > mask) {  // full table: cannot happen at load <= 1/2
                             atomicOr(a.err, kErrHashFull);
                             break;
                           }
                           uint32_t c = K[h];
                           if (c == kEmpty) {
                             c = atomicCAS(&K[h], kEmpty, key);
                             if (c == kEmpty) c = key;
                           }
                           if (c == key) {
                             atomicAdd(&Vv[h], inc);
                             break;
                           }
                           h = (h + 1) & mask;
                         }
                       }));
    if (j < a.n_items) nfirst = first_batch<true>(nxt, a.sides[2 * nxt.graph + nxt.side].small_segs);
    wave_sync_lds();
    // p, n <= kSmallGroupWork per key and sum p + n <= kSmallGroupWork
    // per group, so the group's sums of squares stay below 2^19
    SqSums ss;
    const bool hub = (it.flags & kItemHubPairs) != 0;
    const uint32_t kmask = (1u << kb) - 1u;
    for (uint32_t h = lane; h < size; h += kWave) {
      const uint32_t key = K[h];
      if (key != kEmpty) {
        const uint32_t c = Vv[h];
        const uint32_t p = c & 0xffffu, q = c >> 16;
        K[h] = kEmpty;
        Vv[h] = 0;
        if (hub && static_cast<int32_t>(key & kmask) < sc.T)  // singleton group
          sc.hub_pairs[static_cast<size_t>(it.owner) * sc.T + (key & kmask)] =
              (static_cast<unsigned long long>(q) << 32) | p;
        else
          ss.add(p, q);
      }
    }
    tot.add(ss);
    wave_sync_lds();
  }
  if (graph != kNoGraph) tot.flush(a.res + static_cast<size_t>(graph) * kResStride);
}

// ---------------------------------------------------------------------------
// Large items below the window: one workgroup per item, a shared hash table
// with 32-bit symmetric and asymmetric counts; items with more distinct
// endpoints than fit are walked once per key-hash partition.
constexpr int kHashThreads = 512;
constexpr int kHashWaves = kHashThreads / kWave;
constexpr int kHashSlots = 8192;

__global__ __launch_bounds__(kHashThreads) void k_hash(HashArgs a) {
  __shared__ uint32_t keys[kHashSlots];
  __shared__ unsigned long long vals[kHashSlots];
  __shared__ uint32_t mbase[kHashWaves][kGather];
  __shared__ uint8_t mtag[kHashWaves][kGather];
  __shared__ int32_t item_sh;
  __shared__ uint32_t work_sh;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  for (int i = tid; i < kHashSlots; i += kHashThreads) {
    keys[i] = kEmpty;
    vals[i] = 0;
  }
  for (int i = tid; i < kHashWaves * static_cast<int>(kGather); i += kHashThreads) (&mtag[0][0])[i] = 0;
  Sums sums;
  uint32_t graph = kNoGraph;
  for (;;) {
    if (tid == 0) {
      item_sh = static_cast<int32_t>(atomicAdd(a.queue, 1u));
      work_sh = 0;
    }
    __syncthreads();
    const int32_t i = item_sh;
    if (i >= a.n_items) break;
    const Item it = a.items[i];
    if (it.graph != graph) {
      if (graph != kNoGraph) flush_sums(sums, a.res + static_cast<size_t>(graph) * kResStride);
      sums = Sums{};
      graph = it.graph;
    }
    const DevSideConst sc = a.sides[2 * it.graph + it.side];
    const uint32_t seg_end = it.seg_begin + it.seg_count;
    uint32_t w = 0;
    for (uint32_t k = it.seg_begin + tid; k < seg_end; k += kHashThreads) w += sc.segs[k].len_g >> 1;
    atomicAdd(&work_sh, w);
    __syncthreads();
    const uint32_t work = work_sh;
    // about kHashSlots / 4 distinct keys per pass at most on average
    const uint32_t passes = (work + kHashSlots / 4 - 1) / (kHashSlots / 4);
    for (uint32_t pass = 0; pass < passes; ++pass) {
      for (uint32_t k0 = it.seg_begin + wave * kWave; k0 < seg_end; k0 += kHashThreads) {
        const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
        walk_batch<4>(sc.segs, k0, k1, sc.other_adj, Marks<uint8_t>{mbase[wave], mtag[wave]}, a.long_len, hash_tally([&](uint32_t e, uint32_t g) {
          const uint32_t key = e >> 1;
          const uint32_t hk = mix32(key);
          if (passes > 1 && (hk >> 16) % passes != pass) return;
          const unsigned long long inc = ((e ^ g) & 1u) ? (1ull << 32) : 1ull;
          uint32_t h = hk & (kHashSlots - 1);
          for (uint32_t probe = 0;; ++probe) {
            if (probe >= static_cast<uint32_t>(kHashSlots)) {  // full table
              atomicOr(a.err, kErrHashFull);
              break;
            }
            uint32_t cur = keys[h];
            if (cur == kEmpty) {
              cur = atomicCAS(&keys[h], kEmpty, key);
              if (cur == kEmpty) cur = key;
            }
            if (cur == key) {
              atomicAdd(&vals[h], inc);
              break;
            }
            h = (h + 1) & (kHashSlots - 1);
          }
        }));
      }
      __syncthreads();
      for (int h = tid; h < kHashSlots; h += kHashThreads) {
        const uint32_t key = keys[h];
        if (key != kEmpty) {
          const unsigned long long c = vals[h];
          emit(it, key, static_cast<uint32_t>(c), static_cast<uint32_t>(c >> 32), sc, sums);
          keys[h] = kEmpty;
          vals[h] = 0;
        }
      }
      __syncthreads();
    }
  }
  if (graph != kNoGraph) flush_sums(sums, a.res + static_cast<size_t>(graph) * kResStride);
}

// ---------------------------------------------------------------------------
// Multi-part pivots: add the parts' packed counters key by key, then take
// C(., 2) of the combined counts.
constexpr int kReduceThreads = 256;

__global__ __launch_bounds__(kReduceThreads) void k_reduce(ReduceArgs a) {
  Sums sums;
  uint32_t graph = kNoGraph;
  for (int32_t r = blockIdx.x; r < a.n_reduces; r += gridDim.x) {
    const Reduce rd = a.reduces[r];
    if (rd.graph != graph) {
      if (graph != kNoGraph) flush_sums(sums, a.res + static_cast<size_t>(graph) * kResStride);
      sums = Sums{};
      graph = rd.graph;
    }
    const DevSideConst sc = a.sides[2 * rd.graph + rd.side];
    Item it{};
    it.owner = rd.owner;
    it.flags = rd.flags;
    for (int32_t key = rd.key_lo + threadIdx.x; key < rd.key_hi; key += kReduceThreads) {
      uint32_t p = 0, n = 0;
      for (int32_t j = 0; j < rd.n_parts; ++j) {
        const uint32_t c = sc.acc[static_cast<size_t>(rd.acc_slot + j) * sc.acc_width + key];
        p += c & 0xffffu;
        n += c >> 16;
      }
      if (p | n) emit(it, static_cast<uint32_t>(key), p, n, sc, sums);
    }
  }
  if (graph != kNoGraph) flush_sums(sums, a.res + static_cast<size_t>(graph) * kResStride);
}

// Batch assembly: block b copies graph b's list, setting the graph index.
template <class T>
__global__ void k_assemble(const AssembleSrc* __restrict__ srcs, T* __restrict__ dst) {
  const AssembleSrc s = srcs[blockIdx.x];
  const T* __restrict__ src = static_cast<const T*>(s.src);
  for (uint32_t i = threadIdx.x; i < s.n; i += blockDim.x) {
    T v = src[i];
    v.graph = s.graph;
    dst[s.dst_off + i] = v;
  }
}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

}  // namespace dev

// ---- launchers ------------------------------------------------------------------

hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(dev::k_fill_u64, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_assemble_items(const AssembleSrc* srcs, int k, Item* dst, hipStream_t st) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_assemble<Item>, dim3(k), dim3(256), 0, st, srcs, dst);
  return hipGetLastError();
}

hipError_t launch_assemble_reduces(const AssembleSrc* srcs, int k, Reduce* dst, hipStream_t st) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_assemble<Reduce>, dim3(k), dim3(256), 0, st, srcs, dst);
  return hipGetLastError();
}

hipError_t launch_direct(const DirectArgs& a, int grid, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_direct, dim3(grid), dim3(dev::kDirectThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_reverse(const SmallArgs& a, int grid, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_reverse, dim3(grid), dim3(dev::kReverseThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_small(const SmallArgs& a, int grid, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_small, dim3(grid), dim3(dev::kSmallThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_hash(const HashArgs& a, int grid, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_hash, dim3(grid), dim3(dev::kHashThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, int grid, hipStream_t st) {
  if (a.n_reduces == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_reduce, dim3(grid), dim3(dev::kReduceThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace dbbc
