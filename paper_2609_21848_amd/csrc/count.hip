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
constexpr uint32_t kLong = 16;     // segments this long are streamed by the whole wavefront
constexpr uint32_t kChunk = 256;   // entries per wavefront 16-byte load (64 lanes x 4)
constexpr uint32_t kGather = 256;  // per-wavefront staging slots for short segments
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

// One lane's segment of a batch (len 0 = none).
struct SegReg {
  uint32_t start, len, g;
};

__device__ __forceinline__ SegReg load_seg(const Segment* __restrict__ segs, uint32_t k0, uint32_t k1) {
  const uint32_t k = k0 + lane_id();
  SegReg r{0, 0, 0};
  if (k < k1) {
    const Segment s = segs[k];
    r.start = s.start;
    r.len = s.len_g >> 1;
    r.g = s.len_g & 1u;
  }
  return r;
}

// Stage the short-segment wedges with flat positions [done, done + G) of the
// batch into gbuf as (entry index | g << 31).
template <int G>
__device__ __forceinline__ void stage_short(uint32_t* gbuf, uint32_t excl, uint32_t slen, uint32_t start,
                                            uint32_t g, uint32_t done) {
  const uint32_t lo = excl > done ? excl : done;
  const uint32_t hi_a = excl + slen, hi_b = done + G;
  const uint32_t hi = hi_a < hi_b ? hi_a : hi_b;
  for (uint32_t t = lo; t < hi; ++t) gbuf[t - done] = (start + (t - excl)) | (g << 31);
}

// Walk a batch of up to 64 segments (one per lane, in registers) with one
// wavefront, calling f.add(entry, g, valid) once per wedge slot.
//  - Segments of at least kLong entries are consumed as a stream of
//    256-entry chunks: every lane loads 4 aligned entries (16 bytes) per
//    chunk, U chunks are in flight per lane, and a chunk's out-of-segment
//    words are masked.  The chunk loop is wavefront-uniform.
//  - Shorter segments are staged through gbuf (G words of LDS owned by this
//    wavefront) so that lanes read consecutive wedges.  The loads of the
//    first G staged wedges are issued before the long-segment stream, so the
//    two paths wait on memory together.
template <int U, int G, class F>
__device__ __forceinline__ void walk_regs(SegReg sr, const uint32_t* __restrict__ adj, uint32_t* gbuf,
                                          F&& f) {
  constexpr int UG = G / kWave;
  const int lane = lane_id();
  const uint32_t start = sr.start, g = sr.g, len = sr.len;
  uint64_t longm = __ballot(len >= kLong);
  const uint32_t slen = len >= kLong ? 0u : len;
  uint32_t total;
  const uint32_t excl = wave_excl_scan(slen, &total);
  const uint32_t cnt0 = total < static_cast<uint32_t>(G) ? total : static_cast<uint32_t>(G);
  uint32_t sa[UG], se[UG];
  if (total) {
    stage_short<G>(gbuf, excl, slen, start, g, 0);
    wave_sync_lds();
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      const uint32_t t = u * kWave + lane;
      sa[u] = gbuf[t < cnt0 ? t : 0u];
      se[u] = adj[t < cnt0 ? sa[u] & 0x7fffffffu : 0u];
    }
  }
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
        cur_g = readlane(g, j);
        cur_pos = cur_st & ~3u;
        have = true;
      }
      // The load is unconditional (no wait on registers of a skipped load):
      // lanes past the segment end and empty slots read the first entries of
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
  if (!total) return;
#pragma unroll
  for (int u = 0; u < UG; ++u) f.add(se[u], sa[u] >> 31, u * kWave + lane < cnt0);
  for (uint32_t done = G; done < total; done += G) {
    wave_sync_lds();
    stage_short<G>(gbuf, excl, slen, start, g, done);
    wave_sync_lds();
    const uint32_t cnt = total - done < static_cast<uint32_t>(G) ? total - done : static_cast<uint32_t>(G);
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      const uint32_t t = u * kWave + lane;
      sa[u] = gbuf[t < cnt ? t : 0u];
      se[u] = adj[t < cnt ? sa[u] & 0x7fffffffu : 0u];
    }
#pragma unroll
    for (int u = 0; u < UG; ++u) f.add(se[u], sa[u] >> 31, u * kWave + lane < cnt);
  }
  wave_sync_lds();
}

template <int U, int G = kGather, class F>
__device__ __forceinline__ void walk_batch(const Segment* __restrict__ segs, uint32_t k0, uint32_t k1,
                                           const uint32_t* __restrict__ adj, uint32_t* gbuf, F&& f) {
  walk_regs<U, G>(load_seg(segs, k0, k1), adj, gbuf, f);
}

// Walk every segment of an item with one wavefront; the first batch of 64
// segments was loaded beforehand (first).
template <int U, int G = kGather, class F>
__device__ __forceinline__ void walk_item(const Item& it, SegReg first, const Segment* __restrict__ segs,
                                          const uint32_t* __restrict__ adj, uint32_t* gbuf, F&& f) {
  const uint32_t seg_end = it.seg_begin + it.seg_count;
  walk_regs<U, G>(first, adj, gbuf, f);
  for (uint32_t k0 = it.seg_begin + kWave; k0 < seg_end; k0 += kWave) {
    const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
    walk_regs<U, G>(load_seg(segs, k0, k1), adj, gbuf, f);
  }
}

__device__ __forceinline__ SegReg first_batch(const Item& it, const Segment* __restrict__ segs) {
  const uint32_t seg_end = it.seg_begin + it.seg_count;
  return load_seg(segs, it.seg_begin, it.seg_begin + kWave < seg_end ? it.seg_begin + kWave : seg_end);
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
    if (valid) atomicAdd(&cnt[e >> 2], 1u << (((e ^ g) & 3u) << 3));
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

__device__ __forceinline__ int64_t wave_sum64(int64_t x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

// Add the wavefront's sums to res[0..2] (one atomic per wavefront).
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
  __shared__ uint32_t gbuf[kDirectWaves][kGather];
  __shared__ int32_t item_sh;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  for (int i = tid; i < kDirectKeys; i += kDirectThreads) cnt[i] = 0;
  // staged slots always hold valid entry indices
  for (int i = tid; i < kDirectWaves * static_cast<int>(kGather); i += kDirectThreads) (&gbuf[0][0])[i] = 0;
  Sums sums;
  for (;;) {
    if (tid == 0) item_sh = static_cast<int32_t>(atomicAdd(a.queue, 1u));
    __syncthreads();
    const int32_t i = item_sh;
    if (i >= a.n_items) break;
    const Item it = a.items[i];
    const DevSideConst sc = a.side[it.side];
    const uint32_t* __restrict__ adj = sc.other_adj;
    const uint32_t seg_end = it.seg_begin + it.seg_count;
    for (uint32_t k0 = it.seg_begin + wave * kWave; k0 < seg_end; k0 += kDirectThreads) {
      const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
      walk_batch<4>(a.segs, k0, k1, adj, gbuf[wave], DirectTally{cnt});
    }
    __syncthreads();
    if (it.flags & kItemMultiPart) {
      // write the part's counters for the whole key window (zeros included)
      uint32_t* __restrict__ dst = a.acc + static_cast<size_t>(it.acc_slot) * a.acc_width;
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
  flush_sums(sums, a.res);
}

// ---------------------------------------------------------------------------
// Reverse items: one wavefront per item, a private LDS direct array over the
// reverse window [0, R) (R <= kMaxReverseL).  Counters are 8-bit
// (symmetric | asymmetric << 8) in 16-bit halves, two keys per 32-bit word:
// an item (or part) has at most kReverseMaxSegs segments, so no byte
// overflows.  Items flagged kItemMidHash also carry a few keys in [R, L);
// those go to a per-wavefront hash whose 32-bit slots hold
// (key - R + 1) << 16 | asymmetric << 8 | symmetric.
// Items are dealt to wavefronts in a fixed stride; the next item's first
// segments and the descriptor of the one after are loaded while the current
// item is walked.  The sweep reads the whole window with 16-byte LDS loads.
constexpr int kReverseThreads = 1024;
constexpr int kReverseWaves = kReverseThreads / kWave;
constexpr int kReverseWords = kMaxReverseL / 2;
constexpr int kReverseGather = 256;

// Reverse items sum, per key, p^2 + n^2 and p * n (24-bit multiply-adds on
// 32-bit per-item accumulators: at most 64 keys per lane of <= 255 each).
// With W = sum of p + n over the item (its wedge count), the item adds
// (sum p^2 + n^2 - W) / 2 = sum C(p,2) + C(n,2) balanced butterflies and
// sum p * n unbalanced ones; the halving is done once per wavefront.
struct SqSums {
  uint32_t sq = 0, pn = 0;
  __device__ __forceinline__ void add(uint32_t p, uint32_t n) {
    sq += __umul24(p, p);
    sq += __umul24(n, n);
    pn += __umul24(p, n);
  }
  __device__ __forceinline__ void add_word(uint32_t c2) {  // two keys
    add(c2 & 0xffu, (c2 >> 8) & 0xffu);
    add((c2 >> 16) & 0xffu, c2 >> 24);
  }
};

struct RevTally {
  uint32_t* cnt;
  uint32_t* hsh;
  uint32_t R;
  unsigned long long* res;
  __device__ __forceinline__ void add(uint32_t e, uint32_t g, bool valid) const {
    if (!valid) return;
    const uint32_t key = e >> 1;
    if (key < R) {
      // bit 0 (negative) ^ g picks the symmetric / asymmetric byte, bit 1
      // (key parity) the 16-bit half of the word
      atomicAdd(&cnt[e >> 2], 1u << (((e ^ g) & 3u) << 3));
      return;
    }
    const uint32_t k = key - R + 1;
    const uint32_t inc = ((e ^ g) & 1u) ? 0x100u : 1u;
    uint32_t h = (k * 0x9e3779b1u) >> 24;
    for (int probe = 0; probe < kMidHashSlots; ++probe) {
      const uint32_t cur = hsh[h];
      if ((cur >> 16) == k) {
        atomicAdd(&hsh[h], inc);
        return;
      }
      if (cur == 0) {
        const uint32_t old = atomicCAS(&hsh[h], 0u, (k << 16) | inc);
        if (old == 0) return;
        if ((old >> 16) == k) {
          atomicAdd(&hsh[h], inc);
          return;
        }
      }
      h = (h + 1) & (kMidHashSlots - 1);
    }
    atomicOr(res + kResError, kErrHashFull);  // cannot happen at load <= 1/2
  }
};

__global__ __launch_bounds__(kReverseThreads) void k_reverse(SmallArgs a) {
  __shared__ uint32_t cnt[kReverseWaves][kReverseWords];
  __shared__ uint32_t hsh[kReverseWaves][kMidHashSlots];
  __shared__ uint32_t gbuf[kReverseWaves][kReverseGather];
  const int wave = threadIdx.x / kWave;
  const int lane = lane_id();
  uint32_t* C = cnt[wave];
  uint32_t* H = hsh[wave];
  for (int i = lane; i < kReverseWords; i += kWave) C[i] = 0;
  for (int i = lane; i < kMidHashSlots; i += kWave) H[i] = 0;
  for (int i = lane; i < kReverseGather; i += kWave) gbuf[wave][i] = 0;
  wave_sync_lds();
  uint64_t sq_total = 0, pn_total = 0;  // per lane
  uint64_t w_total = 0;                 // wavefront-uniform: wedges of swept items
  const int32_t n = a.n_items;
  const int32_t stride = static_cast<int32_t>(gridDim.x) * kReverseWaves;
  int32_t i = static_cast<int32_t>(blockIdx.x) * kReverseWaves + wave;
  Item cur{}, nxt{};
  SegReg cfirst{0, 0, 0};
  if (i < n) {
    cur = a.items[i];
    cfirst = first_batch(cur, a.segs);
  }
  if (i + stride < n) nxt = a.items[i + stride];
  for (; i < n; i += stride) {
    const Item it = cur;
    const SegReg first = cfirst;
    const int32_t j = i + stride, j2 = j + stride;
    SegReg nfirst{0, 0, 0};
    if (j < n) nfirst = first_batch(nxt, a.segs);
    Item nxt2{};
    if (j2 < n) nxt2 = a.items[j2];
    const DevSideConst sc = a.side[it.side];
    if (it.flags & kItemMidHash)
      walk_item<8, kReverseGather>(it, first, a.segs, sc.other_adj, gbuf[wave],
                                   RevTally{C, H, static_cast<uint32_t>(sc.R), a.res});
    else
      walk_item<8, kReverseGather>(it, first, a.segs, sc.other_adj, gbuf[wave], PairTally{C});
    wave_sync_lds();
    const int32_t kh = it.key_hi < sc.R ? it.key_hi : sc.R;
    const int32_t w_hi = (kh + 1) >> 1;  // counter words of the direct window
    if (it.flags & kItemMultiPart) {
      uint32_t* __restrict__ dst = a.acc + static_cast<size_t>(it.acc_slot) * a.acc_width;
      for (int32_t wd = lane; wd < w_hi; wd += kWave) {
        const uint32_t c2 = C[wd];
        C[wd] = 0;
        dst[2 * wd] = (c2 & 0xffu) | (((c2 >> 8) & 0xffu) << 16);
        if (2 * wd + 1 < kh) dst[2 * wd + 1] = ((c2 >> 16) & 0xffu) | ((c2 >> 24) << 16);
      }
    } else {
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
      if (it.flags & kItemMidHash) {
        const uint4 h4 = *reinterpret_cast<uint4*>(&H[4 * lane]);
        if (h4.x | h4.y | h4.z | h4.w) {
          *reinterpret_cast<uint4*>(&H[4 * lane]) = make_uint4(0, 0, 0, 0);
          // slot = key << 16 | asym << 8 | sym: the low half is a counter word
          ss.add(h4.x & 0xffu, (h4.x >> 8) & 0xffu);
          ss.add(h4.y & 0xffu, (h4.y >> 8) & 0xffu);
          ss.add(h4.z & 0xffu, (h4.z >> 8) & 0xffu);
          ss.add(h4.w & 0xffu, (h4.w >> 8) & 0xffu);
        }
      }
      sq_total += ss.sq;
      pn_total += ss.pn;
      w_total += it.work;
    }
    wave_sync_lds();
    cur = nxt;
    cfirst = nfirst;
    nxt = nxt2;
  }
  const int64_t sq = wave_sum64(static_cast<int64_t>(sq_total));
  const int64_t pn = wave_sum64(static_cast<int64_t>(pn_total));
  if (lane == 0) {
    const int64_t bal = (sq - static_cast<int64_t>(w_total)) / 2;
    if (bal) atomicAdd(a.res + kResBalanced, static_cast<unsigned long long>(bal));
    if (pn) atomicAdd(a.res + kResUnbalanced, static_cast<unsigned long long>(pn));
    if (bal + pn) atomicAdd(a.res + kResTotal, static_cast<unsigned long long>(bal + pn));
  }
}

// ---------------------------------------------------------------------------
// Small items: one wavefront per item, open-addressing hash counters in LDS
// sized to the item (at least twice its wedge count).
constexpr int kSmallThreads = 256;
constexpr int kSmallWaves = kSmallThreads / kWave;
constexpr int kSmallSlots = 2048;  // per wavefront, >= 2 * max small work (1024)

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
  __shared__ uint32_t gbuf[kSmallWaves][kGather];
  const int wave = threadIdx.x / kWave;
  const int lane = lane_id();
  uint32_t* K = keys[wave];
  uint32_t* Vv = vals[wave];
  for (int i = lane; i < kSmallSlots; i += kWave) {
    K[i] = kEmpty;
    Vv[i] = 0;
  }
  for (int i = lane; i < static_cast<int>(kGather); i += kWave) gbuf[wave][i] = 0;
  wave_sync_lds();
  Sums sums;
  const int32_t stride = static_cast<int32_t>(gridDim.x) * kSmallWaves;
  int32_t i = static_cast<int32_t>(blockIdx.x) * kSmallWaves + wave;
  Item nxt{};
  SegReg nfirst{0, 0, 0};
  if (i < a.n_items) {
    nxt = a.items[i];
    nfirst = first_batch(nxt, a.segs);
  }
  for (; i < a.n_items; i += stride) {
    const Item it = nxt;
    const SegReg first = nfirst;
    const int32_t j = i + stride;
    if (j < a.n_items) nxt = a.items[j];
    const DevSideConst sc = a.side[it.side];
    // table size: a power of two >= 2 * work, at least 64
    uint32_t size = 64;
    while (size < 2 * it.work) size <<= 1;
    const uint32_t mask = size - 1;
    {
      walk_item<4>(it, first, a.segs, sc.other_adj, gbuf[wave], hash_tally([&](uint32_t e, uint32_t g) {
        const uint32_t key = e >> 1;
        const uint32_t inc = wedge_inc(e, g);
        uint32_t h = mix32(key) & mask;
        for (uint32_t probe = 0;; ++probe) {
          if (probe > mask) {  // full table: cannot happen at load <= 1/2
            atomicOr(a.res + kResError, kErrHashFull);
            break;
          }
          uint32_t cur = K[h];
          if (cur == kEmpty) {
            cur = atomicCAS(&K[h], kEmpty, key);
            if (cur == kEmpty) cur = key;
          }
          if (cur == key) {
            atomicAdd(&Vv[h], inc);
            break;
          }
          h = (h + 1) & mask;
        }
      }));
    }
    if (j < a.n_items) nfirst = first_batch(nxt, a.segs);
    wave_sync_lds();
    for (uint32_t h = lane; h < size; h += kWave) {
      const uint32_t key = K[h];
      if (key != kEmpty) {
        const uint32_t c = Vv[h];
        emit(it, key, c & 0xffffu, c >> 16, sc, sums);
        K[h] = kEmpty;
        Vv[h] = 0;
      }
    }
    wave_sync_lds();
  }
  flush_sums(sums, a.res);
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
  __shared__ uint32_t gbuf[kHashWaves][kGather];
  __shared__ int32_t item_sh;
  __shared__ uint32_t work_sh;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  for (int i = tid; i < kHashSlots; i += kHashThreads) {
    keys[i] = kEmpty;
    vals[i] = 0;
  }
  for (int i = tid; i < kHashWaves * static_cast<int>(kGather); i += kHashThreads) (&gbuf[0][0])[i] = 0;
  Sums sums;
  for (;;) {
    if (tid == 0) {
      item_sh = static_cast<int32_t>(atomicAdd(a.queue, 1u));
      work_sh = 0;
    }
    __syncthreads();
    const int32_t i = item_sh;
    if (i >= a.n_items) break;
    const Item it = a.items[i];
    const DevSideConst sc = a.side[it.side];
    const uint32_t seg_end = it.seg_begin + it.seg_count;
    uint32_t w = 0;
    for (uint32_t k = it.seg_begin + tid; k < seg_end; k += kHashThreads) w += a.segs[k].len_g >> 1;
    atomicAdd(&work_sh, w);
    __syncthreads();
    const uint32_t work = work_sh;
    // about kHashSlots / 4 distinct keys per pass at most on average
    const uint32_t passes = (work + kHashSlots / 4 - 1) / (kHashSlots / 4);
    for (uint32_t pass = 0; pass < passes; ++pass) {
      for (uint32_t k0 = it.seg_begin + wave * kWave; k0 < seg_end; k0 += kHashThreads) {
        const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
        walk_batch<4>(a.segs, k0, k1, sc.other_adj, gbuf[wave], hash_tally([&](uint32_t e, uint32_t g) {
          const uint32_t key = e >> 1;
          const uint32_t hk = mix32(key);
          if (passes > 1 && (hk >> 16) % passes != pass) return;
          const unsigned long long inc = ((e ^ g) & 1u) ? (1ull << 32) : 1ull;
          uint32_t h = hk & (kHashSlots - 1);
          for (uint32_t probe = 0;; ++probe) {
            if (probe >= static_cast<uint32_t>(kHashSlots)) {  // full table
              atomicOr(a.res + kResError, kErrHashFull);
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
  flush_sums(sums, a.res);
}

// ---------------------------------------------------------------------------
// Multi-part pivots: add the parts' packed counters key by key, then take
// C(., 2) of the combined counts.
constexpr int kReduceThreads = 256;

__global__ __launch_bounds__(kReduceThreads) void k_reduce(ReduceArgs a) {
  Sums sums;
  for (int32_t r = blockIdx.x; r < a.n_reduces; r += gridDim.x) {
    const Reduce rd = a.reduces[r];
    const DevSideConst sc = a.side[rd.side];
    Item it{};
    it.owner = rd.owner;
    it.flags = rd.flags;
    for (int32_t key = rd.key_lo + threadIdx.x; key < rd.key_hi; key += kReduceThreads) {
      uint32_t p = 0, n = 0;
      for (int32_t j = 0; j < rd.n_parts; ++j) {
        const uint32_t c = a.acc[static_cast<size_t>(rd.acc_slot + j) * a.acc_width + key];
        p += c & 0xffffu;
        n += c >> 16;
      }
      if (p | n) emit(it, static_cast<uint32_t>(key), p, n, sc, sums);
    }
  }
  flush_sums(sums, a.res);
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
