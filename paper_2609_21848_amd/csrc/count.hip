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
#include "walk.h"

namespace dbbc {
namespace dev {

// ---------------------------------------------------------------------------
// Window items: one workgroup per item (or item part), counters for keys
// [0, L) in LDS; the sweep reads the item's whole key window.
constexpr int kDirectThreads = 1024;
constexpr int kDirectWaves = kDirectThreads / kWave;
constexpr int kDirectKeys = 32768;
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(kDirectThreads) void k_direct(DirectArgs a) {
  __shared__ uint32_t cnt[kDirectKeys + kDirectThreads];  // counters, then one dummy per thread
  __shared__ __attribute__((aligned(16))) uint32_t mtab[kDirectWaves][kGather];
  __shared__ uint8_t mflag[kDirectWaves][kGather];
  __shared__ int32_t item_sh;
  __shared__ unsigned long long blk[2];
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  for (int i = tid; i < kDirectKeys; i += kDirectThreads) cnt[i] = 0;
  for (int i = tid; i < kDirectWaves * static_cast<int>(kGather); i += kDirectThreads) (&mflag[0][0])[i] = 0;
  if (tid == 0) blk[0] = blk[1] = 0;
  // Per thread, for the current graph: twice the balanced count (sum of
  // p^2 + n^2 minus the wedges) and the unbalanced count.  Only the
  // workgroup's total of sq2 is even, so the halving happens there.
  int64_t sq2 = 0;
  uint64_t pnx = 0;
  auto flush_block = [&](uint32_t g) {
    const int64_t q = wave_sum64(sq2), x = wave_sum64(static_cast<int64_t>(pnx));
    if ((tid & (kWave - 1)) == 0) {
      atomicAdd(&blk[0], static_cast<unsigned long long>(q));
      atomicAdd(&blk[1], static_cast<unsigned long long>(x));
    }
    __syncthreads();
    if (tid == 0) {
      const int64_t bal = static_cast<int64_t>(blk[0]) / 2, unb = static_cast<int64_t>(blk[1]);
      unsigned long long* res = a.res + static_cast<size_t>(g) * kResStride;
      if (bal) atomicAdd(res + kResBalanced, static_cast<unsigned long long>(bal));
      if (unb) atomicAdd(res + kResUnbalanced, static_cast<unsigned long long>(unb));
      if (bal + unb) atomicAdd(res + kResTotal, static_cast<unsigned long long>(bal + unb));
      blk[0] = blk[1] = 0;
    }
    __syncthreads();
    sq2 = 0;
    pnx = 0;
  };
  uint32_t graph = kNoGraph;
  for (;;) {
    if (tid == 0) item_sh = static_cast<int32_t>(atomicAdd(a.queue, 1u));
    __syncthreads();
    const int32_t i = item_sh;
    if (i >= a.n_items) break;
    const Item it = load_const(a.items, i);
    if (it.graph != graph) {
      if (graph != kNoGraph) flush_block(graph);
      graph = it.graph;
    }
    const DevSideConst sc = load_const(a.sides, 2 * it.graph + it.side);
    const uint32_t* __restrict__ adj = sc.other_adj;
    const uint32_t seg_end = it.seg_begin + it.seg_count;
    // the wavefronts take the item's segments interleaved (wavefront w the
    // segments w, w + 16, ...), 64 per batch, so that every wavefront gets
    // a similar mix of long and short runs
    for (uint32_t k0 = it.seg_begin + wave; k0 < seg_end; k0 += kDirectThreads)
      walk_batch<8, false, true>(sc.segs, k0, seg_end, adj, Marks<uint8_t>{mtab[wave], mflag[wave]}, a.long_len,
                    DirectTallyBF<kDirectKeys>{cnt, cnt + kDirectKeys + tid}, kDirectWaves);
    __syncthreads();
    if (it.flags & kItemMultiPart) {
      // write the part's counters for the whole key window (zeros included)
      global_t<uint32_t>* __restrict__ dst = as_global(sc.acc) + static_cast<size_t>(it.acc_slot) * sc.acc_width;
      for (uint32_t key = it.key_lo + tid; key < static_cast<uint32_t>(it.key_hi); key += kDirectThreads) {
        dst[key] = cnt[key];
        cnt[key] = 0;
      }
    } else {
      // Sums of squares (see SqSums): every wedge of a single-part item lies
      // in its window, so thread 0 takes the item's wedges off once; the
      // wedges of pairs handed to the dense path are added back.  A key's
      // p + n is at most the item's runs (< 2^16), so p^2 + n^2 <= (p + n)^2
      // and 2 p n are exact in 32 bits: one 16-bit dot product of the
      // counter word with itself, and one with its halves swapped.
      // With at most 8,192 runs, (p + n)^2 <= 2^26 and a thread's at most 32
      // keys of the item sum below 2^31: the dot products then accumulate
      // in 32 bits (sq32, pn32) and reach the 64-bit sums once per item.
      if (tid == 0) sq2 -= static_cast<int64_t>(it.work);
      const bool hub = (it.flags & kItemHubPairs) != 0;
      const bool acc32 = it.seg_count <= 8192u;
      const uint32_t lo = static_cast<uint32_t>(it.key_lo) & ~3u;
      const uint32_t hi = static_cast<uint32_t>(it.key_hi);
      const uint32_t hub_hi = hub ? static_cast<uint32_t>(sc.T) : 0u;  // keys below: dense-path pairs
      uint32_t sq32 = 0, pn32 = 0;
      for (uint32_t key = lo + 4 * tid; key < hi; key += 4 * kDirectThreads) {
        const uint4 c4 = *reinterpret_cast<uint4*>(&cnt[key]);
        if ((c4.x | c4.y | c4.z | c4.w) == 0) continue;
        *reinterpret_cast<uint4*>(&cnt[key]) = make_uint4(0, 0, 0, 0);
        const uint32_t cv[4] = {c4.x, c4.y, c4.z, c4.w};
        if (key < hub_hi) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t p = cv[j] & 0xffffu, n = cv[j] >> 16;
            if (key + j < hub_hi) {
              if (cv[j]) {
                hub_partial(sc, it.owner, key + j, p, n);
                sq2 += p + n;
              }
            } else {
              sq2 += static_cast<int64_t>(__umul24(p, p)) + static_cast<int64_t>(__umul24(n, n));
              pnx += __umul24(p, n);
            }
          }
        } else if (acc32) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const u16x2 h = __builtin_bit_cast(u16x2, cv[j]);
            const u16x2 r = __builtin_bit_cast(u16x2, __builtin_amdgcn_alignbit(cv[j], cv[j], 16));
            sq32 = __builtin_amdgcn_udot2(h, h, sq32, false);
            pn32 = __builtin_amdgcn_udot2(h, r, pn32, false);
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const u16x2 h = __builtin_bit_cast(u16x2, cv[j]);
            const u16x2 r = __builtin_bit_cast(u16x2, __builtin_amdgcn_alignbit(cv[j], cv[j], 16));
            sq2 += __builtin_amdgcn_udot2(h, h, 0u, false);
            pnx += __builtin_amdgcn_udot2(h, r, 0u, false) >> 1;
          }
        }
      }
      sq2 += sq32;
      pnx += pn32 >> 1;  // a sum of 2 p n terms: even
    }
    __syncthreads();
  }
  if (graph != kNoGraph) flush_block(graph);
}

// ---------------------------------------------------------------------------
// Reverse items: one wavefront per item, a private LDS direct array over the
// reverse window [0, R) (R <= kMaxReverseL).  Counters are 8-bit
// (symmetric | asymmetric << 8) in 16-bit halves, two keys per 32-bit word:
// an item (or part) has at most kReverseCountMaxSegs segments, so no byte
// exceeds 127.  Items are dealt to wavefronts in a fixed stride; the next
// item's first segments and the descriptor of the one after are loaded while
// the current item is walked.  The sweep reads the whole window with 16-byte
// LDS loads.
typedef int v4i __attribute__((ext_vector_type(4)));
// sweep products an accumulator may hold before its diagonal is moved out:
// 2000 * 64 * 127^2 < 2^31
constexpr int32_t kAccItersMax = 2000 - 2 * kMaxReverseL / (4 * kWave);
constexpr int kReverseThreads = 1024;
constexpr int kReverseWaves = kReverseThreads / kWave;
constexpr int kReverseWords = kMaxReverseL / 2;

__global__ __launch_bounds__(kReverseThreads) void k_reverse(SmallArgs a) {
  // counters, each wavefront's array aligned to its size; one dummy word per lane
  __shared__ __attribute__((aligned(kReverseWords * 4))) uint32_t cnt[kReverseWaves][kReverseWords];
  __shared__ uint32_t dummies[kReverseWaves][kWave];
  __shared__ __attribute__((aligned(16))) uint32_t mtab[kReverseWaves][kGather];
  __shared__ uint8_t mflag[kReverseWaves][kGather];
  // wave index, known to the compiler as wavefront-uniform
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int lane = lane_id();
  uint32_t* C = cnt[wave];
  // the tally's AND-OR addresses need each array aligned to its size
  if (lane == 0 && (lds_addr(C) & (kReverseWords * 4 - 1)) != 0) atomicOr(a.err, kErrLdsLayout);
  for (int i = lane; i < kReverseWords; i += kWave) C[i] = 0;
  for (int i = lane; i < static_cast<int>(kGather); i += kWave) mflag[wave][i] = 0;
  wave_sync_lds();
  SqTotals tot;
  // matrix-core accumulators of the sweeps (see below) and the number of
  // products they hold; the diagonal of a 16 x 16 result is held by lanes
  // 20 g + q (g, q < 4) in register q
  v4i acc_sq = {0, 0, 0, 0}, acc_pn = {0, 0, 0, 0};
  int32_t acc_iters = 0;
  auto flush_acc = [&]() {
    const int q = (lane & 15) - 4 * (lane >> 4);
    int32_t dsq = 0, dpn = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      dsq = q == r ? acc_sq[r] : dsq;
      dpn = q == r ? acc_pn[r] : dpn;
    }
    tot.sq += static_cast<uint32_t>(dsq);
    tot.pn2 += static_cast<uint32_t>(dpn);
    acc_sq = v4i{0, 0, 0, 0};
    acc_pn = v4i{0, 0, 0, 0};
    acc_iters = 0;
  };
  const int32_t n = a.n_items;
  const int32_t stride = static_cast<int32_t>(gridDim.x) * kReverseWaves;
  int32_t i = static_cast<int32_t>(blockIdx.x) * kReverseWaves + wave;
  Item cur{}, nxt{};
  SegReg cfirst{0, 0, 0};
  if (i < n) {
    cur = load_const(a.items, i);
    cfirst = first_batch(cur, load_const(a.sides, 2 * cur.graph + cur.side).segs);
  }
  if (i + stride < n) nxt = load_const(a.items, i + stride);
  uint32_t graph = kNoGraph;
  for (; i < n; i += stride) {
    const Item it = cur;
    const SegReg first = cfirst;
    const int32_t j = i + stride, j2 = j + stride;
    if (it.graph != graph) {
      if (graph != kNoGraph) {
        flush_acc();
        tot.flush(a.res + static_cast<size_t>(graph) * kResStride);
      }
      tot = SqTotals{};
      graph = it.graph;
    }
    SegReg nfirst{0, 0, 0};
    if (j < n) nfirst = first_batch(nxt, load_const(a.sides, 2 * nxt.graph + nxt.side).segs);
    Item nxt2{};
    if (j2 < n) nxt2 = load_const(a.items, j2);
    const DevSideConst sc = load_const(a.sides, 2 * it.graph + it.side);
    walk_item<8, false, true>(it, first, sc.segs, sc.other_adj, Marks<uint8_t>{mtab[wave], mflag[wave]}, a.long_len,
                 PairTallyBF<kReverseWords>{lds_addr(C), lds_addr(&dummies[wave][lane])});
    wave_sync_lds();
    const int32_t w_hi = (it.key_hi + 1) >> 1;  // counter words of the item's keys
    if (it.flags & kItemMultiPart) {
      global_t<uint32_t>* __restrict__ dst = as_global(sc.acc) + static_cast<size_t>(it.acc_slot) * sc.acc_width;
      for (int32_t wd = lane; wd < w_hi; wd += kWave) {
        const uint32_t c2 = C[wd];
        C[wd] = 0;
        dst[2 * wd] = (c2 & 0xffu) | (((c2 >> 8) & 0xffu) << 16);
        if (2 * wd + 1 < it.key_hi) dst[2 * wd + 1] = ((c2 >> 16) & 0xffu) | ((c2 >> 24) << 16);
      }
    } else {
      // The item's sums over its keys, Σ p^2 + n^2 and 2 Σ p n, as traces of
      // signed 8-bit matrix products (p, n <= kReverseCountMaxSegs < 128):
      // 16 bytes per lane form a 16 x 64 operand A, and with the same
      // register as the other operand the product is A A^T, whose diagonal
      // holds each row's sum of squares; with the bytes of every 16-bit half
      // swapped (p <-> n) it holds 2 Σ p n.  The loop is uniform (the matrix
      // core needs every lane); words past the item's keys are zero.  Every
      // key of the item lies in the window, so its swept wedges are the
      // item's wedges (added once, by lane 0).
      const int32_t n_it = (w_hi + 4 * kWave - 1) / (4 * kWave);
      for (int32_t k = 0; k < n_it; ++k) {
        const int32_t wd = k * 4 * kWave + 4 * lane;
        const v4i c = *reinterpret_cast<const v4i*>(&C[wd]);
        *reinterpret_cast<uint4*>(&C[wd]) = make_uint4(0, 0, 0, 0);
        v4i cs;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          cs[q] = static_cast<int>(__builtin_amdgcn_perm(static_cast<uint32_t>(c[q]), static_cast<uint32_t>(c[q]),
                                                         0x02030001u));
        acc_sq = __builtin_amdgcn_mfma_i32_16x16x64_i8(c, c, acc_sq, 0, 0, 0);
        acc_pn = __builtin_amdgcn_mfma_i32_16x16x64_i8(c, cs, acc_pn, 0, 0, 0);
      }
      acc_iters += n_it;
      if (lane == 0) tot.w += it.work;
      // every product adds at most 64 * 127^2 to an entry: move the
      // diagonals out before an int32 entry could overflow
      if (acc_iters > kAccItersMax) flush_acc();
    }
    wave_sync_lds();
    cur = nxt;
    cfirst = nfirst;
    nxt = nxt2;
  }
  if (graph != kNoGraph) flush_acc();
  __shared__ WaveSums wsum[kReverseWaves];
  flush_block_end(tot, graph, wsum, kReverseWaves, a.res);
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

// Insertion of a group's wedges into its hash table, with no divergent
// branch: every lane issues every probe's compare-and-swap, a lane with
// nothing (left) to insert aims it at its own sink word, and the probe loop
// ends when the wavefront has no pending lane (a ballot).  One
// compare-and-swap per probe claims an empty slot or finds the key; after
// the loop each lane adds its count to the slot found (or to its sink).
// Probes step by an odd stride from a second multiplicative hash of the key
// (double hashing): without linear probing's clusters the wavefront's
// longest probe chain, which every lane waits for, is shorter.
struct SmallInsert {
  uint32_t* K;
  uint32_t* V;
  uint32_t* sink;  // this lane's sink word
  uint32_t kb, hshift, mask;
  unsigned long long* err;
  __device__ __forceinline__ void add(uint32_t e, uint32_t tag, bool valid) const {
    const uint32_t key = ((tag >> 1) << kb) | (e >> 1);
    const uint32_t inc = wedge_inc(e, tag);
    uint32_t h = (key * 0x9E3779B1u) >> hshift;
    const uint32_t step = ((key * 0x85EBCA6Bu) >> hshift) | 1u;  // odd: size probes visit every slot
    bool pend = valid;
    uint32_t at = 0;  // the slot found
    for (uint32_t probe = 0;; ++probe) {
      const uint32_t c = atomicCAS(pend ? &K[h] : sink, kEmpty, key);
      const bool hit = pend && (c == kEmpty || c == key);
      at = hit ? h : at;
      pend = pend && !hit;
      if (__ballot(pend) == 0) break;
      if (probe == mask) {  // full table: cannot happen at load <= 1/2
        if (lane_id() == 0) atomicOr(err, kErrHashFull);
        break;
      }
      h = (h + step) & mask;
    }
    atomicAdd(valid && !pend ? &V[at] : sink, inc);
  }
};

__global__ __launch_bounds__(kSmallThreads) void k_small(SmallArgs a) {
  __shared__ __attribute__((aligned(16))) uint32_t keys[kSmallWaves][kSmallSlots];
  __shared__ __attribute__((aligned(16))) uint32_t vals[kSmallWaves][kSmallSlots];
  // staging marks: bases, and 16-bit tags (item index in the group << 1 | g,
  // with the presence bit; a group holds at most kSmallMaxItems items)
  __shared__ __attribute__((aligned(16))) uint32_t mbase[kSmallWaves][kGather];
  __shared__ uint16_t mtag[kSmallWaves][kGather];
  __shared__ uint32_t sinks[kSmallWaves][kWave];
  static_assert(2 * kSmallMaxItems + 1 < (1u << 15), "group tags fit 15 bits");
  // wave index, known to the compiler as wavefront-uniform
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int lane = lane_id();
  uint32_t* K = keys[wave];
  uint32_t* Vv = vals[wave];
  for (int i = lane; i < kSmallSlots; i += kWave) {
    K[i] = kEmpty;
    Vv[i] = 0;
  }
  for (int i = lane; i < static_cast<int>(kGather); i += kWave) mtag[wave][i] = 0;
  wave_sync_lds();
  SqTotals tot;
  const int32_t stride = static_cast<int32_t>(gridDim.x) * kSmallWaves;
  int32_t i = static_cast<int32_t>(blockIdx.x) * kSmallWaves + wave;
  Item nxt{};
  SegReg nfirst{0, 0, 0};
  if (i < a.n_items) {
    nxt = load_const(a.items, i);
    nfirst = first_batch<true>(nxt, load_const(a.sides, 2 * nxt.graph + nxt.side).small_segs);
  }
  uint32_t graph = kNoGraph;
  for (; i < a.n_items; i += stride) {
    const Item it = nxt;
    const SegReg first = nfirst;
    const int32_t j = i + stride;
    if (j < a.n_items) nxt = load_const(a.items, j);
    if (it.graph != graph) {
      if (graph != kNoGraph) tot.flush(a.res + static_cast<size_t>(graph) * kResStride);
      tot = SqTotals{};
      graph = it.graph;
    }
    const DevSideConst sc = load_const(a.sides, 2 * it.graph + it.side);
    const uint32_t kb = static_cast<uint32_t>(sc.key_bits);
    // table size: a power of two >= 2 * work, at least 64; the home slot is
    // the top log2(size) bits of the key times 2^32 / golden ratio
    // (multiplicative hashing: one multiply)
    const uint32_t w2 = 2 * it.work;
    const uint32_t size = w2 <= 64 ? 64u : 1u << (32 - __builtin_clz(w2 - 1));
    const uint32_t mask = size - 1;
    const uint32_t hshift = 32u - static_cast<uint32_t>(__builtin_ctz(size));
    walk_item<4, true>(it, first, sc.small_segs, sc.other_adj, Marks<uint16_t>{mbase[wave], mtag[wave]}, a.long_len,
                       SmallInsert{K, Vv, &sinks[wave][lane], kb, hshift, mask, a.err});
    if (j < a.n_items) nfirst = first_batch<true>(nxt, load_const(a.sides, 2 * nxt.graph + nxt.side).small_segs);
    wave_sync_lds();
    // p, n <= kSmallGroupWork per key and sum p + n <= kSmallGroupWork
    // per group, so the group's sums of squares stay below 2^19.  16-byte
    // LDS accesses, 4 slots per lane; an empty slot's count is 0, which adds
    // nothing to the sums.
    SqSums ss;
    if (!(it.flags & kItemHubPairs)) {
      // the keys are only reset; a slot's p^2 + n^2 and 2 p n are 16-bit dot
      // products of its count word with itself and with its halves swapped,
      // and the sum of p + n over the group is its work
      uint32_t sq32 = 0, pn32 = 0;
      for (uint32_t h = 4 * lane; h < size; h += 4 * kWave) {
        const uint4 c4 = *reinterpret_cast<const uint4*>(&Vv[h]);
        *reinterpret_cast<uint4*>(&K[h]) = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
        *reinterpret_cast<uint4*>(&Vv[h]) = make_uint4(0, 0, 0, 0);
        const uint32_t cv[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const u16x2 hh = __builtin_bit_cast(u16x2, cv[q4]);
          const u16x2 rr = __builtin_bit_cast(u16x2, __builtin_amdgcn_alignbit(cv[q4], cv[q4], 16));
          sq32 = __builtin_amdgcn_udot2(hh, hh, sq32, false);
          pn32 = __builtin_amdgcn_udot2(hh, rr, pn32, false);
        }
      }
      tot.sq += sq32;
      tot.pn2 += pn32;
      if (lane == 0) tot.w += it.work;
    } else {
      // a hub pivot's item (alone in its group): keys below T are hub pairs
      const uint32_t kmask = (1u << kb) - 1u;
      for (uint32_t h = 4 * lane; h < size; h += 4 * kWave) {
        const uint4 k4 = *reinterpret_cast<const uint4*>(&K[h]);
        const uint4 c4 = *reinterpret_cast<const uint4*>(&Vv[h]);
        *reinterpret_cast<uint4*>(&K[h]) = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
        *reinterpret_cast<uint4*>(&Vv[h]) = make_uint4(0, 0, 0, 0);
        const uint32_t kk[4] = {k4.x, k4.y, k4.z, k4.w}, cc[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const uint32_t key = kk[q4], p = cc[q4] & 0xffffu, q = cc[q4] >> 16;
          if (key != kEmpty && static_cast<int32_t>(key & kmask) < sc.T)
            hub_partial(sc, it.owner, key & kmask, p, q);
          else
            ss.add(p, q);
        }
      }
    }
    tot.add(ss);
    wave_sync_lds();
  }
  __shared__ WaveSums wsum[kSmallWaves];
  flush_block_end(tot, graph, wsum, kSmallWaves, a.res);
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
  __shared__ __attribute__((aligned(16))) uint32_t mtab[kHashWaves][kGather];
  __shared__ uint8_t mflag[kHashWaves][kGather];
  __shared__ int32_t item_sh;
  __shared__ uint32_t work_sh;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  for (int i = tid; i < kHashSlots; i += kHashThreads) {
    keys[i] = kEmpty;
    vals[i] = 0;
  }
  for (int i = tid; i < kHashWaves * static_cast<int>(kGather); i += kHashThreads) (&mflag[0][0])[i] = 0;
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
    const Item it = load_const(a.items, i);
    if (it.graph != graph) {
      if (graph != kNoGraph) flush_sums(sums, a.res + static_cast<size_t>(graph) * kResStride);
      sums = Sums{};
      graph = it.graph;
    }
    const DevSideConst sc = load_const(a.sides, 2 * it.graph + it.side);
    const uint32_t seg_end = it.seg_begin + it.seg_count;
    uint32_t w = 0;
    for (uint32_t k = it.seg_begin + tid; k < seg_end; k += kHashThreads) w += as_global(&sc.segs[k].len_g)[0] >> 1;
    atomicAdd(&work_sh, w);
    __syncthreads();
    const uint32_t work = work_sh;
    // about kHashSlots / 4 distinct keys per pass at most on average; the
    // table in use is a power of two >= twice a pass's wedges (at least 512
    // slots), so a small item's sweep reads only that much
    const uint32_t passes = (work + kHashSlots / 4 - 1) / (kHashSlots / 4);
    const uint32_t per_pass = (work + passes - 1) / (passes > 0 ? passes : 1);
    uint32_t size = 512;
    while (size < 2 * per_pass && size < static_cast<uint32_t>(kHashSlots)) size <<= 1;
    const uint32_t mask = size - 1;
    for (uint32_t pass = 0; pass < passes; ++pass) {
      for (uint32_t k0 = it.seg_begin + wave * kWave; k0 < seg_end; k0 += kHashThreads) {
        const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
        walk_batch<4>(sc.segs, k0, k1, sc.other_adj, Marks<uint8_t>{mtab[wave], mflag[wave]}, a.long_len, hash_tally([&](uint32_t e, uint32_t g) {
          const uint32_t key = e >> 1;
          const uint32_t hk = mix32(key);
          if (passes > 1 && (hk >> 16) % passes != pass) return;
          const unsigned long long inc = ((e ^ g) & 1u) ? (1ull << 32) : 1ull;
          uint32_t h = hk & mask;
          const uint32_t st = probe_step(key, mask);
          for (uint32_t probe = 0;; ++probe) {
            if (probe > mask) {  // full table
              atomicOr(a.err, kErrHashFull);
              break;
            }
            // one compare-and-swap per probe (claims an empty slot)
            const uint32_t cur = atomicCAS(&keys[h], kEmpty, key);
            if (cur == kEmpty || cur == key) {
              atomicAdd(&vals[h], inc);
              break;
            }
            h = (h + st) & mask;
          }
        }));
      }
      __syncthreads();
      for (int h = tid; h < static_cast<int>(size); h += kHashThreads) {
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
  __shared__ WaveSums wsum[kHashWaves];
  flush_block_end(sums, graph, wsum, kHashWaves, a.res);
}

// ---------------------------------------------------------------------------
// Multi-part pivots: add the parts' packed counters key by key, then take
// C(., 2) of the combined counts.
constexpr int kReduceThreads = 256;
constexpr int kReduceSlices = 8;  // workgroups per reduce (a few dozen reduces fill no GPU)

__global__ __launch_bounds__(kReduceThreads) void k_reduce(ReduceArgs a) {
  Sums sums;
  uint32_t graph = kNoGraph;
  // work units: kReduceSlices interleaved key slices of every reduce
  const int64_t units = static_cast<int64_t>(a.n_reduces) * kReduceSlices;
  for (int64_t unit = blockIdx.x; unit < units; unit += gridDim.x) {
    const int32_t r = static_cast<int32_t>(unit / kReduceSlices), slice = static_cast<int32_t>(unit % kReduceSlices);
    const Reduce rd = load_const(a.reduces, r);
    if (rd.graph != graph) {
      if (graph != kNoGraph) flush_sums(sums, a.res + static_cast<size_t>(graph) * kResStride);
      sums = Sums{};
      graph = rd.graph;
    }
    const DevSideConst sc = load_const(a.sides, 2 * rd.graph + rd.side);
    Item it{};
    it.owner = rd.owner;
    it.flags = rd.flags;
    const global_t<uint32_t>* acc = as_global(sc.acc) + static_cast<size_t>(rd.acc_slot) * sc.acc_width;
    for (int32_t key = rd.key_lo + slice * kReduceThreads + static_cast<int32_t>(threadIdx.x); key < rd.key_hi;
         key += kReduceSlices * kReduceThreads) {
      uint32_t p = 0, n = 0;
      // eight independent part loads per step
      int32_t j = 0;
      for (; j + 8 <= rd.n_parts; j += 8) {
        uint32_t c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) c[q] = acc[static_cast<size_t>(j + q) * sc.acc_width + key];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          p += c[q] & 0xffffu;
          n += c[q] >> 16;
        }
      }
      for (; j < rd.n_parts; ++j) {
        const uint32_t c = acc[static_cast<size_t>(j) * sc.acc_width + key];
        p += c & 0xffffu;
        n += c >> 16;
      }
      if (p | n) emit(it, static_cast<uint32_t>(key), p, n, sc, sums);
    }
  }
  __shared__ WaveSums wsum[kReduceThreads / kWave];
  flush_block_end(sums, graph, wsum, kReduceThreads / kWave, a.res);
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

// Store a graph's two side-table entries (passed by value) at dst.
struct SidePair {
  DevSideConst s[2];
};
__global__ void k_store_sides(SidePair t, DevSideConst* dst) {
  if (threadIdx.x < 2) dst[threadIdx.x] = t.s[threadIdx.x];
}

}  // namespace dev

// ---- launchers ------------------------------------------------------------------

hipError_t launch_store_sides(const DevSideConst* src2, DevSideConst* dst, hipStream_t st) {
  dev::SidePair t;
  t.s[0] = src2[0];
  t.s[1] = src2[1];
  hipLaunchKernelGGL(dev::k_store_sides, dim3(1), dim3(64), 0, st, t, dst);
  return hipGetLastError();
}

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

hipError_t launch_reduce(const ReduceArgs& a, int max_grid, hipStream_t st) {
  if (a.n_reduces == 0) return hipSuccess;
  const int64_t units = static_cast<int64_t>(a.n_reduces) * dev::kReduceSlices;
  const int grid = static_cast<int>(units < max_grid ? units : max_grid);
  hipLaunchKernelGGL(dev::k_reduce, dim3(grid), dim3(dev::kReduceThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace dbbc
