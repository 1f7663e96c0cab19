// HIP kernels (gfx950) of the per-vertex pass: for every vertex, the number
// of balanced and unbalanced butterflies that contain it (the vertex measure
// of Section I's applications).
//
// Each butterfly is counted once, at the pair (x, w) that owns it under the
// vertex priority (Algorithm 1, Phase 5): x and w are its two same-side
// vertices and its two mids are wedge mids of the pair.  With the pair's
// symmetric and asymmetric wedge counts p and n (Lemma 1):
//   - x and w each lie in C(p,2) + C(n,2) balanced and p n unbalanced
//     butterflies of the pair;
//   - the mid of a symmetric wedge lies in p - 1 balanced ones (paired with
//     each other symmetric mid) and n unbalanced ones, the mid of an
//     asymmetric wedge in n - 1 balanced and p unbalanced ones.
// So every item is walked twice: a tally of p and n per key as in the count
// pass, then a credit walk that reads each wedge's final p and n and adds
// the mid's share; the sweep credits the key vertices and, summed, the
// item's owner.  The plan of this pass has no multi-part items, so every
// pair's counts are complete inside one item -- except the hub pairs of a
// dense block, whose completed counts the block's products leave in hub_xy
// (hubpv.hip) before these kernels run.
//
// Mid credits are summed per run (a run has one mid) in registers, then per
// batch in a per-wavefront LDS slot of the run's lane, and reach HBM as one
// 64-bit atomic per run; key and owner credits are one atomic per nonzero
// pair and per item.  Walk tags here are (item index in group << 7) |
// (run lane << 1) | g.
//
// Per-edge counts (the edge measure of the same section, kEdge): a wedge's
// share (p - 1 and n, or n - 1 and p) is also the number of butterflies of
// the pair that contain each of its two edges, since such a butterfly is the
// union of this wedge and one other wedge of the pair.  The run's first edge
// takes the run's summed share with the mid; the walked entry's edge takes
// its wedge's share at its position in the other side's CSR, one 64-bit
// atomic per wedge with both values packed (two for runs flagged kMidWide).
// The credit walk then reads long runs lane-major, so that the atomics of a
// wavefront hit consecutive positions.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"
#include "walk.h"

namespace dbbc {
namespace dev {

// The runs k0 + stride * lane (< k1) of a batch with per-vertex tags, and
// each lane's mid (and, with kEdge, the position of its first edge).
struct RunEnds {
  uint32_t mid = 0, edge = 0, wide = 0;
};

template <bool kTagged, bool kEdge>
__device__ __forceinline__ SegReg load_seg_pv(const Segment* __restrict__ segs,
                                              const uint32_t* __restrict__ mids,
                                              const uint32_t* __restrict__ edges, uint32_t k0, uint32_t k1,
                                              RunEnds& re, uint32_t stride = 1) {
  SegReg r = load_seg<kTagged>(segs, k0, k1, stride);
  const uint32_t lane = static_cast<uint32_t>(lane_id());
  const uint32_t g = r.tag & 1u;
  r.tag = kTagged ? (((r.tag >> 1) << 7) | (lane << 1) | g) : ((lane << 1) | g);
  const uint32_t k = k0 + stride * lane;
  const bool in = k < k1;
  const uint32_t m = in ? as_global(mids)[k] : 0u;
  re.mid = m & ~kMidWide;
  if (kEdge) {
    re.edge = in ? as_global(edges)[k] : 0u;
    re.wide = m & kMidWide;
  }
  return r;
}

// Credit walk: Look(e, tag, p, n) gives the pair counts of a wedge's key
// (false: the key is not counted by this item or pass).  Credits of the
// lane's current run are kept in registers and added to the run's LDS slot
// when the lane moves to another run; with kEdge every wedge's share is
// also added to the walked entry's edge (by entry position: packed in ep,
// or in wb and wu for a wide run: bit j of `wide` for the run of lane j).
// Non-returning 64-bit add to global memory (device scope).
__device__ __forceinline__ void add_global(global_t<unsigned long long>* p, unsigned long long v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class Look, bool kEdge, class Acc, bool kHoist = false, bool kPack = false>
struct Credit {
  // kHoist: a staging round's four slots read their counters before any is
  // used (add_staged); Look must then be branch-free and safe for any entry
  static constexpr bool kStaged = kHoist;
  Look look;
  Acc* cb;  // per-wavefront LDS: balanced credit per run lane (kPack: both,
            // balanced in the low and unbalanced in the high 32 bits)
  Acc* cu;  // unbalanced (unused with kPack)
  global_t<unsigned long long>* ep;
  global_t<unsigned long long>* wb;
  global_t<unsigned long long>* wu;
  uint64_t wide = 0;  // runs (by lane) whose credits take two words
  uint32_t cur = 0xffffffffu;  // the run of the chunk slots summed in sb, su (wave-uniform)
  Acc sb = 0, su = 0;
  // the wedge's shares: balanced b and unbalanced u (false: not a wedge of
  // this item or pass)
  __device__ __forceinline__ bool share(uint32_t e, uint32_t tag, bool valid, uint32_t& b, uint32_t& u) {
    uint32_t p, n;
    if (!valid || !look(e, tag, p, n)) return false;
    const bool sym = ((e ^ tag) & 1u) == 0;
    b = sym ? p - 1u : n - 1u;
    u = sym ? n : p;
    return true;
  }
  __device__ __forceinline__ void edge(uint32_t j, uint32_t pos, uint32_t b, uint32_t u) {
    if (kEdge) {
      if ((wide >> j) & 1u) {
        if (b) add_global(wb + pos, b);
        if (u) add_global(wu + pos, u);
      } else if (b | u) {
        add_global(ep + pos, (static_cast<unsigned long long>(u) << 32) | b);
      }
    }
  }
  // a run's LDS slot takes b and u: one 64-bit add with kPack (each half
  // stays below 2^32: the caller's runs bound their credits)
  __device__ __forceinline__ void slot_add(uint32_t j, Acc b, Acc u) {
    if constexpr (kPack) {
      if (b | u) atomicAdd(&cb[j], (u << 32) | b);
    } else {
      if (b) atomicAdd(&cb[j], b);
      if (u) atomicAdd(&cu[j], u);
    }
  }
  __device__ __forceinline__ void put() {
    if (cur != 0xffffffffu) slot_add(cur, sb, su);
    sb = su = 0;
  }
  // a staged position (lanes in different runs): its shares straight to its
  // run's LDS slot
  __device__ __forceinline__ void add(uint32_t e, uint32_t tag, bool valid, uint32_t pos) {
    uint32_t b, u;
    if (!share(e, tag, valid, b, u)) return;
    const uint32_t j = (tag >> 1) & 63u;
    slot_add(j, b, u);
    edge(j, pos, b, u);
  }
  // a staging round's slots (their runs' LDS slots take the shares)
  __device__ __forceinline__ void add_staged(const Staged& s) {
    uint32_t p[kStageU], n[kStageU];
    bool ok[kStageU];
#pragma unroll
    for (int q = 0; q < kStageU; ++q) ok[q] = look(s.valid[q] ? s.e[q] : 0u, s.tag[q], p[q], n[q]) && s.valid[q];
#pragma unroll
    for (int q = 0; q < kStageU; ++q) {
      if (!ok[q]) continue;
      const bool sym = ((s.e[q] ^ s.tag[q]) & 1u) == 0;
      const uint32_t b = sym ? p[q] - 1u : n[q] - 1u;
      const uint32_t u = sym ? n[q] : p[q];
      const uint32_t j = (s.tag[q] >> 1) & 63u;
      slot_add(j, b, u);
      edge(j, s.pos[q], b, u);
    }
  }
  // a chunk slot (every lane in the chunk's run): summed in registers until
  // the run changes (a wave-uniform test)
  __device__ __forceinline__ void add_chunk(uint32_t e, uint32_t tag, bool valid, uint32_t pos) {
    const uint32_t j = (tag >> 1) & 63u;
    if (j != cur) {
      put();
      cur = j;
    }
    uint32_t b, u;
    if (!share(e, tag, valid, b, u)) return;
    sb += b;
    su += u;
    edge(j, pos, b, u);
  }
  __device__ __forceinline__ void flush() {
    put();
    cur = 0xffffffffu;
  }
};

template <bool kEdge, bool kHoist = false, bool kPack = false, class Look, class Acc>
__device__ __forceinline__ Credit<Look, kEdge, Acc, kHoist, kPack> credit(Look l, Acc* cb, Acc* cu,
                                                                          const DevSideConst& sc, const RunEnds& re) {
  static_assert(!kPack || sizeof(Acc) == 8, "packed slots are 64-bit");
  Credit<Look, kEdge, Acc, kHoist, kPack> c{l, cb, cu, as_global(sc.epack_o), as_global(sc.ewb_o),
                                            as_global(sc.ewu_o)};
  if (kEdge) c.wide = __ballot(re.wide != 0);
  return c;
}

// A run's credits b and u to its mid (and, with kEdge, to its first edge).
template <bool kEdge>
__device__ __forceinline__ void mid_credits_out(unsigned long long b, unsigned long long u, RunEnds re,
                                                const DevSideConst& sc) {
  const int32_t id = sc.orig_mid[re.mid];
  if (b) atomicAdd(&sc.bal_mid[id], b);
  if (u) atomicAdd(&sc.unb_mid[id], u);
  if (kEdge) {
    if (re.wide) {
      if (b) add_global(as_global(sc.ewb) + re.edge, b);
      if (u) add_global(as_global(sc.ewu) + re.edge, u);
    } else {  // the run's credits are below 2^32 (no wide flag)
      add_global(as_global(sc.epack) + re.edge, (u << 32) | b);
    }
  }
}

// After a batch's credit walk: each lane adds its run's credits to the mid
// (and, with kEdge, to the run's first edge).
template <bool kEdge, class Acc>
__device__ __forceinline__ void flush_mid_credits(Acc* cb, Acc* cu, RunEnds re, const DevSideConst& sc) {
  wave_sync_lds();
  const int lane = lane_id();
  const unsigned long long b = cb[lane], u = cu[lane];
  if (b | u) {
    cb[lane] = 0;
    cu[lane] = 0;
    mid_credits_out<kEdge>(b, u, re, sc);
  }
  wave_sync_lds();
}

// The same for packed slots (balanced | unbalanced << 32).
template <bool kEdge>
__device__ __forceinline__ void flush_mid_credits_packed(unsigned long long* cbu, RunEnds re,
                                                         const DevSideConst& sc) {
  wave_sync_lds();
  const int lane = lane_id();
  const unsigned long long v = cbu[lane];
  if (v) {
    cbu[lane] = 0;
    mid_credits_out<kEdge>(v & 0xffffffffull, v >> 32, re, sc);
  }
  wave_sync_lds();
}

// Completed counts of the hub pair (x, key) (dense block of the pass): the
// block's products store X = p + n and Y = p - n in hub_xy.
__device__ __forceinline__ void hub_counts(const DevSideConst& sc, uint32_t x, uint32_t key, uint32_t& p,
                                           uint32_t& n) {
  const size_t T = static_cast<size_t>(sc.T);
  const global_t<int32_t>* h = as_global(sc.hub_xy) + x * T + key;
  const int32_t X = h[0], Y = h[T * T];
  p = static_cast<uint32_t>((X + Y) / 2);
  n = static_cast<uint32_t>((X - Y) / 2);
}

// Key credits of one pair (p, n) at key vertex `key` of side s.
struct PairCredit {
  int64_t c = 0, x = 0;  // owner sums
  __device__ __forceinline__ void add(const DevSideConst& sc, uint32_t key, uint32_t p, uint32_t n, Sums& s) {
    s.add(p, n);
    const int64_t P = p, N = n;
    const int64_t cb = P * (P - 1) / 2 + N * (N - 1) / 2, cx = P * N;
    if (cb) atomicAdd(&sc.bal[sc.orig[key]], static_cast<unsigned long long>(cb));
    if (cx) atomicAdd(&sc.unb[sc.orig[key]], static_cast<unsigned long long>(cx));
    c += cb;
    x += cx;
  }
  // The wavefront's owner sums to `owner` (one atomic per wavefront).
  __device__ __forceinline__ void to_owner(const DevSideConst& sc, int32_t owner) {
    const int64_t c2 = wave_sum64(c), x2 = wave_sum64(x);
    if (lane_id() == 0) {
      if (c2) atomicAdd(&sc.bal[sc.orig[owner]], static_cast<unsigned long long>(c2));
      if (x2) atomicAdd(&sc.unb[sc.orig[owner]], static_cast<unsigned long long>(x2));
    }
    c = x = 0;
  }
};

// ---------------------------------------------------------------------------
// Direct items: one workgroup per item, p and n counters over the item's
// key window, 32-bit each (at most kPVWindow keys) or, for items with fewer
// than 2^16 runs (kItemPacked), 16|16 bits in one word (at most
// kPVWindowPacked keys, the whole window of the count pass, so a pivot's
// runs are walked once per walk); windows of one pivot share their runs and
// skip the keys of the others.  The walks stage short runs in the run-table
// form (a 64-entry table per wavefront), which leaves the LDS to the
// counters.  Key credits are global atomics (the keys that many items
// share, a side's top vertices, are the dense block's when it is on).
constexpr int kPVDirectThreads = 1024;
constexpr int kPVDirectWaves = kPVDirectThreads / kWave;

template <bool kEdge>
__global__ __launch_bounds__(kPVDirectThreads) void k_pv_direct(DirectArgs a) {
  __shared__ uint32_t C[kPVWindowPacked];  // P | N, or packed words
  __shared__ __attribute__((aligned(16))) uint32_t mtab[kPVDirectWaves][2 * kWave];
  __shared__ uint8_t mflag[kPVDirectWaves][kGather];
  __shared__ unsigned long long cb[kPVDirectWaves][kWave], cu[kPVDirectWaves][kWave];
  __shared__ int32_t item_sh;
  static_assert(2 * kPVWindow == kPVWindowPacked, "P | N halves fill the packed window");
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = lane_id();
  for (int i = tid; i < kPVWindowPacked; i += kPVDirectThreads) C[i] = 0;
  uint32_t* const P = C;
  uint32_t* const N = C + kPVWindow;
  for (int i = tid; i < kPVDirectWaves * static_cast<int>(kGather); i += kPVDirectThreads) (&mflag[0][0])[i] = 0;
  cb[wave][lane] = 0;
  cu[wave][lane] = 0;
  const Marks<uint8_t> mk{mtab[wave], mflag[wave]};
  Sums sums;                              // unpacked items' pairs
  uint64_t sq64 = 0, pn64 = 0, w64 = 0;   // packed items' pairs: sums of p^2 + n^2, p n, p + n
  auto flush_all = [&](uint32_t g) {
    unsigned long long* res = a.res + static_cast<size_t>(g) * kResStride;
    flush_sums(sums, res);
    const int64_t q = wave_sum64(static_cast<int64_t>(sq64)), x = wave_sum64(static_cast<int64_t>(pn64));
    const int64_t ww = wave_sum64(static_cast<int64_t>(w64));
    if (lane == 0) {
      const int64_t bal = (q - ww) / 2;
      if (bal) atomicAdd(res + kResBalanced, static_cast<unsigned long long>(bal));
      if (x) atomicAdd(res + kResUnbalanced, static_cast<unsigned long long>(x));
      if (bal + x) atomicAdd(res + kResTotal, static_cast<unsigned long long>(bal + x));
    }
    sums = Sums{};
    sq64 = pn64 = w64 = 0;
  };
  uint32_t graph = kNoGraph;
  for (;;) {
    if (tid == 0) item_sh = static_cast<int32_t>(atomicAdd(a.queue, 1u));
    __syncthreads();
    const int32_t i = item_sh;
    if (i >= a.n_items) break;
    const Item it = load_const(a.items, i);
    if (it.graph != graph) {
      if (graph != kNoGraph) flush_all(graph);
      graph = it.graph;
    }
    const DevSideConst sc = load_const(a.sides, 2 * it.graph + it.side);
    const uint32_t lo = static_cast<uint32_t>(it.key_lo), hi = static_cast<uint32_t>(it.key_hi);
    const uint32_t seg_end = it.seg_begin + it.seg_count;
    const bool packed = (it.flags & kItemPacked) != 0;
    // a hub pivot's keys below T are hub pairs: their completed counts come
    // from the dense block and their key credits were given there
    const uint32_t hubT = (it.flags & kItemHubPairs) ? static_cast<uint32_t>(sc.T) : 0u;
    // tally (the wavefronts take the item's segments interleaved, so that
    // every wavefront gets a similar mix of long and short runs)
    for (uint32_t k0 = it.seg_begin + wave; k0 < seg_end; k0 += kPVDirectThreads) {
      RunEnds re;
      const SegReg sr = load_seg_pv<false, kEdge>(sc.segs, sc.seg_mid, sc.seg_edge, k0, seg_end, re, kPVDirectWaves);
      if (packed)
        walk_regs<4, false, true>(sr, sc.other_adj, mk, a.long_len, hash_tally([&](uint32_t e, uint32_t tag) {
                                    const uint32_t key = e >> 1;
                                    if (key >= lo && key < hi) atomicAdd(&C[key - lo], wedge_inc(e, tag));
                                  }));
      else
        walk_regs<4, false, true>(sr, sc.other_adj, mk, a.long_len, hash_tally([&](uint32_t e, uint32_t tag) {
                                    const uint32_t key = e >> 1;
                                    if (key >= lo && key < hi)
                                      atomicAdd(((e ^ tag) & 1u) ? &N[key - lo] : &P[key - lo], 1u);
                                  }));
    }
    __syncthreads();
    // credit the mids
    for (uint32_t k0 = it.seg_begin + wave; k0 < seg_end; k0 += kPVDirectThreads) {
      RunEnds re;
      const SegReg sr = load_seg_pv<false, kEdge>(sc.segs, sc.seg_mid, sc.seg_edge, k0, seg_end, re, kPVDirectWaves);
      if (packed && hubT == 0) {
        // p, n < 2^16 and at most kPVWindowPacked keys per window: a run's
        // credits per window stay below 2^31, so one packed LDS word per run
        auto c = credit<kEdge, false, true>(
            [&](uint32_t e, uint32_t, uint32_t& p, uint32_t& n) {
              const uint32_t key = e >> 1;
              if (key < lo || key >= hi) return false;
              const uint32_t v = C[key - lo];
              p = v & 0xffffu;
              n = v >> 16;
              return true;
            },
            cb[wave], static_cast<unsigned long long*>(nullptr), sc, re);
        walk_regs<4, kEdge, true>(sr, sc.other_adj, mk, a.long_len, c);
        c.flush();
        flush_mid_credits_packed<kEdge>(cb[wave], re, sc);
        continue;
      }
      auto c = credit<kEdge>(
          [&](uint32_t e, uint32_t, uint32_t& p, uint32_t& n) {
            const uint32_t key = e >> 1;
            if (key < lo || key >= hi) return false;
            if (key < hubT) {
              hub_counts(sc, static_cast<uint32_t>(it.owner), key, p, n);
              return true;
            }
            if (packed) {
              const uint32_t v = C[key - lo];
              p = v & 0xffffu;
              n = v >> 16;
            } else {
              p = P[key - lo];
              n = N[key - lo];
            }
            return true;
          },
          cb[wave], cu[wave], sc, re);
      walk_regs<4, kEdge, true>(sr, sc.other_adj, mk, a.long_len, c);
      c.flush();
      flush_mid_credits<kEdge>(cb[wave], cu[wave], re, sc);
    }
    __syncthreads();
    // credit the keys and the owner (packed counts: p + n < 2^16, so a
    // key's credits fit 32 bits).  Key credits go to the rank-indexed sums
    // (the threads' keys are consecutive: one instruction's atomics touch a
    // few cache lines, where input-id order would scatter them over 64).
    PairCredit pc;
    for (uint32_t k = tid; k < hi - lo; k += kPVDirectThreads) {
      const uint32_t v = C[k];
      const uint32_t p = packed ? v & 0xffffu : v, n = packed ? v >> 16 : N[k];
      if (p | n) {
        C[k] = 0;
        if (!packed) N[k] = 0;
        const uint32_t key = lo + k;
        if (key < hubT) continue;  // a hub pair: credited by the dense block
        if (packed) {
          const uint32_t cb2 = (__umul24(p, p - 1u) + __umul24(n, n - 1u)) >> 1, cx = __umul24(p, n);
          sq64 += static_cast<uint64_t>(__umul24(p, p)) + __umul24(n, n);
          pn64 += cx;
          w64 += p + n;
          if (cb2) atomicAdd(&sc.key_bal[key], static_cast<unsigned long long>(cb2));
          if (cx) atomicAdd(&sc.key_unb[key], static_cast<unsigned long long>(cx));
          pc.c += cb2;
          pc.x += cx;
        } else {
          sums.add(p, n);
          const int64_t P64 = p, N64 = n;
          const int64_t cb64 = P64 * (P64 - 1) / 2 + N64 * (N64 - 1) / 2, cx64 = P64 * N64;
          if (cb64) atomicAdd(&sc.key_bal[key], static_cast<unsigned long long>(cb64));
          if (cx64) atomicAdd(&sc.key_unb[key], static_cast<unsigned long long>(cx64));
          pc.c += cb64;
          pc.x += cx64;
        }
      }
    }
    pc.to_owner(sc, it.owner);
    __syncthreads();
  }
  {
    const int64_t q = wave_sum64(static_cast<int64_t>(sq64)), x = wave_sum64(static_cast<int64_t>(pn64));
    const int64_t ww = wave_sum64(static_cast<int64_t>(w64));
    __shared__ WaveSums wsum[kPVDirectWaves];
    flush_block_end(wave_sum64(sums.bal) + (q - ww) / 2, wave_sum64(sums.unb) + x, graph, wsum, kPVDirectWaves,
                    a.res);
  }
}

// The direct items' key credits of side s (by rank, ranks below n) into the
// per-vertex outputs (input-id order).
__global__ void k_pv_key_flush(const DevSideConst* sides, int32_t s, int32_t n) {
  const DevSideConst sc = load_const(sides, s);
  for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const unsigned long long b = sc.key_bal[k], u = sc.key_unb[k];
    if (b | u) {
      const int32_t id = sc.orig[k];
      if (b) atomicAdd(&sc.bal[id], b);
      if (u) atomicAdd(&sc.unb[id], u);
    }
  }
}

// ---------------------------------------------------------------------------
// Reverse items (at most kReverseMaxSegs runs): one wavefront per item, 8-bit
// p and n per key over the reverse window, two keys per 32-bit word.  The
// keys are the reverse window's vertices, shared by every item of a side, so
// their credits are summed per workgroup in LDS and reach HBM once per
// workgroup at the end (a launch holds the items of one side).  A pair's
// credit is below 2^15 (p + n <= 255), so the workgroup's 32-bit key sums
// hold up to 2^16 items (the launch sizes its grid for that).
constexpr int kPVReverseWaves = 12;
constexpr int kPVReverseThreads = kPVReverseWaves * kWave;
constexpr int kPVReverseWords = kMaxReverseL / 2;

template <bool kEdge>
__global__ __launch_bounds__(kPVReverseThreads) void k_pv_reverse(SmallArgs a) {
  // counters, each wavefront's array aligned to its size (the tally's
  // AND-OR addresses); one dummy word per lane
  __shared__ __attribute__((aligned(kPVReverseWords * 4))) uint32_t cnt[kPVReverseWaves][kPVReverseWords];
  __shared__ uint32_t dummies[kPVReverseWaves][kWave];
  __shared__ __attribute__((aligned(16))) uint32_t mtab[kPVReverseWaves][kGather];
  __shared__ uint8_t mflag[kPVReverseWaves][kGather];
  // a run's mid credits, balanced | unbalanced << 32: each at most the
  // run's length (< 4096) times 255
  __shared__ unsigned long long cbu[kPVReverseWaves][kWave];
  // the workgroup's key credits, balanced | unbalanced << 32 (each half
  // below 2^31, see above)
  __shared__ unsigned long long ksum[kMaxReverseL];
  // chunk slots in flight per walk: 8 where the registers allow (the
  // per-edge walks keep 4)
  constexpr int kU = kEdge ? 4 : 8;
  // wave index, known to the compiler as wavefront-uniform
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int lane = lane_id();
  uint32_t* C = cnt[wave];
  if (lane == 0 && (lds_addr(C) & (kPVReverseWords * 4 - 1)) != 0) atomicOr(a.err, kErrLdsLayout);
  for (int i = threadIdx.x; i < kMaxReverseL; i += kPVReverseThreads) ksum[i] = 0;
  for (int i = lane; i < kPVReverseWords; i += kWave) C[i] = 0;
  for (int i = lane; i < static_cast<int>(kGather); i += kWave) mflag[wave][i] = 0;
  cbu[wave][lane] = 0;
  wave_sync_lds();
  const Marks<uint8_t> mk{mtab[wave], mflag[wave]};
  SqTotals tot;  // the pass's global counts, from 32-bit per-item sums
  uint32_t graph = kNoGraph;
  const int32_t stride = static_cast<int32_t>(gridDim.x) * kPVReverseWaves;
  for (int32_t i = static_cast<int32_t>(blockIdx.x) * kPVReverseWaves + wave; i < a.n_items; i += stride) {
    const Item it = load_const(a.items, i);
    if (it.graph != graph) {
      if (graph != kNoGraph) tot.flush(a.res + static_cast<size_t>(graph) * kResStride);
      tot = SqTotals{};
      graph = it.graph;
    }
    const DevSideConst sc = load_const(a.sides, 2 * it.graph + it.side);
    const uint32_t seg_end = it.seg_begin + it.seg_count;
    for (uint32_t k0 = it.seg_begin; k0 < seg_end; k0 += kWave) {
      const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
      RunEnds re;
      walk_regs<kU, false, true>(load_seg_pv<false, kEdge>(sc.segs, sc.seg_mid, sc.seg_edge, k0, k1, re), sc.other_adj,
                                mk, a.long_len, PairTallyBF<kPVReverseWords>{lds_addr(C), lds_addr(&dummies[wave][lane])});
    }
    wave_sync_lds();
    for (uint32_t k0 = it.seg_begin; k0 < seg_end; k0 += kWave) {
      const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
      RunEnds re;
      const SegReg sr = load_seg_pv<false, kEdge>(sc.segs, sc.seg_mid, sc.seg_edge, k0, k1, re);
      auto c = credit<kEdge, true, true>(
          [&](uint32_t e, uint32_t, uint32_t& p, uint32_t& n) {
            const uint32_t key = e >> 1;  // (masked: the hoisted reads also take masked slots)
            const uint32_t h = C[(key >> 1) & (kPVReverseWords - 1)] >> ((key & 1u) << 4);
            p = h & 0xffu;
            n = (h >> 8) & 0xffu;
            return true;
          },
          cbu[wave], static_cast<unsigned long long*>(nullptr), sc, re);
      walk_regs<kU, kEdge>(sr, sc.other_adj, mk, a.long_len, c);
      c.flush();
      flush_mid_credits_packed<kEdge>(cbu[wave], re, sc);
    }
    // the key credits: 16-byte reads of the counter words, quads of zero
    // words skipped; a pair with one wedge adds nothing.  p, n <= 255, so a
    // lane's sums over its keys of one item stay in 32 bits.
    SqSums ss;
    uint32_t oc = 0, ox = 0;  // owner sums
    auto local = [&](uint32_t key, uint32_t p, uint32_t n) {
      ss.add(p, n);
      const uint32_t cb2 = (__umul24(p, p - 1u) + __umul24(n, n - 1u)) >> 1, cx = __umul24(p, n);
      if (cb2 | cx) atomicAdd(&ksum[key], (static_cast<unsigned long long>(cx) << 32) | cb2);
      oc += cb2;
      ox += cx;
    };
    const int32_t w_hi = (it.key_hi + 1) >> 1;
    for (int32_t w0 = 4 * lane; w0 < w_hi; w0 += 4 * kWave) {
      const uint4 c4 = *reinterpret_cast<const uint4*>(&C[w0]);
      if ((c4.x | c4.y | c4.z | c4.w) == 0) continue;
      *reinterpret_cast<uint4*>(&C[w0]) = make_uint4(0, 0, 0, 0);
      const uint32_t cw[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t c2 = cw[q];
        const uint32_t wd = static_cast<uint32_t>(w0 + q);
        if (c2 & 0xffffu) local(2 * wd, c2 & 0xffu, (c2 >> 8) & 0xffu);
        if (c2 >> 16) local(2 * wd + 1, (c2 >> 16) & 0xffu, c2 >> 24);
      }
    }
    tot.add(ss);
    const int64_t oc2 = wave_sum64(oc), ox2 = wave_sum64(ox);
    if (lane == 0) {
      if (oc2) atomicAdd(&sc.bal[sc.orig[it.owner]], static_cast<unsigned long long>(oc2));
      if (ox2) atomicAdd(&sc.unb[sc.orig[it.owner]], static_cast<unsigned long long>(ox2));
    }
    wave_sync_lds();
  }
  __shared__ WaveSums wsum[kPVReverseWaves];
  flush_block_end(tot, graph, wsum, kPVReverseWaves, a.res);
  // the workgroup's key credits (all items of a launch are of one side)
  __syncthreads();
  if (a.n_items > 0) {
    const Item i0 = load_const(a.items, 0);
    const DevSideConst sc = load_const(a.sides, 2 * i0.graph + i0.side);
    const int32_t nkeys = sc.R < kMaxReverseL ? sc.R : kMaxReverseL;
    for (int k = threadIdx.x; k < nkeys; k += kPVReverseThreads) {
      const unsigned long long v = ksum[k], b = v & 0xffffffffull, u = v >> 32;
      if (b) atomicAdd(&sc.bal[sc.orig[k]], b);
      if (u) atomicAdd(&sc.unb[sc.orig[k]], u);
    }
  }
}

// ---------------------------------------------------------------------------
// Small-item groups: one wavefront per group, the group hash of the count
// pass; owners come from the group's owner list.
constexpr int kPVSmallThreads = 256;
constexpr int kPVSmallWaves = kPVSmallThreads / kWave;
constexpr int kPVSmallSlots = 2 * kSmallGroupWork;

template <bool kEdge>
__global__ __launch_bounds__(kPVSmallThreads) void k_pv_small(SmallArgs a) {
  __shared__ uint32_t keys[kPVSmallWaves][kPVSmallSlots];
  __shared__ uint32_t vals[kPVSmallWaves][kPVSmallSlots];
  __shared__ __attribute__((aligned(16))) uint32_t mtab[kPVSmallWaves][kGather];
  __shared__ uint32_t mflag[kPVSmallWaves][kGather];
  __shared__ unsigned long long cb[kPVSmallWaves][kWave], cu[kPVSmallWaves][kWave];
  // wave index, known to the compiler as wavefront-uniform
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int lane = lane_id();
  uint32_t* K = keys[wave];
  uint32_t* V = vals[wave];
  for (int i = lane; i < kPVSmallSlots; i += kWave) {
    K[i] = kEmpty;
    V[i] = 0;
  }
  for (int i = lane; i < static_cast<int>(kGather); i += kWave) mflag[wave][i] = 0;
  cb[wave][lane] = 0;
  cu[wave][lane] = 0;
  wave_sync_lds();
  const Marks<uint32_t> mk{mtab[wave], mflag[wave]};
  Sums sums;
  uint32_t graph = kNoGraph;
  const int32_t stride = static_cast<int32_t>(gridDim.x) * kPVSmallWaves;
  for (int32_t i = static_cast<int32_t>(blockIdx.x) * kPVSmallWaves + wave; i < a.n_items; i += stride) {
    const Item it = load_const(a.items, i);
    if (it.graph != graph) {
      if (graph != kNoGraph) flush_sums(sums, a.res + static_cast<size_t>(graph) * kResStride);
      sums = Sums{};
      graph = it.graph;
    }
    const DevSideConst sc = load_const(a.sides, 2 * it.graph + it.side);
    const uint32_t kb = static_cast<uint32_t>(sc.key_bits);
    uint32_t size = 64;
    while (size < 2 * it.work) size <<= 1;
    const uint32_t mask = size - 1;
    const uint32_t seg_end = it.seg_begin + it.seg_count;
    auto hkey = [&](uint32_t e, uint32_t tag) { return (((tag & ~kMidWide) >> 7) << kb) | (e >> 1); };
    // a hub pivot's group (alone in it): keys below T as in k_pv_direct
    const uint32_t hubT = (it.flags & kItemHubPairs) ? static_cast<uint32_t>(sc.T) : 0u;
    for (uint32_t k0 = it.seg_begin; k0 < seg_end; k0 += kWave) {
      const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
      RunEnds re;
      walk_regs<4>(load_seg_pv<true, kEdge>(sc.small_segs, sc.small_seg_mid, sc.small_seg_edge, k0, k1, re), sc.other_adj, mk,
                   a.long_len, hash_tally([&](uint32_t e, uint32_t tag) {
                     const uint32_t key = hkey(e, tag);
                     const uint32_t inc = ((e ^ tag) & 1u) ? 0x10000u : 1u;
                     uint32_t h = mix32(key) & mask;
                     const uint32_t st = probe_step(key, mask);
                     for (uint32_t probe = 0;; ++probe) {
                       if (probe > mask) {  // full table: cannot happen at load <= 1/2
                         atomicOr(a.err, kErrHashFull);
                         break;
                       }
                       // one compare-and-swap per probe (claims an empty slot)
                       const uint32_t c = atomicCAS(&K[h], kEmpty, key);
                       if (c == kEmpty || c == key) {
                         atomicAdd(&V[h], inc);
                         break;
                       }
                       h = (h + st) & mask;
                     }
                   }));
    }
    wave_sync_lds();
    for (uint32_t k0 = it.seg_begin; k0 < seg_end; k0 += kWave) {
      const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
      RunEnds re;
      const SegReg sr = load_seg_pv<true, kEdge>(sc.small_segs, sc.small_seg_mid, sc.small_seg_edge, k0, k1, re);
      if (hubT == 0) {
        // a plain group has at most kSmallGroupWork wedges: a run's credits
        // stay below 2^18, so one packed LDS word per run
        auto c = credit<kEdge, false, true>(
            [&](uint32_t e, uint32_t tag, uint32_t& p, uint32_t& n) {
              const uint32_t key = hkey(e, tag);
              uint32_t h = mix32(key) & mask;
              const uint32_t st = probe_step(key, mask);
              for (uint32_t probe = 0; probe <= mask; ++probe) {
                if (K[h] == key) {
                  const uint32_t v = V[h];
                  p = v & 0xffffu;
                  n = v >> 16;
                  return true;
                }
                h = (h + st) & mask;
              }
              atomicOr(a.err, kErrHashFull);  // a tallied key must be there
              return false;
            },
            cb[wave], static_cast<unsigned long long*>(nullptr), sc, re);
        walk_regs<4, kEdge>(sr, sc.other_adj, mk, a.long_len, c);
        c.flush();
        flush_mid_credits_packed<kEdge>(cb[wave], re, sc);
        continue;
      }
      auto c = credit<kEdge>(
          [&](uint32_t e, uint32_t tag, uint32_t& p, uint32_t& n) {
            if ((e >> 1) < hubT) {
              hub_counts(sc, static_cast<uint32_t>(it.owner), e >> 1, p, n);
              return true;
            }
            const uint32_t key = hkey(e, tag);
            uint32_t h = mix32(key) & mask;
            const uint32_t st = probe_step(key, mask);
            for (uint32_t probe = 0; probe <= mask; ++probe) {
              if (K[h] == key) {
                const uint32_t v = V[h];
                p = v & 0xffffu;
                n = v >> 16;
                return true;
              }
              h = (h + st) & mask;
            }
            atomicOr(a.err, kErrHashFull);  // a tallied key must be there
            return false;
          },
          cb[wave], cu[wave], sc, re);
      walk_regs<4, kEdge>(sr, sc.other_adj, mk, a.long_len, c);
      c.flush();
      flush_mid_credits<kEdge>(cb[wave], cu[wave], re, sc);
    }
    const uint32_t kmask = (1u << kb) - 1u;
    for (uint32_t h = lane; h < size; h += kWave) {
      const uint32_t key = K[h];
      if (key == kEmpty) continue;
      const uint32_t v = V[h];
      K[h] = kEmpty;
      V[h] = 0;
      if ((key & kmask) < hubT) continue;  // a hub pair: credited by the dense block
      PairCredit pc;
      pc.add(sc, key & kmask, v & 0xffffu, v >> 16, sums);
      if (pc.c | pc.x) {  // a pair with one wedge credits nothing
        const int32_t id = sc.orig[sc.small_owner[it.acc_slot + static_cast<int32_t>(key >> kb)]];
        if (pc.c) atomicAdd(&sc.bal[id], static_cast<unsigned long long>(pc.c));
        if (pc.x) atomicAdd(&sc.unb[id], static_cast<unsigned long long>(pc.x));
      }
    }
    wave_sync_lds();
  }
  __shared__ WaveSums wsum[kPVSmallWaves];
  flush_block_end(sums, graph, wsum, kPVSmallWaves, a.res);
}

// ---------------------------------------------------------------------------
// Hash items (large pivots below the window): one workgroup per item, a
// shared hash with 32-bit p and n; items with many endpoints are done in
// passes over a partition of the keys, each pass tallying, crediting and
// sweeping its keys.
constexpr int kPVHashThreads = 512;
constexpr int kPVHashWaves = kPVHashThreads / kWave;
constexpr int kPVHashSlots = 8192;

template <bool kEdge>
__global__ __launch_bounds__(kPVHashThreads) void k_pv_hash(HashArgs a) {
  __shared__ uint32_t keys[kPVHashSlots];
  __shared__ unsigned long long vals[kPVHashSlots];
  __shared__ __attribute__((aligned(16))) uint32_t mtab[kPVHashWaves][kGather];
  __shared__ uint32_t mflag[kPVHashWaves][kGather];
  __shared__ unsigned long long cb[kPVHashWaves][kWave], cu[kPVHashWaves][kWave];
  __shared__ int32_t item_sh;
  __shared__ uint32_t work_sh;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = lane_id();
  for (int i = tid; i < kPVHashSlots; i += kPVHashThreads) {
    keys[i] = kEmpty;
    vals[i] = 0;
  }
  for (int i = tid; i < kPVHashWaves * static_cast<int>(kGather); i += kPVHashThreads) (&mflag[0][0])[i] = 0;
  cb[wave][lane] = 0;
  cu[wave][lane] = 0;
  const Marks<uint32_t> mk{mtab[wave], mflag[wave]};
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
    for (uint32_t k = it.seg_begin + tid; k < seg_end; k += kPVHashThreads) w += as_global(&sc.segs[k].len_g)[0] >> 1;
    atomicAdd(&work_sh, w);
    __syncthreads();
    const uint32_t passes = (work_sh + kPVHashSlots / 4 - 1) / (kPVHashSlots / 4);
    PairCredit pc;
    for (uint32_t pass = 0; pass < passes; ++pass) {
      auto mine = [&](uint32_t key, uint32_t& hk) {
        hk = mix32(key);
        return passes == 1 || (hk >> 16) % passes == pass;
      };
      for (uint32_t k0 = it.seg_begin + wave * kWave; k0 < seg_end; k0 += kPVHashThreads) {
        const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
        RunEnds re;
        walk_regs<4>(load_seg_pv<false, kEdge>(sc.segs, sc.seg_mid, sc.seg_edge, k0, k1, re), sc.other_adj, mk, a.long_len,
                     hash_tally([&](uint32_t e, uint32_t tag) {
                       const uint32_t key = e >> 1;
                       uint32_t hk;
                       if (!mine(key, hk)) return;
                       const unsigned long long inc = ((e ^ tag) & 1u) ? (1ull << 32) : 1ull;
                       uint32_t h = hk & (kPVHashSlots - 1);
                       const uint32_t st = probe_step(key, kPVHashSlots - 1);
                       for (uint32_t probe = 0;; ++probe) {
                         if (probe >= static_cast<uint32_t>(kPVHashSlots)) {
                           atomicOr(a.err, kErrHashFull);
                           break;
                         }
                         // one compare-and-swap per probe (claims an empty slot)
                         const uint32_t c = atomicCAS(&keys[h], kEmpty, key);
                         if (c == kEmpty || c == key) {
                           atomicAdd(&vals[h], inc);
                           break;
                         }
                         h = (h + st) & (kPVHashSlots - 1);
                       }
                     }));
      }
      __syncthreads();
      for (uint32_t k0 = it.seg_begin + wave * kWave; k0 < seg_end; k0 += kPVHashThreads) {
        const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
        RunEnds re;
        const SegReg sr = load_seg_pv<false, kEdge>(sc.segs, sc.seg_mid, sc.seg_edge, k0, k1, re);
        auto c = credit<kEdge>(
            [&](uint32_t e, uint32_t, uint32_t& p, uint32_t& n) {
              const uint32_t key = e >> 1;
              uint32_t hk;
              if (!mine(key, hk)) return false;
              uint32_t h = hk & (kPVHashSlots - 1);
              const uint32_t st = probe_step(key, kPVHashSlots - 1);
              for (int probe = 0; probe < kPVHashSlots; ++probe) {
                if (keys[h] == key) {
                  const unsigned long long v = vals[h];
                  p = static_cast<uint32_t>(v);
                  n = static_cast<uint32_t>(v >> 32);
                  return true;
                }
                h = (h + st) & (kPVHashSlots - 1);
              }
              atomicOr(a.err, kErrHashFull);
              return false;
            },
            cb[wave], cu[wave], sc, re);
        walk_regs<4, kEdge>(sr, sc.other_adj, mk, a.long_len, c);
        c.flush();
        flush_mid_credits<kEdge>(cb[wave], cu[wave], re, sc);
      }
      __syncthreads();
      for (int h = tid; h < kPVHashSlots; h += kPVHashThreads) {
        const uint32_t key = keys[h];
        if (key == kEmpty) continue;
        const unsigned long long v = vals[h];
        keys[h] = kEmpty;
        vals[h] = 0;
        pc.add(sc, key, static_cast<uint32_t>(v), static_cast<uint32_t>(v >> 32), sums);
      }
      __syncthreads();
    }
    pc.to_owner(sc, it.owner);
  }
  __shared__ WaveSums wsum[kPVHashWaves];
  flush_block_end(sums, graph, wsum, kPVHashWaves, a.res);
}

// ---------------------------------------------------------------------------
// Per-edge outputs in input-record order: each edge's credits from both
// CSRs (as a run's first edge on one side and as a walked entry on the
// other) added together.  One thread per U-CSR position, grid-stride.
__global__ __launch_bounds__(256) void k_edge_combine(EdgeCombineArgs a) {
  // edges that can hold two-word credits: U-CSR positions below kcut (rows
  // of U ranks below the first narrow one) or V ends ranked below vcut
  int64_t kcut = 0;
  uint32_t vcut = 0;
  if (a.wide) {
    if (a.wide_all) {
      kcut = a.m;
    } else {
      kcut = as_global(a.off_u)[first_narrow_rank(a.off_u, a.n_u, a.max_deg_v)];
      vcut = static_cast<uint32_t>(first_narrow_rank(a.off_v, a.n_v, a.max_deg_u));
    }
  }
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < a.m; k += stride) {
    const uint32_t r = as_global(a.rec)[k];
    const uint32_t q = as_global(a.pos_v)[k];
    const unsigned long long p0 = as_global(a.e_pack[0])[k], p1 = as_global(a.e_pack[1])[q];
    unsigned long long b = (p0 & 0xffffffffull) + (p1 & 0xffffffffull);
    unsigned long long u = (p0 >> 32) + (p1 >> 32);
    // the two-word words of other edges are zero: not read (the V side's
    // are at random positions, a cache line each)
    if (k < kcut || (as_global(a.adj_u)[k] >> 1) < vcut) {
      b += as_global(a.e_wb[0])[k] + as_global(a.e_wb[1])[q];
      u += as_global(a.e_wu[0])[k] + as_global(a.e_wu[1])[q];
    }
    as_global(a.out_bal)[r] = static_cast<long long>(b);
    as_global(a.out_unb)[r] = static_cast<long long>(u);
  }
}

}  // namespace dev

namespace {

template <bool kEdge>
hipError_t direct_(const DirectArgs& a, int grid, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_pv_direct<kEdge>, dim3(grid), dim3(dev::kPVDirectThreads), 0, st, a);
  return hipGetLastError();
}

template <bool kEdge>
hipError_t reverse_(const SmallArgs& a, int grid, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  // at most 2^16 items per workgroup (its 32-bit key sums)
  const int64_t per = int64_t{1} << 16;
  const int64_t need = (static_cast<int64_t>(a.n_items) + per - 1) / per;
  if (grid < need) grid = static_cast<int>(need);
  hipLaunchKernelGGL(dev::k_pv_reverse<kEdge>, dim3(grid), dim3(dev::kPVReverseThreads), 0, st, a);
  return hipGetLastError();
}

template <bool kEdge>
hipError_t small_(const SmallArgs& a, int grid, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_pv_small<kEdge>, dim3(grid), dim3(dev::kPVSmallThreads), 0, st, a);
  return hipGetLastError();
}

template <bool kEdge>
hipError_t hash_(const HashArgs& a, int grid, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_pv_hash<kEdge>, dim3(grid), dim3(dev::kPVHashThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pv_direct(const DirectArgs& a, int grid, hipStream_t st) { return direct_<false>(a, grid, st); }
hipError_t launch_pv_reverse(const SmallArgs& a, int grid, hipStream_t st) { return reverse_<false>(a, grid, st); }
hipError_t launch_pv_small(const SmallArgs& a, int grid, hipStream_t st) { return small_<false>(a, grid, st); }
hipError_t launch_pv_hash(const HashArgs& a, int grid, hipStream_t st) { return hash_<false>(a, grid, st); }
hipError_t launch_pe_direct(const DirectArgs& a, int grid, hipStream_t st) { return direct_<true>(a, grid, st); }
hipError_t launch_pe_reverse(const SmallArgs& a, int grid, hipStream_t st) { return reverse_<true>(a, grid, st); }
hipError_t launch_pe_small(const SmallArgs& a, int grid, hipStream_t st) { return small_<true>(a, grid, st); }
hipError_t launch_pe_hash(const HashArgs& a, int grid, hipStream_t st) { return hash_<true>(a, grid, st); }

hipError_t launch_pv_key_flush(const DevSideConst* sides, int32_t s, int32_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_pv_key_flush, dim3((n + 255) / 256), dim3(256), 0, st, sides, s, n);
  return hipGetLastError();
}

hipError_t launch_edge_combine(const EdgeCombineArgs& a, int grid, hipStream_t st) {
  if (a.m == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_edge_combine, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace dbbc
