// Device primitives shared by the counting kernels (count.hip) and the
// per-vertex kernels (pervertex.hip): the wavefront walk of CSR runs, the
// counter tallies and the int64 sums of Lemma 1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "internal.h"
#include "kernels.h"

namespace dbbc {
namespace dev {

constexpr int kWave = 64;

// Address-space views.  Pointers read from device tables (the per-graph side
// constants) are generic to the compiler, which would then emit flat
// accesses; CSR runs, entries and accumulators are global memory, so they
// are accessed through global (address space 1) views.  Work lists and side
// tables are never written while a kernel runs, so they are read through
// constant (address space 4) views, which the compiler turns into scalar
// loads when the index is uniform.
template <class T>
using global_t = __attribute__((address_space(1))) T;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <class T>
using const_t = __attribute__((address_space(4))) T;

template <class T>
__device__ __forceinline__ const global_t<T>* as_global(const T* p) {
  return (const global_t<T>*)p;
}
template <class T>
__device__ __forceinline__ global_t<T>* as_global(T* p) {
  return (global_t<T>*)p;
}
// Element i of a read-only table (work list, side table), through a
// constant view, word by word (structs cannot be copied out of another
// address space directly; the words merge into one wide scalar load).
template <class T>
__device__ __forceinline__ T load_const(const T* p, size_t i) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  const const_t<uint32_t>* w = (const const_t<uint32_t>*)(p + i);
  T out;
  uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (size_t k = 0; k < sizeof(T) / 4; ++k) o[k] = w[k];
  return out;
}
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

// Segment k0 + stride * lane of [k0, k1) for each lane.
template <bool kTagged>
__device__ __forceinline__ SegReg load_seg(const Segment* __restrict__ segs, uint32_t k0, uint32_t k1,
                                           uint32_t stride = 1) {
  const uint32_t k = k0 + stride * static_cast<uint32_t>(lane_id());
  SegReg r{0, 0, 0};
  if (k < k1) {
    const u32x2 w = *(const global_t<u32x2>*)(segs + k);
    const Segment s{w.x, w.y};
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
// to lanes as t = done + 64 u + lane (coalesced loads), and finds every
// position's run in one of two forms (both keep their per-position LDS
// words zero between rounds: each lane clears what it read):
//  - marks: every run that starts in the round, or continues into it,
//    writes its base and its tag (with the top bit set as a presence flag)
//    at its first position of the round; a position's run is the last mark
//    at or before it (a ballot per block of 64 positions, the highest set
//    bit, two ds_bpermute, carried across blocks);
//  - table: the batch's non-empty short runs are listed in lane order in a
//    run table (base, tag) once per batch, every run that starts in the
//    round flags its first position, and the run of position t is entry
//    r(t) = (flags at or before t) - 1: the flags of earlier blocks
//    (carried) plus a ballot and a masked bit count in its own block.
//    Blocks wholly past the batch's last position are skipped.  Fewer
//    instructions per position, one more dependent LDS read: it pays where
//    the walk is bound by instruction issue.
constexpr int kStageU = kGather / kWave;

// The marks buffers of a wavefront: kGather words (the marks' bases, or
// the run table) and kGather TagT entries (the marks' tags with the
// presence bit, or the start flags).  TagT holds a run's tag plus the
// presence bit: 8 bits for plain runs (tag = g), 32 bits for small-item
// groups.
template <class TagT>
struct Marks {
  uint32_t* base;  // kGather words, 8-byte aligned
  TagT* tag;       // kGather entries, zero between rounds
  static constexpr uint32_t kBit = 1u << (8 * sizeof(TagT) - 1);
};

struct Staged {
  uint32_t e[kStageU], tag[kStageU], pos[kStageU];
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
    s.pos[u] = b + t;
    s.e[u] = as_global(adj)[s.valid[u] ? b + t : 0u];
  }
}

// Count of set bits of m in the lanes below this one.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

// Table form: list the batch's non-empty short runs (before its first
// staging round, whose fence orders these writes before its reads).
template <class M>
__device__ __forceinline__ void fill_table(M mk, uint32_t slen, uint32_t base, uint32_t tag) {
  wave_sync_lds();  // the previous batch's rounds have read the table
  const uint64_t ne = __ballot(slen != 0);
  if (slen != 0) {
    const uint32_t k = mbcnt(ne);
    *reinterpret_cast<u32x2*>(mk.base + 2 * k) = u32x2{base, tag};
  }
}

template <class M>
__device__ __forceinline__ void stage_round_table(Staged& s, M mk, uint32_t excl, uint32_t slen, uint32_t total,
                                                  uint32_t done, uint32_t& carry,
                                                  const uint32_t* __restrict__ adj) {
  const int lane = lane_id();
  wave_sync_lds();
  if (slen != 0 && excl >= done && excl < done + kGather) mk.tag[excl - done] = 1;
  wave_sync_lds();
#pragma unroll
  for (int u = 0; u < kStageU; ++u) {
    s.valid[u] = false;
    if (done + static_cast<uint32_t>(u * kWave) < total) {
      const uint32_t f = static_cast<uint32_t>(mk.tag[u * kWave + lane]);
      mk.tag[u * kWave + lane] = 0;
      const uint64_t fm = __ballot(f != 0);
      const uint32_t r = carry + mbcnt(fm) + f - 1u;  // f is 0 or 1
      carry += static_cast<uint32_t>(__popcll(fm));
      const u32x2 bt = *reinterpret_cast<const u32x2*>(mk.base + 2 * r);
      const uint32_t t = done + static_cast<uint32_t>(u * kWave + lane);
      s.valid[u] = t < total;
      s.tag[u] = bt.y;
      s.pos[u] = bt.x + t;
      s.e[u] = as_global(adj)[s.valid[u] ? bt.x + t : 0u];
    }
  }
}

// Hand one wedge slot to a walk functor: f.add(entry, tag, valid, pos) when
// the functor takes the entry's position in the CSR array (per-edge
// credits), else f.add(entry, tag, valid).
template <class F>
__device__ __forceinline__ auto walk_add(F& f, uint32_t e, uint32_t tag, bool valid, uint32_t pos, int)
    -> decltype(f.add(e, tag, valid, pos), void()) {
  f.add(e, tag, valid, pos);
}
template <class F>
__device__ __forceinline__ void walk_add(F& f, uint32_t e, uint32_t tag, bool valid, uint32_t, long) {
  f.add(e, tag, valid);
}
// A slot of a streamed chunk: every lane's slot belongs to the same run (the
// chunk's), so a functor may keep per-run state wave-uniform
// (f.add_chunk(entry, tag, valid, pos)); otherwise as walk_add.
template <class F>
__device__ __forceinline__ auto walk_add_chunk(F& f, uint32_t e, uint32_t tag, bool valid, uint32_t pos, int)
    -> decltype(f.add_chunk(e, tag, valid, pos), void()) {
  f.add_chunk(e, tag, valid, pos);
}
template <class F>
__device__ __forceinline__ void walk_add_chunk(F& f, uint32_t e, uint32_t tag, bool valid, uint32_t pos, long) {
  walk_add(f, e, tag, valid, pos, 0);
}

// A functor that takes a staging round's slots at once (add_staged(Staged)),
// flagged by a static member kStaged.
template <class F, class = void>
struct HasStaged : std::false_type {};
template <class F>
struct HasStaged<F, std::enable_if_t<F::kStaged>> : std::true_type {};

// Walk a batch of up to 64 runs (one per lane, in registers) with one
// wavefront, calling f.add(entry, tag, valid[, pos]) once per wedge slot.
//  - Runs of at least long_len entries are consumed as a stream of
//    256-entry chunks: every lane loads 4 aligned entries (16 bytes) per
//    chunk, U chunks are in flight per lane, and a chunk's words past the
//    run's end are masked.  The chunk loop is wavefront-uniform.  The 0-3
//    entries before a long run's first 16-byte boundary are staged with the
//    short runs, so every chunk starts inside its run and a slot's test is
//    one compare of its offset in the chunk with the run's remaining
//    length.  With kLaneMajor the lane's 4 entries are instead 64 apart
//    (four 4-byte loads), so that each of the 4 calls of a chunk sees 64
//    consecutive positions across the lanes (per-position global atomics
//    of a functor then coalesce).
//  - Shorter runs are staged (stage_round) so that every lane holds wedges;
//    the loads of the first round are issued before the long stream and the
//    next round's loads before the current round is tallied.
// kCompact selects the issue-lean form: staging by run table, and chunks
// that lie wholly inside their run tallied without the slot test.  The
// counting kernels with direct LDS counters use it; the hash-table and
// per-vertex walks (bound by latency, or with functors whose code is large)
// measured faster in the plain form.
template <int U, bool kLaneMajor = false, bool kCompact = false, class M, class F>
__device__ __forceinline__ void walk_regs(SegReg sr, const uint32_t* __restrict__ adj, M marks,
                                          uint32_t long_len, F&& f) {
  const int lane = lane_id();
  const uint32_t start = sr.start, tag = sr.tag, len = sr.len;
  // long_len >= 16, so a long run keeps at least 13 entries after its head
  const bool is_long = len >= long_len;
  const uint32_t head = is_long ? (0u - start) & 3u : 0u;
  uint64_t longm = __ballot(is_long);
  const uint32_t slen = is_long ? head : len;
  uint32_t total;
  const uint32_t excl = wave_excl_scan(slen, &total);
  const uint32_t base = start - excl;
  const uint32_t lstart = start + head, lend = start + len;
  Staged cur;
  uint32_t carry = 0;  // table form: flags of the staged blocks before the current one
  // The first staging round's loads go out before the long stream's (marks
  // form) or right after its first chunk loads (issue-lean form, so that
  // the chunk loads need not wait for them).
  bool staged = false;
  auto first_round = [&]() {
    staged = true;
    if (!total) return;
    if (kCompact) {
      fill_table(marks, slen, base, tag);
      stage_round_table(cur, marks, excl, slen, total, 0, carry, adj);
    } else {
      stage_round(cur, marks, excl, slen, base, tag, total, 0, adj);
    }
  };
  if (!kCompact) first_round();
  uint32_t cur_end = 0, cur_g = 0, cur_pos = 0;
  bool have = false;
  // offset of a lane's word q in a chunk (loop-invariant)
  uint32_t koff[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) koff[q] = kLaneMajor ? lane + q * kWave : 4 * lane + q;
  while (longm || have) {
    u32x4 v[U];
    uint32_t vrem[U], vg[U], vpos[U];
    int nv = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!have) {
        if (!longm) break;  // the batch's long runs are done (uniform)
        const int j = __ffsll(static_cast<unsigned long long>(longm)) - 1;
        longm &= longm - 1;
        cur_pos = readlane(lstart, j);
        cur_end = readlane(lend, j);
        cur_g = readlane(tag, j);
        have = true;
      }
      // The load is unconditional within the chunk: lanes past the run's
      // end read the first entries of the array, and their words fail the
      // offset test below.
      const uint32_t p = cur_pos + (kLaneMajor ? lane : 4 * lane);
      vg[u] = cur_g;
      vpos[u] = cur_pos;
      vrem[u] = cur_end - cur_pos;  // entries left in the run from the chunk's start
      if (kLaneMajor) {
        const global_t<uint32_t>* a = as_global(adj);
        v[u].x = a[p < cur_end ? p : 0u];
        v[u].y = a[p + kWave < cur_end ? p + kWave : 0u];
        v[u].z = a[p + 2 * kWave < cur_end ? p + 2 * kWave : 0u];
        v[u].w = a[p + 3 * kWave < cur_end ? p + 3 * kWave : 0u];
      } else {
        v[u] = *(const global_t<u32x4>*)(adj + (p < cur_end ? p : 0u));
      }
      nv = u + 1;
      cur_pos += kChunk;
      if (cur_pos >= cur_end) have = false;
    }
    if (!staged) first_round();
    // slots past the last issued chunk (the batch's long runs ran out) hold
    // no entries: skip them (nv is wavefront-uniform)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (u < nv) {
        const uint32_t e4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
        if (kCompact && vrem[u] >= kChunk) {  // the whole chunk lies in the run (uniform)
#pragma unroll
          for (int q = 0; q < 4; ++q) walk_add_chunk(f, e4[q], vg[u], true, vpos[u] + koff[q], 0);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) walk_add_chunk(f, e4[q], vg[u], koff[q] < vrem[u], vpos[u] + koff[q], 0);
        }
      }
    }
  }
  if (!staged) first_round();
  for (uint32_t done = 0; done < total; done += kGather) {
    const bool more = done + kGather < total;
    Staged nxt;
    if (more) {
      if (kCompact)
        stage_round_table(nxt, marks, excl, slen, total, done + kGather, carry, adj);
      else
        stage_round(nxt, marks, excl, slen, base, tag, total, done + kGather, adj);
    }
    if constexpr (HasStaged<std::remove_reference_t<F>>::value) {
      f.add_staged(cur);
    } else {
#pragma unroll
      for (int u = 0; u < kStageU; ++u)
        if (!kCompact || done + static_cast<uint32_t>(u * kWave) < total)
          walk_add(f, cur.e[u], cur.tag[u], cur.valid[u], cur.pos[u], 0);
    }
    if (!more) break;
    cur = nxt;
  }
}

template <int U, bool kTagged = false, bool kCompact = false, class M, class F>
__device__ __forceinline__ void walk_batch(const Segment* __restrict__ segs, uint32_t k0, uint32_t k1,
                                           const uint32_t* __restrict__ adj, M marks,
                                           uint32_t long_len, F&& f, uint32_t stride = 1) {
  walk_regs<U, false, kCompact>(load_seg<kTagged>(segs, k0, k1, stride), adj, marks, long_len, f);
}

// Walk every run of an item with one wavefront; the first batch of 64 runs
// was loaded beforehand (first).
template <int U, bool kTagged = false, bool kCompact = false, class M, class F>
__device__ __forceinline__ void walk_item(const Item& it, SegReg first, const Segment* __restrict__ segs,
                                          const uint32_t* __restrict__ adj, M marks,
                                          uint32_t long_len, F&& f) {
  const uint32_t seg_end = it.seg_begin + it.seg_count;
  walk_regs<U, false, kCompact>(first, adj, marks, long_len, f);
  for (uint32_t k0 = it.seg_begin + kWave; k0 < seg_end; k0 += kWave) {
    const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
    walk_regs<U, false, kCompact>(load_seg<kTagged>(segs, k0, k1), adj, marks, long_len, f);
  }
}

template <bool kTagged = false>
__device__ __forceinline__ SegReg first_batch(const Item& it, const Segment* __restrict__ segs) {
  const uint32_t seg_end = it.seg_begin + it.seg_count;
  return load_seg<kTagged>(segs, it.seg_begin,
                           it.seg_begin + kWave < seg_end ? it.seg_begin + kWave : seg_end);
}

// Packed counter increment of one wedge: +1 symmetric or +2^16 asymmetric,
// i.e. 1 << 16 (e ^ g) taken mod 32 (only bit 0 of e and g matters).  Sums
// are XORs mod 2, so the shift is the one multiply-add 16 e + 16 g, whose
// bits past the fifth the shift instruction ignores.
__device__ __forceinline__ uint32_t wedge_inc(uint32_t e, uint32_t g) {
  return 1u << (((e << 4) + (g << 4)) & 31u);
}

// Tally functors for walk_regs: add(entry, g, valid) counts a valid
// entry's wedge in the counter of its key (a non-returning LDS atomic, so a
// wavefront never waits on its own counter updates).  In a pair-counter
// word (8|8-bit counters, two keys per 32-bit word) the entry's low bits
// select the byte: bit 0 (negative) ^ g picks the symmetric / asymmetric
// byte, bit 1 (key parity) the 16-bit half.
// A masked slot adds into a dummy word of its own lane (outside the
// counters) instead of switching the execution mask around every atomic;
// dummy words are never read.  DirectTallyBF reduces the key index modulo
// its array's size (a power of two; valid keys are always below it), so a
// key can never address past the array.  PairTallyBF does no such
// reduction: it relies on every key of a reverse item lying in the reverse
// window, a bound the planner checks once per plan.
template <uint32_t kWords>
struct DirectTallyBF {
  uint32_t* cnt;    // kWords counters
  uint32_t* dummy;  // this lane's dummy word
  __device__ __forceinline__ void add(uint32_t e, uint32_t g, bool valid) const {
    static_assert((kWords & (kWords - 1)) == 0, "power of two");
    atomicAdd(valid ? cnt + ((e >> 1) & (kWords - 1)) : dummy, wedge_inc(e, g));
  }
};

// 8|8-bit pair counters addressed by LDS byte address: base is aligned to
// the array's size and a valid slot's key is below 2 kWords (every key of a
// reverse item lies in the reverse window), so the word's address
// base | (e & ~3) is one AND-OR instruction.
typedef __attribute__((address_space(3))) uint32_t lds_u32;
__device__ __forceinline__ uint32_t lds_addr(uint32_t* p) {
  return static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_u32*)p));
}
template <uint32_t kWords>
struct PairTallyBF {
  uint32_t base;   // LDS address of kWords counter words (2 kWords keys), aligned to 4 kWords
  uint32_t dummy;  // LDS address of this lane's dummy word
  __device__ __forceinline__ void add(uint32_t e, uint32_t g, bool valid) const {
    const uint32_t a = valid ? base | (e & ~3u) : dummy;
    atomicAdd((uint32_t*)(lds_u32*)static_cast<uintptr_t>(a), 1u << (((e ^ (g & 1u)) & 3u) << 3));
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

// The sparse wedges of hub pair (owner, key), handed to the dense path as
// p + n and p - n (the form of its accumulators).
__device__ __forceinline__ void hub_partial(const DevSideConst& sc, int32_t owner, uint32_t key, uint32_t p,
                                            uint32_t n) {
  const size_t i = static_cast<size_t>(owner) * sc.T + key;
  global_t<int32_t>* xy = as_global(sc.hub_xy);
  xy[i] = static_cast<int32_t>(p + n);
  xy[i + static_cast<size_t>(sc.T) * sc.T] = static_cast<int32_t>(p) - static_cast<int32_t>(n);
}

// Final fate of one pair count of an item.
__device__ __forceinline__ void emit(const Item& it, uint32_t key, uint32_t p, uint32_t n,
                                     const DevSideConst& sc, Sums& s) {
  if ((it.flags & kItemHubPairs) && static_cast<int32_t>(key) < sc.T) {
    hub_partial(sc, it.owner, key, p, n);
  } else {
    s.add(p, n);
  }
}

// Per-key sums of squares: with W the wedges of the swept keys (sum of
// p + n), sum C(p,2) + C(n,2) = (sum p^2 + n^2 - W) / 2 and the unbalanced
// sum is sum p * n.  32-bit per-item accumulators (24-bit multiply-adds):
// the callers bound p and n so that an item's sums stay below 2^32.
struct SqSums {
  uint32_t sq = 0, pn = 0, w = 0;
  __device__ __forceinline__ void add(uint32_t p, uint32_t n) {
    sq += __umul24(p, p);
    sq += __umul24(n, n);
    pn += __umul24(p, n);
    w += p + n;
  }
};

// Running per-lane totals of SqSums (and of twice a sum p * n, pn2, where
// it comes as such), flushed once per wavefront.
struct SqTotals {
  uint64_t sq = 0, pn = 0, pn2 = 0, w = 0;
  __device__ __forceinline__ void add(const SqSums& s) {
    sq += s.sq;
    pn += s.pn;
    w += s.w;
  }
  __device__ __forceinline__ void flush(unsigned long long* res) const {
    const int64_t q = wave_sum64(static_cast<int64_t>(sq));
    const int64_t x = wave_sum64(static_cast<int64_t>(pn)) + wave_sum64(static_cast<int64_t>(pn2)) / 2;
    const int64_t ww = wave_sum64(static_cast<int64_t>(w));
    if (lane_id() == 0) {
      const int64_t bal = (q - ww) / 2;
      if (bal) atomicAdd(res + kResBalanced, static_cast<unsigned long long>(bal));
      if (x) atomicAdd(res + kResUnbalanced, static_cast<unsigned long long>(x));
      if (bal + x) atomicAdd(res + kResTotal, static_cast<unsigned long long>(bal + x));
    }
  }
};

// The last flush of a launch, taken by every wavefront of a workgroup at
// the kernel's end: each wavefront's sums go to LDS, and one thread adds them
// to the result slots once per graph (a run of wavefronts of one graph).
// Every wavefront of a launch adds to the same few words, and atomics to one
// address are serialized, so per-wavefront atomics would cost a few
// microseconds per thousand wavefronts at the end of the kernel.
// The first rank of a side whose degree d has d * other < 2^32 (side ranks
// are in non-increasing degree order).  Edges at rows of lower rank, or
// whose mid in a run is of lower rank, may hold per-edge credits of 2^32 or
// more: two-word credits; any other edge's credits stay below 2^32 (an edge
// (x, y) lies in at most (deg x - 1)(deg y - 1) butterflies).
__device__ __forceinline__ int32_t first_narrow_rank(const uint32_t* off, int32_t n, unsigned long long other) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = lo + (hi - lo) / 2;
    const unsigned long long d = as_global(off)[mid + 1] - as_global(off)[mid];
    if (d * other >= (1ull << 32))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

struct WaveSums {
  int64_t bal, unb;
  uint32_t graph, pad;
};
// bal, unb: the wavefront's balanced and unbalanced counts (wavefront-uniform)
__device__ __forceinline__ void flush_block_end(int64_t bal, int64_t unb, uint32_t graph, WaveSums* sh, int nwaves,
                                                unsigned long long* res) {
  const int wave = static_cast<int>(threadIdx.x) / kWave;
  if (lane_id() == 0) sh[wave] = WaveSums{bal, unb, graph, 0u};
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t g = kNoGraph;
    int64_t b = 0, u = 0;
    auto add = [&]() {
      unsigned long long* r = res + static_cast<size_t>(g) * kResStride;
      if (b) atomicAdd(r + kResBalanced, static_cast<unsigned long long>(b));
      if (u) atomicAdd(r + kResUnbalanced, static_cast<unsigned long long>(u));
      if (b + u) atomicAdd(r + kResTotal, static_cast<unsigned long long>(b + u));
    };
    for (int w = 0; w < nwaves; ++w) {
      const WaveSums v = sh[w];
      if (v.graph == kNoGraph) continue;  // a wavefront without items
      if (v.graph != g) {
        if (g != kNoGraph) add();
        g = v.graph;
        b = u = 0;
      }
      b += v.bal;
      u += v.unb;
    }
    if (g != kNoGraph) add();
  }
}
__device__ __forceinline__ void flush_block_end(const SqTotals& t, uint32_t graph, WaveSums* sh, int nwaves,
                                                unsigned long long* res) {
  const int64_t q = wave_sum64(static_cast<int64_t>(t.sq));
  const int64_t x = wave_sum64(static_cast<int64_t>(t.pn)) + wave_sum64(static_cast<int64_t>(t.pn2)) / 2;
  const int64_t ww = wave_sum64(static_cast<int64_t>(t.w));
  flush_block_end((q - ww) / 2, x, graph, sh, nwaves, res);
}
// (Sums: its total is bal + unb, C(p + n, 2) = C(p, 2) + C(n, 2) + p n)
__device__ __forceinline__ void flush_block_end(const Sums& s, uint32_t graph, WaveSums* sh, int nwaves,
                                                unsigned long long* res) {
  flush_block_end(wave_sum64(s.bal), wave_sum64(s.unb), graph, sh, nwaves, res);
}

// Probe stride of key in a power-of-two table (mask = size - 1): odd, so
// size probes visit every slot; from a multiplicative hash independent of
// the home slot's (double hashing: no clusters of consecutive taken slots).
__device__ __forceinline__ uint32_t probe_step(uint32_t key, uint32_t mask) {
  return (((key * 0x85EBCA6Bu) >> 16) | 1u) & mask;
}

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

}  // namespace dev
}  // namespace dbbc
