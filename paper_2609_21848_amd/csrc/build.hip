// Device construction of the priority-ordered CSR pair (Definition 3 relabel,
// the paper's Phase 2 "global index" on one device) with the per-entry
// reverse positions that let a wedge walk start without a search, and the
// closed-form VP wedge count.  Radix sorts (hipCUB) do the orderings:
//   1. last-wins dedup: records sorted by (u, v), stable, so the last record
//      of a run of equal pairs is the one kept;
//   2. per side, vertices sorted by (degree desc, id desc): side ranks;
//      all vertices together by (degree desc, global id desc): global ranks;
//   3. per side, kept records sorted by (own side rank, other side rank):
//      the rows of the CSR, each row's neighbours in priority order.
// The host receives a copy of the arrays the planner reads; the device keeps
// the CSR entry arrays (with the zero padding the 16-byte walk loads need)
// and the row offsets.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "build_dev.h"
#include "kernels.h"

namespace dbbc {
namespace {

constexpr int kThreads = 256;

int grid_for(int64_t n) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 1 << 16)));
}

#define GRID_STRIDE(i, n)                                                                    \
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); \
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)

// Bits needed for the values 0 .. n - 1 (at least 1).
int bits_for(int64_t n) {
  int b = 1;
  while ((int64_t{1} << b) < n) ++b;
  return b;
}

// Smallest bad record per kind: bad[0] an id out of range, bad[1] a sign
// other than +1 / -1.
__global__ void k_validate(const int32_t* u, const int32_t* v, const int8_t* s, int64_t m, int32_t n_u,
                           int32_t n_v, unsigned long long* bad) {
  GRID_STRIDE(i, m) {
    const int32_t a = u[i], b = v[i];
    if (a < 0 || a >= n_u || b < 0 || b >= n_v) atomicMin(&bad[0], static_cast<unsigned long long>(i));
    const int8_t g = s[i];
    if (g != 1 && g != -1) atomicMin(&bad[1], static_cast<unsigned long long>(i));
  }
}

__global__ void k_pair_keys(const int32_t* u, const int32_t* v, int64_t m, int vbits, uint64_t* keys,
                            uint32_t* vals) {
  GRID_STRIDE(i, m) {
    keys[i] = (static_cast<uint64_t>(u[i]) << vbits) | static_cast<uint32_t>(v[i]);
    vals[i] = static_cast<uint32_t>(i);
  }
}

// Sorted (u, v) keys: the last record of each run of equal keys is kept.
__global__ void k_last_of_run(const uint64_t* keys, int64_t m, uint8_t* keep) {
  GRID_STRIDE(i, m) keep[i] = (i + 1 == m || keys[i + 1] != keys[i]) ? 1 : 0;
}

// Degrees from the sorted (u, v) keys of all records and their keep flags.
// Records of one u are adjacent: each wavefront adds the kept records of a
// run of equal u with one atomic (the heavy rows' counters would otherwise
// take one atomic per edge); the v counters take one atomic per kept record.
__global__ void k_degrees(const uint64_t* keys, const uint8_t* keep, int64_t m, int vbits, uint32_t* deg_u,
                          uint32_t* deg_v) {
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const uint64_t vmask = (uint64_t{1} << vbits) - 1;
  // whole wavefronts loop together (the run sums use the whole wavefront)
  const int64_t span = (m + 63) / 64 * 64;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < span;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const bool in = i < m;
    const uint64_t key = in ? keys[i] : ~uint64_t{0};
    const bool kept = in && keep[i];
    const uint32_t u = static_cast<uint32_t>(key >> vbits);
    const uint32_t u_prev = __shfl_up(u, 1, 64);
    const bool head = lane == 0 || u != u_prev;
    const unsigned long long heads = __ballot(head);
    const unsigned long long keeps = __ballot(kept);
    if (kept) atomicAdd(&deg_v[key & vmask], 1u);
    if (head && in) {
      // this lane's run: lanes [lane, next head)
      const unsigned long long later = heads & ~((2ull << lane) - 1ull);
      const int next = later ? __builtin_ctzll(later) : 64;
      const unsigned long long upto = next == 64 ? ~0ull : ((1ull << next) - 1ull);
      const uint32_t c = static_cast<uint32_t>(__popcll(keeps & upto & ~((1ull << lane) - 1ull)));
      if (c) atomicAdd(&deg_u[u], c);
    }
  }
}

// Key of vertex x for the order (degree desc, id desc): ascending keys.
__global__ void k_prio_keys(const uint32_t* deg, int32_t n, uint32_t maxdeg, int idbits, uint64_t* keys) {
  GRID_STRIDE(x, n) {
    keys[x] = (static_cast<uint64_t>(maxdeg - deg[x]) << idbits) | static_cast<uint64_t>(n - 1 - x);
  }
}

// Sorted keys -> ord (side rank -> id) and sr (id -> side rank).
__global__ void k_prio_ranks(const uint64_t* sorted, int32_t n, int idbits, int32_t* ord, int32_t* sr) {
  GRID_STRIDE(r, n) {
    const int32_t x = n - 1 - static_cast<int32_t>(sorted[r] & ((uint64_t{1} << idbits) - 1));
    ord[r] = x;
    sr[x] = static_cast<int32_t>(r);
  }
}

// Both sides in one order: global id gid = x for U, n_u + y for V.
__global__ void k_global_keys(const uint32_t* deg_u, const uint32_t* deg_v, int32_t n_u, int32_t n_v,
                              uint32_t maxdeg, int idbits, uint64_t* keys) {
  const int32_t n = n_u + n_v;
  GRID_STRIDE(gid, n) {
    const uint32_t d = gid < n_u ? deg_u[gid] : deg_v[gid - n_u];
    keys[gid] = (static_cast<uint64_t>(maxdeg - d) << idbits) | static_cast<uint64_t>(n - 1 - gid);
  }
}

// Global rank of each vertex, stored by side rank.
__global__ void k_global_ranks(const uint64_t* sorted, int32_t n_u, int32_t n_v, int idbits, const int32_t* sr_u,
                               const int32_t* sr_v, int32_t* grank_u, int32_t* grank_v) {
  const int32_t n = n_u + n_v;
  GRID_STRIDE(r, n) {
    const int32_t gid = n - 1 - static_cast<int32_t>(sorted[r] & ((uint64_t{1} << idbits) - 1));
    if (gid < n_u)
      grank_u[sr_u[gid]] = static_cast<int32_t>(r);
    else
      grank_v[sr_v[gid - n_u]] = static_cast<int32_t>(r);
  }
}

// Kept record r as a CSR entry of side a: key (sr_a[a[r]], sr_b[b[r]]).
__global__ void k_csr_keys(const uint32_t* kept, int64_t me, const int32_t* a, const int32_t* b, const int32_t* sr_a,
                           const int32_t* sr_b, int bbits, uint64_t* keys, uint32_t* vals) {
  GRID_STRIDE(k, me) {
    const uint32_t r = kept[k];
    keys[k] = (static_cast<uint64_t>(sr_a[a[r]]) << bbits) | static_cast<uint32_t>(sr_b[b[r]]);
    vals[k] = r;
  }
}

__global__ void k_deg_by_rank(const int32_t* ord, const uint32_t* deg, int32_t n, uint32_t* out) {
  GRID_STRIDE(r, n) out[r] = deg[ord[r]];
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

// Packed CSR entries (neighbour side rank << 1 | negative) of side a's rows.
__global__ void k_fill_adj(const uint32_t* by, int64_t me, const int32_t* b, const int8_t* sign, const int32_t* sr_b,
                           uint32_t* adj) {
  GRID_STRIDE(k, me) {
    const uint32_t r = by[k];
    adj[k] = (static_cast<uint32_t>(sr_b[b[r]]) << 1) | (sign[r] < 0 ? 1u : 0u);
  }
}

__global__ void k_record_pos(const uint32_t* by, int64_t me, uint32_t* pos) {
  GRID_STRIDE(k, me) pos[by[k]] = static_cast<uint32_t>(k);
}

// rev of both sides: for U entry k of edge (x, y), the index of x inside row
// y of V, and the converse.
__global__ void k_rev(const uint32_t* by_u, int64_t me, const int32_t* u, const int32_t* v, const int32_t* sr_u,
                      const int32_t* sr_v, const uint32_t* off_u, const uint32_t* off_v, const uint32_t* pos_v,
                      int32_t* rev_u, int32_t* rev_v) {
  GRID_STRIDE(k, me) {
    const uint32_t r = by_u[k];
    const uint32_t pv = pos_v[r];
    rev_u[k] = static_cast<int32_t>(pv - off_v[sr_v[v[r]]]);
    rev_v[pv] = static_cast<int32_t>(static_cast<uint32_t>(k) - off_u[sr_u[u[r]]]);
  }
}

// cut[x]: neighbours of higher priority than x (a prefix of row x).
__global__ void k_cut(const uint32_t* off, const uint32_t* adj, int32_t n, const int32_t* grank_self,
                      const int32_t* grank_other, int32_t* cut) {
  GRID_STRIDE(x, n) {
    uint32_t lo = off[x], hi = off[x + 1];
    const uint32_t b = lo;
    const int32_t gx = grank_self[x];
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo) / 2;
      if (grank_other[adj[mid] >> 1] < gx)
        lo = mid + 1;
      else
        hi = mid;
    }
    cut[x] = static_cast<int32_t>(lo - b);
  }
}

// W_VP: a down-edge (x, y) walks the entries of row y after x; one
// wavefront per row, sums kept per wavefront until the end.
__global__ void k_wedges(const uint32_t* off, const uint32_t* adj, const int32_t* rev, const int32_t* cut,
                         const uint32_t* off_other, int32_t n, unsigned long long* res) {
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  unsigned long long w_all = 0, active = 0;
  for (int64_t x = wave; x < n; x += waves) {
    unsigned long long wx = 0;
    for (uint32_t e = off[x] + static_cast<uint32_t>(cut[x]) + lane; e < off[x + 1]; e += 64) {
      const uint32_t y = adj[e] >> 1;
      wx += off_other[y + 1] - off_other[y] - 1u - static_cast<uint32_t>(rev[e]);
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) wx += __shfl_xor(wx, d, 64);
    w_all += wx;
    active += wx > 0 ? 1 : 0;
  }
  if (lane == 0 && (w_all | active)) {
    atomicAdd(&res[0], w_all);
    atomicAdd(&res[1], active);
  }
}

// Entries of the top T x T block of side 0 for T = 4096, 2048, 1024 (the
// dense block's fill, which picks its default size): per row x < 4096, the
// entries of rank below each T, by binary search.
__global__ void k_hub_nnz(const uint32_t* off, const uint32_t* adj, int32_t n, unsigned long long* res) {
  const int32_t rows = min(n, 4096);
  for (int32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < rows; x += gridDim.x * blockDim.x) {
    const uint32_t b = off[x], e = off[x + 1];
    for (int k = 0; k < 3; ++k) {
      const int32_t T = 4096 >> k;
      if (x >= T) continue;
      const uint32_t key = static_cast<uint32_t>(T) << 1;
      uint32_t lo = b, hi = e;
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (adj[mid] < key)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo > b) atomicAdd(&res[k], static_cast<unsigned long long>(lo - b));
    }
  }
}

// Device memory of one build step, freed on scope exit (at least 16 bytes,
// so that even an empty array has an address).
struct Tmp : DevBuf {
  hipError_t alloc(size_t bytes) { return DevBuf::alloc(std::max<size_t>(bytes, 16)); }
};

struct Fail {
  int status;
  std::string msg;
};

#define DEV_TRY(expr)                                                                                   \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess)                                                                               \
      throw Fail{e_ == hipErrorOutOfMemory ? DBBC_E_OOM : DBBC_E_DEVICE,                                \
                 std::string(#expr) + ": " + hipGetErrorString(e_)};                                    \
  } while (0)

// hipCUB calls take their temporary storage from one growing buffer.
struct CubTmp {
  Tmp buf;
  size_t bytes = 0;
  void* get(size_t need) {
    if (need > bytes) {
      DEV_TRY(buf.alloc(need));
      bytes = need;
    }
    return buf.p;
  }
};

template <class T>
void to_host(std::vector<T>& out, const void* src, size_t n, hipStream_t st) {
  out.resize(n);
  if (n) DEV_TRY(hipMemcpyAsync(out.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, st));
}

void sort_keys(CubTmp& ct, uint64_t* in, uint64_t* out, int64_t n, int end_bit, hipStream_t st) {
  size_t need = 0;
  DEV_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, need, in, out, static_cast<int>(n), 0, end_bit, st));
  void* t = ct.get(need);
  DEV_TRY(hipcub::DeviceRadixSort::SortKeys(t, need, in, out, static_cast<int>(n), 0, end_bit, st));
}

void sort_pairs(CubTmp& ct, uint64_t* kin, uint64_t* kout, uint32_t* vin, uint32_t* vout, int64_t n, int end_bit,
                hipStream_t st) {
  size_t need = 0;
  DEV_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, need, kin, kout, vin, vout, static_cast<int>(n), 0, end_bit,
                                             st));
  void* t = ct.get(need);
  DEV_TRY(hipcub::DeviceRadixSort::SortPairs(t, need, kin, kout, vin, vout, static_cast<int>(n), 0, end_bit, st));
}

uint32_t max_of(CubTmp& ct, const uint32_t* in, int64_t n, uint32_t* d_out, hipStream_t st) {
  size_t need = 0;
  DEV_TRY(hipcub::DeviceReduce::Max(nullptr, need, in, d_out, static_cast<int>(n), st));
  void* t = ct.get(need);
  DEV_TRY(hipcub::DeviceReduce::Max(t, need, in, d_out, static_cast<int>(n), st));
  uint32_t h = 0;
  DEV_TRY(hipMemcpyAsync(&h, d_out, sizeof(h), hipMemcpyDeviceToHost, st));
  DEV_TRY(hipStreamSynchronize(st));
  return h;
}

void build(int32_t n_u, int32_t n_v, int64_t m, const int32_t* u_in, const int32_t* v_in, const int8_t* s_in,
           uint32_t flags, hipStream_t st, HostGraph& g, DeviceCsr& out) {
  const size_t M = static_cast<size_t>(m);
  CubTmp ct;
  // inputs on the device
  Tmp du, dv, ds;
  const int32_t* u = u_in;
  const int32_t* v = v_in;
  const int8_t* s = s_in;
  if (!(flags & DBBC_INPUT_DEVICE)) {
    DEV_TRY(du.alloc(M * 4));
    DEV_TRY(dv.alloc(M * 4));
    DEV_TRY(ds.alloc(M));
    if (m) {
      DEV_TRY(hipMemcpyAsync(du.p, u_in, M * 4, hipMemcpyHostToDevice, st));
      DEV_TRY(hipMemcpyAsync(dv.p, v_in, M * 4, hipMemcpyHostToDevice, st));
      DEV_TRY(hipMemcpyAsync(ds.p, s_in, M, hipMemcpyHostToDevice, st));
    }
    u = du.as<int32_t>();
    v = dv.as<int32_t>();
    s = ds.as<int8_t>();
  }
  Tmp small;  // 7 u64 words: bad[2], wedge sums[2], hub block entries[3]
  DEV_TRY(small.alloc(7 * sizeof(unsigned long long)));
  unsigned long long* words = small.as<unsigned long long>();
  DEV_TRY(launch_fill_u64(words, 2, ~0ull, st));
  DEV_TRY(launch_fill_u64(words + 2, 5, 0ull, st));
  if (m) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(m)), dim3(kThreads), 0, st, u, v, s, m, n_u, n_v, words);
    DEV_TRY(hipGetLastError());
  }
  unsigned long long bad[2];
  DEV_TRY(hipMemcpyAsync(bad, words, sizeof(bad), hipMemcpyDeviceToHost, st));
  DEV_TRY(hipStreamSynchronize(st));
  if (bad[0] != ~0ull || bad[1] != ~0ull) {
    // the first bad record, ids checked before the sign
    if (bad[0] <= bad[1])
      throw Fail{DBBC_E_ID_RANGE, "edge " + std::to_string(bad[0]) + " has a vertex id out of range"};
    int8_t sv = 0;
    DEV_TRY(hipMemcpyAsync(&sv, s + bad[1], 1, hipMemcpyDeviceToHost, st));
    DEV_TRY(hipStreamSynchronize(st));
    throw Fail{DBBC_E_SIGN, "edge " + std::to_string(bad[1]) + " has sign " + std::to_string(int(sv)) +
                                " (must be +1 or -1)"};
  }

  const int ubits = bits_for(n_u), vbits = bits_for(n_v);
  Tmp k0, k1, v0, v1;
  const size_t nmax = std::max<size_t>(M, static_cast<size_t>(n_u) + n_v);
  DEV_TRY(k0.alloc(nmax * 8));
  DEV_TRY(k1.alloc(nmax * 8));
  DEV_TRY(v0.alloc(M * 4));
  DEV_TRY(v1.alloc(M * 4));
  // 1. last-wins dedup
  Tmp kept, keep, nsel;
  DEV_TRY(kept.alloc(M * 4));
  DEV_TRY(keep.alloc(M));
  DEV_TRY(nsel.alloc(sizeof(int)));
  int64_t me = 0;
  if (m) {
    hipLaunchKernelGGL(k_pair_keys, dim3(grid_for(m)), dim3(kThreads), 0, st, u, v, m, vbits, k0.as<uint64_t>(),
                       v0.as<uint32_t>());
    DEV_TRY(hipGetLastError());
    sort_pairs(ct, k0.as<uint64_t>(), k1.as<uint64_t>(), v0.as<uint32_t>(), v1.as<uint32_t>(), m, ubits + vbits, st);
    hipLaunchKernelGGL(k_last_of_run, dim3(grid_for(m)), dim3(kThreads), 0, st, k1.as<uint64_t>(), m,
                       keep.as<uint8_t>());
    DEV_TRY(hipGetLastError());
    size_t need = 0;
    DEV_TRY(hipcub::DeviceSelect::Flagged(nullptr, need, v1.as<uint32_t>(), keep.as<uint8_t>(), kept.as<uint32_t>(),
                                          nsel.as<int>(), static_cast<int>(m), st));
    void* t = ct.get(need);
    DEV_TRY(hipcub::DeviceSelect::Flagged(t, need, v1.as<uint32_t>(), keep.as<uint8_t>(), kept.as<uint32_t>(),
                                          nsel.as<int>(), static_cast<int>(m), st));
    int hsel = 0;
    DEV_TRY(hipMemcpyAsync(&hsel, nsel.p, sizeof(int), hipMemcpyDeviceToHost, st));
    DEV_TRY(hipStreamSynchronize(st));
    me = hsel;
  }
  const int64_t dups = m - me;
  if (dups && (flags & DBBC_DUP_REJECT)) throw Fail{DBBC_E_DUPLICATE, std::to_string(dups) + " duplicate (u, v) records"};
  g.n_u = n_u;
  g.n_v = n_v;
  g.m = me;
  g.m_in = m;
  g.dups_dropped = dups;

  // 2. degrees and priority orders
  const int32_t n[2] = {n_u, n_v};
  Tmp deg[2], sr[2];
  DevBuf* ord = out.ord;
  DevBuf* grank = out.grank;
  for (int x = 0; x < 2; ++x) {
    DEV_TRY(deg[x].alloc(static_cast<size_t>(n[x]) * 4));
    DEV_TRY(ord[x].alloc(static_cast<size_t>(n[x]) * 4));
    DEV_TRY(sr[x].alloc(static_cast<size_t>(n[x]) * 4));
    DEV_TRY(grank[x].alloc(static_cast<size_t>(n[x]) * 4));
    DEV_TRY(hipMemsetAsync(deg[x].p, 0, static_cast<size_t>(n[x]) * 4, st));
  }
  if (me) {
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(m)), dim3(kThreads), 0, st, k1.as<uint64_t>(), keep.as<uint8_t>(), m,
                       vbits, deg[0].as<uint32_t>(), deg[1].as<uint32_t>());
    DEV_TRY(hipGetLastError());
  }
  Tmp dmax;
  DEV_TRY(dmax.alloc(sizeof(uint32_t)));
  uint32_t maxdeg[2];
  for (int x = 0; x < 2; ++x) {
    maxdeg[x] = max_of(ct, deg[x].as<uint32_t>(), n[x], dmax.as<uint32_t>(), st);
    const int idb = bits_for(n[x]);
    hipLaunchKernelGGL(k_prio_keys, dim3(grid_for(n[x])), dim3(kThreads), 0, st, deg[x].as<uint32_t>(), n[x],
                       maxdeg[x], idb, k0.as<uint64_t>());
    DEV_TRY(hipGetLastError());
    sort_keys(ct, k0.as<uint64_t>(), k1.as<uint64_t>(), n[x], idb + bits_for(int64_t{maxdeg[x]} + 1), st);
    hipLaunchKernelGGL(k_prio_ranks, dim3(grid_for(n[x])), dim3(kThreads), 0, st, k1.as<uint64_t>(), n[x], idb,
                       ord[x].as<int32_t>(), sr[x].as<int32_t>());
    DEV_TRY(hipGetLastError());
  }
  {
    const uint32_t md = std::max(maxdeg[0], maxdeg[1]);
    const int64_t nn = static_cast<int64_t>(n_u) + n_v;
    const int idb = bits_for(nn);
    hipLaunchKernelGGL(k_global_keys, dim3(grid_for(nn)), dim3(kThreads), 0, st, deg[0].as<uint32_t>(),
                       deg[1].as<uint32_t>(), n_u, n_v, md, idb, k0.as<uint64_t>());
    DEV_TRY(hipGetLastError());
    sort_keys(ct, k0.as<uint64_t>(), k1.as<uint64_t>(), nn, idb + bits_for(int64_t{md} + 1), st);
    hipLaunchKernelGGL(k_global_ranks, dim3(grid_for(nn)), dim3(kThreads), 0, st, k1.as<uint64_t>(), n_u, n_v, idb,
                       sr[0].as<int32_t>(), sr[1].as<int32_t>(), grank[0].as<int32_t>(), grank[1].as<int32_t>());
    DEV_TRY(hipGetLastError());
  }

  // 3. the two CSRs: rows by own side rank, neighbours by the other's
  const int32_t* ends[2] = {u, v};
  const int bitsv[2] = {ubits, vbits};
  Tmp by1, off[2], adj[2], dbr;
  DevBuf* by[2] = {&out.rec, &by1};
  DevBuf* rev = out.rev;
  DevBuf* cut = out.cut;
  DEV_TRY(dbr.alloc((static_cast<size_t>(std::max(n_u, n_v)) + 1) * 4));
  for (int x = 0; x < 2; ++x) {
    const int o = 1 - x;
    DEV_TRY(by[x]->alloc(static_cast<size_t>(me) * 4));
    DEV_TRY(off[x].alloc((static_cast<size_t>(n[x]) + 1) * 4));
    DEV_TRY(adj[x].alloc((static_cast<size_t>(me) + kAdjPad) * 4));
    DEV_TRY(rev[x].alloc(static_cast<size_t>(me) * 4));
    DEV_TRY(cut[x].alloc(static_cast<size_t>(n[x]) * 4));
    DEV_TRY(hipMemsetAsync(adj[x].as<uint32_t>() + me, 0, kAdjPad * 4, st));
    if (me) {
      hipLaunchKernelGGL(k_csr_keys, dim3(grid_for(me)), dim3(kThreads), 0, st, kept.as<uint32_t>(), me, ends[x],
                         ends[o], sr[x].as<int32_t>(), sr[o].as<int32_t>(), bitsv[o], k0.as<uint64_t>(),
                         v0.as<uint32_t>());
      DEV_TRY(hipGetLastError());
      sort_pairs(ct, k0.as<uint64_t>(), k1.as<uint64_t>(), v0.as<uint32_t>(), by[x]->as<uint32_t>(), me,
                 bitsv[x] + bitsv[o], st);
      hipLaunchKernelGGL(k_fill_adj, dim3(grid_for(me)), dim3(kThreads), 0, st, by[x]->as<uint32_t>(), me, ends[o], s,
                         sr[o].as<int32_t>(), adj[x].as<uint32_t>());
      DEV_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_deg_by_rank, dim3(grid_for(n[x])), dim3(kThreads), 0, st, ord[x].as<int32_t>(),
                       deg[x].as<uint32_t>(), n[x], dbr.as<uint32_t>());
    DEV_TRY(hipGetLastError());
    size_t need = 0;
    DEV_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, need, dbr.as<uint32_t>(), off[x].as<uint32_t>(), n[x], st));
    void* t = ct.get(need);
    DEV_TRY(hipcub::DeviceScan::ExclusiveSum(t, need, dbr.as<uint32_t>(), off[x].as<uint32_t>(), n[x], st));
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, st, off[x].as<uint32_t>() + n[x], static_cast<uint32_t>(me));
    DEV_TRY(hipGetLastError());
  }
  if (me) {
    Tmp pos_v;
    DEV_TRY(pos_v.alloc(M * 4));
    hipLaunchKernelGGL(k_record_pos, dim3(grid_for(me)), dim3(kThreads), 0, st, by[1]->as<uint32_t>(), me,
                       pos_v.as<uint32_t>());
    DEV_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_rev, dim3(grid_for(me)), dim3(kThreads), 0, st, by[0]->as<uint32_t>(), me, u, v,
                       sr[0].as<int32_t>(), sr[1].as<int32_t>(), off[0].as<uint32_t>(), off[1].as<uint32_t>(),
                       pos_v.as<uint32_t>(), rev[0].as<int32_t>(), rev[1].as<int32_t>());
    DEV_TRY(hipGetLastError());
    DEV_TRY(hipStreamSynchronize(st));  // pos_v leaves scope
  }
  for (int x = 0; x < 2; ++x) {
    hipLaunchKernelGGL(k_cut, dim3(grid_for(n[x])), dim3(kThreads), 0, st, off[x].as<uint32_t>(),
                       adj[x].as<uint32_t>(), n[x], grank[x].as<int32_t>(), grank[1 - x].as<int32_t>(),
                       cut[x].as<int32_t>());
    DEV_TRY(hipGetLastError());
  }
  for (int x = 0; x < 2; ++x) {
    const int64_t waves = std::min<int64_t>(n[x], 1 << 16);
    hipLaunchKernelGGL(k_wedges, dim3(static_cast<int>((waves * 64 + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       st, off[x].as<uint32_t>(), adj[x].as<uint32_t>(), rev[x].as<int32_t>(), cut[x].as<int32_t>(),
                       off[1 - x].as<uint32_t>(), n[x], words + 2);
    DEV_TRY(hipGetLastError());
  }

  hipLaunchKernelGGL(k_hub_nnz, dim3(16), dim3(kThreads), 0, st, off[0].as<uint32_t>(), adj[0].as<uint32_t>(), n[0],
                     words + 4);
  DEV_TRY(hipGetLastError());

  // 4. the sizes the host keeps (the arrays stay on the device)
  for (int x = 0; x < 2; ++x) {
    HostSide& S = g.side[x];
    S = HostSide{};
    S.n = n[x];
    S.max_deg = maxdeg[x];
  }
  g.arrays = false;
  unsigned long long wsum[5];
  DEV_TRY(hipMemcpyAsync(wsum, words + 2, sizeof(wsum), hipMemcpyDeviceToHost, st));
  DEV_TRY(hipStreamSynchronize(st));
  g.wedges_vp = static_cast<int64_t>(wsum[0]);
  g.pivots_active = static_cast<int64_t>(wsum[1]);
  for (int k = 0; k < 3; ++k) g.hub_nnz[k] = static_cast<int64_t>(wsum[2 + k]);
  for (int x = 0; x < 2; ++x) {
    out.adj[x] = std::move(adj[x]);
    out.off[x] = std::move(off[x]);
  }
}

}  // namespace

int fetch_host_arrays(const DevGraphView& d, HostGraph& g, hipStream_t st, std::string& err) {
  if (g.arrays) return DBBC_OK;
  try {
    const size_t me = static_cast<size_t>(g.m);
    for (int x = 0; x < 2; ++x) {
      HostSide& S = g.side[x];
      const size_t n = static_cast<size_t>(S.n);
      to_host(S.off, d.off[x], n + 1, st);
      to_host(S.adj, d.adj[x], me, st);
      to_host(S.rev, d.rev[x], me, st);
      to_host(S.cut, d.cut[x], n, st);
      to_host(S.grank, d.grank[x], n, st);
      to_host(S.orig, d.ord[x], n, st);
    }
    to_host(g.side[0].rec, d.rec, me, st);
    g.side[1].rec.clear();
    DEV_TRY(hipStreamSynchronize(st));
  } catch (const Fail& f) {
    err = f.msg;
    (void)hipStreamSynchronize(st);
    return f.status;
  } catch (const std::bad_alloc&) {
    err = "host allocation failed while copying the graph";
    (void)hipStreamSynchronize(st);
    return DBBC_E_OOM;
  }
  g.arrays = true;
  return DBBC_OK;
}

int build_device_graph(int32_t n_u, int32_t n_v, int64_t m, const int32_t* u, const int32_t* v,
                       const int8_t* sign, uint32_t flags, hipStream_t st, HostGraph& g, DeviceCsr& out,
                       std::string& err) {
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
  try {
    build(n_u, n_v, m, u, v, sign, flags, st, g, out);
  } catch (const Fail& f) {
    err = f.msg;
    (void)hipStreamSynchronize(st);
    return f.status;
  } catch (const std::bad_alloc&) {
    err = "host allocation failed while building the graph";
    (void)hipStreamSynchronize(st);
    return DBBC_E_OOM;
  }
  return DBBC_OK;
}

}  // namespace dbbc
