// Explicit-verification counting, the baseline of the paper's study of the
// symmetric / asymmetric wedge separation (Section V, Table IV): without
// the two buckets of Lemma 1, the wedges of each vertex pair are gathered
// and every pair of them -- a candidate 4-cycle -- is checked on its signs
// one by one.  Same enumeration order (Algorithm 1, Phase 5, vertex
// priority) and same results as the bucketed count; the work is one check
// per butterfly instead of one update per wedge.  It exists to measure what
// the separation saves on the same device.
//
// One workgroup per pivot x (a queue), with per-workgroup scratch in HBM:
//   A. walk x's wedges x - y - w (w ranked below x, y below x): count each
//      endpoint's wedges and list the endpoints touched;
//   B. prefix sums over the touched endpoints place each one's wedges;
//   C. walk again, writing each wedge's symmetry bit (s(x,y) s(y,w) = -1)
//      into its endpoint's segment;
//   D. for every endpoint, every pair of its wedges: equal bits make a
//      balanced butterfly, different bits an unbalanced one.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "build_dev.h"
#include "kernels.h"

namespace dbbc {
namespace dev {

constexpr int kExThreads = 256;
constexpr int kExWaves = kExThreads / 64;

__global__ __launch_bounds__(kExThreads) void k_explicit(ExplicitArgs a) {
  __shared__ uint32_t nt_sh, total_sh, scan_sh[kExThreads];
  __shared__ int32_t pivot_sh;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const size_t n = static_cast<size_t>(a.n_s);
  uint32_t* cnt = a.scratch + static_cast<size_t>(blockIdx.x) * 4 * n;
  uint32_t* fill = cnt + n;
  uint32_t* touched = fill + n;
  uint32_t* base = touched + n;
  uint8_t* list = a.lists + static_cast<size_t>(blockIdx.x) * static_cast<size_t>(a.list_cap);
  unsigned long long bal = 0, unb = 0;
  if (tid == 0) nt_sh = 0;
  for (;;) {
    if (tid == 0) pivot_sh = static_cast<int32_t>(atomicAdd(a.queue, 1u));
    __syncthreads();
    const int32_t x = pivot_sh;
    if (x >= a.n_s) break;
    const uint32_t e0 = a.off_s[x] + static_cast<uint32_t>(a.cut_s[x]), e1 = a.off_s[x + 1];
    // A: tally (a wavefront per down-edge, its lanes over the edge's run)
    for (uint32_t e = e0 + wave; e < e1; e += kExWaves) {
      const uint32_t y = a.adj_s[e] >> 1;
      const uint32_t j1 = a.off_o[y + 1];
      for (uint32_t j = a.off_o[y] + static_cast<uint32_t>(a.rev_s[e]) + 1 + lane; j < j1; j += 64) {
        const uint32_t w = a.adj_o[j] >> 1;
        if (atomicAdd(&cnt[w], 1u) == 0u) touched[atomicAdd(&nt_sh, 1u)] = w;
      }
    }
    __syncthreads();
    // B: segment starts of the touched endpoints (block scan in chunks)
    const uint32_t nt = nt_sh;
    uint32_t running = 0;
    for (uint32_t c0 = 0; c0 < nt; c0 += kExThreads) {
      const uint32_t i = c0 + tid;
      const uint32_t v = i < nt ? cnt[touched[i]] : 0u;
      scan_sh[tid] = v;
      __syncthreads();
      for (int d = 1; d < kExThreads; d <<= 1) {
        const uint32_t add = tid >= d ? scan_sh[tid - d] : 0u;
        __syncthreads();
        scan_sh[tid] += add;
        __syncthreads();
      }
      if (i < nt) {
        const uint32_t b = running + scan_sh[tid] - v;
        base[i] = b;
        fill[touched[i]] = b;
      }
      if (tid == kExThreads - 1) total_sh = scan_sh[tid];
      __syncthreads();
      running += total_sh;
      __syncthreads();
    }
    if (running > a.list_cap && tid == 0) atomicOr(a.err, 1ull);  // cannot happen: cap = max wedges of a pivot
    __syncthreads();
    // C: the symmetry bit of every wedge into its endpoint's segment
    if (running <= a.list_cap) {
      for (uint32_t e = e0 + wave; e < e1; e += kExWaves) {
        const uint32_t ye = a.adj_s[e];
        const uint32_t y = ye >> 1;
        const uint32_t j1 = a.off_o[y + 1];
        for (uint32_t j = a.off_o[y] + static_cast<uint32_t>(a.rev_s[e]) + 1 + lane; j < j1; j += 64) {
          const uint32_t we = a.adj_o[j];
          list[atomicAdd(&fill[we >> 1], 1u)] = static_cast<uint8_t>((we ^ ye) & 1u);
        }
      }
    }
    __syncthreads();
    // D: every pair of wedges of every endpoint, checked on its signs
    for (uint32_t i = wave; i < nt; i += kExWaves) {
      const uint32_t w = touched[i];
      const uint32_t c = cnt[w], b = base[i];
      if (running <= a.list_cap) {
        for (uint32_t p = lane; p < c; p += 64) {
          const uint8_t tp = list[b + p];
          for (uint32_t q = p + 1; q < c; ++q) {
            if (list[b + q] == tp)
              ++bal;
            else
              ++unb;
          }
        }
      }
      if (lane == 0) cnt[w] = fill[w] = 0u;
    }
    __syncthreads();
    if (tid == 0) nt_sh = 0;
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    bal += __shfl_xor(bal, d, 64);
    unb += __shfl_xor(unb, d, 64);
  }
  if (lane == 0) {
    if (bal) atomicAdd(a.res + kResBalanced, bal);
    if (unb) atomicAdd(a.res + kResUnbalanced, unb);
    if (bal + unb) atomicAdd(a.res + kResTotal, bal + unb);
  }
}

}  // namespace dev

hipError_t launch_explicit(const ExplicitArgs& a, int grid, hipStream_t st) {
  if (a.n_s == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_explicit, dim3(grid), dim3(dev::kExThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace dbbc
