// Dense hub block on the matrix cores (gfx950 int8 MFMA, int32 accumulate).
//
// For the T highest-priority vertices x, w of one side and the K highest-
// priority mids y of the other side, let B[x][y] be the edge sign (+1, -1) or
// 0, and Bm[x][y] = B[x][y] when y ranks below x, else 0 (the mid filter of
// Algorithm 1).  Then for w ranked below x
//   X[x][w] = sum_y |Bm[x][y]| |B[w][y]|   wedges x - y - w through hub mids
//   Y[x][w] = sum_y  Bm[x][y]   B[w][y]    (symmetric minus asymmetric)
// so the hub-mid wedges split as P = (X + Y) / 2 symmetric and
// N = (X - Y) / 2 asymmetric (Definitions 5 and 6).  The sparse kernels
// leave the remaining wedges of each hub pair as p + n and p - n in hub_xy;
// they are the accumulators' starting values, so the accumulators end as
// the pair's full X = P + N and Y = P - N before Lemma 1 is applied (the
// binomials are not additive).  In these terms
//   C(P,2) + C(N,2) = (X^2 + Y^2 - 2X) / 4,   P N = (X^2 - Y^2) / 4,
// both exact (X and Y have the same parity), and C(P + N, 2) is their sum.
// Entries are below 2^31: exact in int32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace dbbc {
namespace dev {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kHubTile = 128;     // output tile (rows x and columns w)
constexpr int kHubThreads = 256;  // 2 x 2 wavefronts, each 64 x 64 of the tile
constexpr int kHubKStep = kHubKPad;  // k bytes of both operands per pipeline stage
constexpr int kHubStages = 4;        // stages in flight (LDS ring)
constexpr int kHubStage = kHubTile * kHubKStep;  // bytes of one operand per stage

// LDS position of the 16-byte chunk c of a staged row: rows are 64 bytes,
// chunks permuted by ((row >> 1) ^ (row >> 3)) mod 4 so that the 16-byte
// operand reads of 8 (or 16) consecutive rows hit distinct banks.
__device__ __forceinline__ int hub_slot(int row, int c) { return row * kHubKStep + ((c ^ ((row >> 1) ^ (row >> 3))) & 3) * 16; }

// One 128 x 128 tile of the upper triangle per workgroup.  The operands
// stream through a ring of kHubStages LDS stages (128 rows x 64 k of Bm for
// rows x and of B for rows w per stage), filled by direct global-to-LDS
// loads (global_load_lds_dwordx4: no staging registers), kHubStages - 1
// stages ahead of the matrix work: each wavefront waits only for its own
// loads of the stage it is about to read, then the workgroup barrier makes
// every wavefront's part visible.
// Both sides of a graph share one launch: the first tiles0 workgroups work
// on s[0], the rest on s[1] (wavefront-uniform choice).
struct HubPair {
  HubArgs s[2];
  int32_t tiles0;
};

__global__ __launch_bounds__(kHubThreads, 2) void k_hub(HubPair hp) {
  __shared__ __attribute__((aligned(16))) int8_t sm[kHubStages][2][kHubStage];
  // workgroups are dealt to the 8 XCDs in turn: give each XCD a run of
  // consecutive tiles (rows of the upper triangle share their Bm panel)
  const int nb = static_cast<int>(gridDim.x), b = static_cast<int>(blockIdx.x);
  const int q8 = nb / 8;
  const int lin = b < 8 * q8 ? (b % 8) * q8 + b / 8 : b;
  const bool second = lin >= hp.tiles0;
  const HubArgs a = second ? hp.s[1] : hp.s[0];
  // upper-triangular tile (ti <= tj) from the linear block index
  const int nt = a.T / kHubTile;
  int t = lin - (second ? hp.tiles0 : 0), ti = 0;
  while (t >= nt - ti) {
    t -= nt - ti;
    ++ti;
  }
  const int tj = ti + t;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int row0 = ti * kHubTile + (wave >> 1) * 64;
  const int col0 = tj * kHubTile + (wave & 1) * 64;
  const int r = lane & 31;
  // accumulators start at the sparse partials.  32 x 32 accumulator layout:
  // lane l, register q holds row 8 (q / 4) + 4 (l / 32) + q % 4 and column
  // l % 32 of the block.
  const size_t TT = static_cast<size_t>(a.T) * a.T;
  v16i X[2][2], Y[2][2];
  int64_t x0 = 0;  // sparse wedges of the wave's pairs
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int32_t* px = a.hub_xy + static_cast<size_t>(row0 + i * 32 + 4 * (lane >> 5)) * a.T + col0 + j * 32 +
                          (lane & 31);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int off = (8 * (q >> 2) + (q & 3)) * a.T;  // wavefront-uniform
        X[i][j][q] = px[off];
        Y[i][j][q] = px[TT + off];
      }
    }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) x0 += X[i][j][q];
  // keep the sum here (sunk past the loop it would hold the starting
  // values live through the loop)
  asm volatile("" : "+v"(x0));
  const size_t K = static_cast<size_t>(a.K);
  // Loads of one stage: each wavefront fills 2 x 1 KB of each operand; lane
  // l of part q writes LDS chunk 64 q + l (row (64 q + l) / 4, slot l % 4)
  // and so fetches the global chunk that belongs in that slot.
  const int8_t* src[2][2];
  int dst[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int part = wave * 2 + q;
    const int S = part * 64 + lane;
    const int row = S >> 2, slot = S & 3;
    const int c = (slot ^ ((row >> 1) ^ (row >> 3))) & 3;
    src[0][q] = a.Bm + static_cast<size_t>(ti * kHubTile + row) * K + c * 16;
    src[1][q] = a.B + static_cast<size_t>(tj * kHubTile + row) * K + c * 16;
    dst[q] = part * 1024;
  }
  auto issue = [&](int stage, int k) {
#pragma unroll
    for (int op = 0; op < 2; ++op)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src[op][q] + k),
                                         (__attribute__((address_space(3))) void*)(&sm[stage][op][dst[q]]), 16, 0, 0);
  };
  const int nsteps = a.K / kHubKStep;
#pragma unroll
  for (int st = 0; st < kHubStages - 1; ++st)
    if (st < nsteps) issue(st, st * kHubKStep);
  const v4i ones = {0x01010101, 0x01010101, 0x01010101, 0x01010101};
  const int ar = (wave >> 1) * 64 + r, br = (wave & 1) * 64 + r;
  const int ch = lane >> 5;  // the lane's 16-byte chunk within 32 k
  for (int step = 0; step < nsteps; ++step) {
    // this wavefront's loads of stage `step` are complete once at most the
    // loads of the stages after it (issued before this point) are pending
    const int after = min(nsteps, step + kHubStages - 1) - step - 1;
    if (after >= 2)
      __builtin_amdgcn_s_waitcnt(0xF70 | 8);  // vmcnt(8): 4 loads per stage
    else if (after == 1)
      __builtin_amdgcn_s_waitcnt(0xF70 | 4);
    else
      __builtin_amdgcn_s_waitcnt(0xF70 | 0);
    // every wavefront's part of the stage is in LDS (each waited for its own
    // loads above), and every wavefront's reads of the stage read last step
    // have returned (its matrix work used them), so that stage may be
    // refilled.  A bare barrier: a __syncthreads fence would also wait for
    // the loads of the later stages; the empty asm statements keep the
    // compiler from moving memory accesses across it.
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    const int nxt = step + kHubStages - 1;
    if (nxt < nsteps) issue(nxt % kHubStages, nxt * kHubKStep);
    const int8_t* sA = sm[step % kHubStages][0];
    const int8_t* sB = sm[step % kHubStages][1];
#pragma unroll
    for (int kk = 0; kk < kHubKStep / 16; kk += 2) {
      // a lane feeds 16 consecutive k of its row to both operands, so the
      // two operands agree on which k each byte slot holds
      const int c = kk + ch;
      const v4i A0 = *reinterpret_cast<const v4i*>(&sA[hub_slot(ar, c)]);
      const v4i A1 = *reinterpret_cast<const v4i*>(&sA[hub_slot(ar + 32, c)]);
      const v4i B0 = *reinterpret_cast<const v4i*>(&sB[hub_slot(br, c)]);
      const v4i B1 = *reinterpret_cast<const v4i*>(&sB[hub_slot(br + 32, c)]);
      // |s| of an int8 in {-1, 0, 1} is its lowest bit
      const v4i A0a = A0 & ones, A1a = A1 & ones, B0a = B0 & ones, B1a = B1 & ones;
      X[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0a, B0a, X[0][0], 0, 0, 0);
      X[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0a, B1a, X[0][1], 0, 0, 0);
      X[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1a, B0a, X[1][0], 0, 0, 0);
      X[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1a, B1a, X[1][1], 0, 0, 0);
      Y[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, B0, Y[0][0], 0, 0, 0);
      Y[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, B1, Y[0][1], 0, 0, 0);
      Y[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, B0, Y[1][0], 0, 0, 0);
      Y[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, B1, Y[1][1], 0, 0, 0);
    }
  }
  // Epilogue: sums of X^2, Y^2 and X over the pairs with w below x.
  // (only diagonal tiles hold pairs with w not below x)
  int64_t sxx = 0, syy = 0, sx = 0;
  const bool diag = ti == tj;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int x = row0 + i * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        const int w = col0 + j * 32 + (lane & 31);
        const bool keep = !diag || w > x;
        const int32_t xv = keep ? X[i][j][q] : 0, yv = keep ? Y[i][j][q] : 0;
        sxx += static_cast<int64_t>(xv) * xv;
        syy += static_cast<int64_t>(yv) * yv;
        sx += xv;
      }
  if (a.bal) {
    // per-vertex pass: store the completed counts (zeros where w is not
    // below x) and credit each pair's C(P,2) + C(N,2) and P N to x (row
    // sums) and w (column sums)
    int32_t* hx = a.hub_xy;
    int64_t cb[2] = {0, 0}, cu[2] = {0, 0};  // column sums per j
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int x = row0 + i * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        int64_t rb = 0, ru = 0;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int w = col0 + j * 32 + (lane & 31);
          const bool keep = !diag || w > x;
          const int64_t xv = keep ? X[i][j][q] : 0, yv = keep ? Y[i][j][q] : 0;
          hx[static_cast<size_t>(x) * a.T + w] = static_cast<int32_t>(xv);
          hx[TT + static_cast<size_t>(x) * a.T + w] = static_cast<int32_t>(yv);
          const int64_t fb = (xv * xv + yv * yv - 2 * xv) / 4, fu = (xv * xv - yv * yv) / 4;
          rb += fb;
          ru += fu;
          cb[j] += fb;
          cu[j] += fu;
        }
#pragma unroll
        for (int d = 16; d > 0; d >>= 1) {
          rb += __shfl_xor(rb, d, 64);
          ru += __shfl_xor(ru, d, 64);
        }
        if ((lane & 31) == 0) {
          const int32_t id = a.orig[x];
          if (rb) atomicAdd(&a.bal[id], static_cast<unsigned long long>(rb));
          if (ru) atomicAdd(&a.unb[id], static_cast<unsigned long long>(ru));
        }
      }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      int64_t b = cb[j], u = cu[j];
      b += __shfl_xor(b, 32, 64);
      u += __shfl_xor(u, 32, 64);
      if (lane < 32) {
        const int32_t id = a.orig[col0 + j * 32 + lane];
        if (b) atomicAdd(&a.bal[id], static_cast<unsigned long long>(b));
        if (u) atomicAdd(&a.unb[id], static_cast<unsigned long long>(u));
      }
    }
  }
  int64_t bal = (sxx + syy - 2 * sx) / 4, unb = (sxx - syy) / 4;
  int64_t tot = bal + unb, wd = sx - x0;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    bal += __shfl_xor(bal, d, 64);
    unb += __shfl_xor(unb, d, 64);
    tot += __shfl_xor(tot, d, 64);
    wd += __shfl_xor(wd, d, 64);
  }
  // one set of atomics per workgroup: every workgroup adds to the same four
  // words, and atomics to one address are serialized (per wavefront they
  // took half the kernel's time)
  __shared__ int64_t wsum[kHubThreads / 64][4];
  if (lane == 0) {
    wsum[wave][0] = bal;
    wsum[wave][1] = unb;
    wsum[wave][2] = tot;
    wsum[wave][3] = wd;
  }
  __syncthreads();
  if (tid < 4) {
    int64_t v = 0;
#pragma unroll
    for (int w = 0; w < kHubThreads / 64; ++w) v += wsum[w][tid];
    if (v) atomicAdd(a.res + tid, static_cast<unsigned long long>(v));
  }
}

}  // namespace dev

hipError_t launch_hub(const HubArgs* sides, int n, hipStream_t st) {
  dev::HubPair hp{};
  int32_t tiles[2] = {0, 0};
  int k = 0;
  for (int i = 0; i < n; ++i) {
    const HubArgs& a = sides[i];
    if (a.T <= 0) continue;
    if (a.T % dev::kHubTile != 0 || a.K % dev::kHubKStep != 0) return hipErrorInvalidValue;
    const int nt = a.T / dev::kHubTile;
    hp.s[k] = a;
    tiles[k++] = nt * (nt + 1) / 2;
  }
  if (k == 0) return hipSuccess;
  hp.tiles0 = tiles[0];
  hipLaunchKernelGGL(dev::k_hub, dim3(tiles[0] + tiles[1]), dim3(dev::kHubThreads), 0, st, hp);
  return hipGetLastError();
}

}  // namespace dbbc
