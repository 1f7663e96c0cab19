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
// leave the remaining wedges of each hub pair in hub_pairs; the epilogue adds
// them before taking Lemma 1's C(P,2) + C(N,2), P * N and C(P + N, 2), since
// the binomials are not additive.  Entries are at most K < 2^31: exact.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace dbbc {
namespace dev {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kHubTile = 128;     // output tile (rows x and columns w)
constexpr int kHubThreads = 256;  // 2 x 2 wavefronts, each 64 x 64 of the tile
constexpr int kHubKStep = kHubKPad;  // k bytes of both operands staged per step
constexpr int kHubRow = kHubKStep + 16;  // LDS bytes per staged row (+16 spreads banks)
constexpr int kHubLoads = kHubTile * kHubKStep / 16 / kHubThreads;  // 16-byte loads per thread and operand

// One 128 x 128 tile of the upper triangle per workgroup.  Each step stages
// 128 rows x 128 k of Bm (rows x) and of B (rows w) in LDS with coalesced
// 16-byte loads (8 lanes per row), double-buffered: the next step's loads
// are in flight while the current step's 32 MFMAs per wavefront run (a step
// of 128 k gives each load round trip twice the matrix work of 64 k).
__global__ __launch_bounds__(kHubThreads, 2) void k_hub(HubArgs a) {
  __shared__ __attribute__((aligned(16))) int8_t sA[2][kHubTile * kHubRow];
  __shared__ __attribute__((aligned(16))) int8_t sB[2][kHubTile * kHubRow];
  // upper-triangular tile (ti <= tj) from the linear block index
  const int nt = a.T / kHubTile;
  int t = blockIdx.x, ti = 0;
  while (t >= nt - ti) {
    t -= nt - ti;
    ++ti;
  }
  const int tj = ti + t;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int row0 = ti * kHubTile + (wave >> 1) * 64;
  const int col0 = tj * kHubTile + (wave & 1) * 64;
  const int r = lane & 31;
  const int kh = (lane >> 5) * 16;
  v16i X[2][2], Y[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      X[i][j] = v16i{};
      Y[i][j] = v16i{};
    }
  // staging: chunk c = tid + 256 i is row c / 8, bytes 16 (c % 8)
  const size_t K = static_cast<size_t>(a.K);
  const int8_t* gA = a.Bm + static_cast<size_t>(ti * kHubTile) * K;
  const int8_t* gB = a.B + static_cast<size_t>(tj * kHubTile) * K;
  int srow[kHubLoads], spart[kHubLoads];
#pragma unroll
  for (int i = 0; i < kHubLoads; ++i) {
    const int c = tid + kHubThreads * i;
    srow[i] = c / (kHubKStep / 16);
    spart[i] = (c % (kHubKStep / 16)) * 16;
  }
  v4i ra[kHubLoads], rb[kHubLoads];
  auto gload = [&](int k) {
#pragma unroll
    for (int i = 0; i < kHubLoads; ++i) {
      ra[i] = *reinterpret_cast<const v4i*>(gA + srow[i] * K + k + spart[i]);
      rb[i] = *reinterpret_cast<const v4i*>(gB + srow[i] * K + k + spart[i]);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < kHubLoads; ++i) {
      *reinterpret_cast<v4i*>(&sA[buf][srow[i] * kHubRow + spart[i]]) = ra[i];
      *reinterpret_cast<v4i*>(&sB[buf][srow[i] * kHubRow + spart[i]]) = rb[i];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  const v4i ones = {0x01010101, 0x01010101, 0x01010101, 0x01010101};
  const int ar = (wave >> 1) * 64 + r, br = (wave & 1) * 64 + r;
  for (int k0 = 0, buf = 0; k0 < a.K; k0 += kHubKStep, buf ^= 1) {
    const bool more = k0 + kHubKStep < a.K;
    if (more) gload(k0 + kHubKStep);
#pragma unroll
    for (int kk = 0; kk < kHubKStep; kk += 32) {
      // a lane feeds 16 consecutive k of its row to both operands, so the
      // two operands agree on which k each byte slot holds
      const v4i A0 = *reinterpret_cast<const v4i*>(&sA[buf][ar * kHubRow + kk + kh]);
      const v4i A1 = *reinterpret_cast<const v4i*>(&sA[buf][(ar + 32) * kHubRow + kk + kh]);
      const v4i B0 = *reinterpret_cast<const v4i*>(&sB[buf][br * kHubRow + kk + kh]);
      const v4i B1 = *reinterpret_cast<const v4i*>(&sB[buf][(br + 32) * kHubRow + kk + kh]);
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
    if (more) sstore(buf ^ 1);
    __syncthreads();
  }
  // Epilogue.  32 x 32 accumulator layout: lane l, register q holds row
  // 8 * (q / 4) + 4 * (l / 32) + q % 4 and column l % 32 of the block.
  int64_t bal = 0, unb = 0, tot = 0, wd = 0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int x = row0 + i * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        const int w = col0 + j * 32 + (lane & 31);
        if (w <= x) continue;
        const int32_t xv = X[i][j][q], yv = Y[i][j][q];
        const unsigned long long sp = a.hub_pairs[static_cast<size_t>(x) * a.T + w];
        const int64_t P = (xv + yv) / 2 + static_cast<int64_t>(sp & 0xffffffffull);
        const int64_t N = (xv - yv) / 2 + static_cast<int64_t>(sp >> 32);
        bal += P * (P - 1) / 2 + N * (N - 1) / 2;
        unb += P * N;
        tot += (P + N) * (P + N - 1) / 2;
        wd += xv;
      }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    bal += __shfl_xor(bal, d, 64);
    unb += __shfl_xor(unb, d, 64);
    tot += __shfl_xor(tot, d, 64);
    wd += __shfl_xor(wd, d, 64);
  }
  if (lane == 0) {
    if (bal) atomicAdd(a.res + 0, static_cast<unsigned long long>(bal));
    if (unb) atomicAdd(a.res + 1, static_cast<unsigned long long>(unb));
    if (tot) atomicAdd(a.res + 2, static_cast<unsigned long long>(tot));
    if (wd) atomicAdd(a.res + 3, static_cast<unsigned long long>(wd));
  }
}

}  // namespace dev

hipError_t launch_hub(const HubArgs& a, hipStream_t st) {
  if (a.T <= 0) return hipSuccess;
  if (a.T % dev::kHubTile != 0 || a.K % dev::kHubKStep != 0) return hipErrorInvalidValue;
  const int nt = a.T / dev::kHubTile;
  const int tiles = nt * (nt + 1) / 2;
  hipLaunchKernelGGL(dev::k_hub, dim3(tiles), dim3(dev::kHubThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace dbbc
