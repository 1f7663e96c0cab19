// The dense hub block in the per-vertex and per-edge passes (gfx950).
//
// Every butterfly is counted at the pair (x, w) of its two same-side
// vertices of highest priority (Theorem 1).  For a hub pair (x, w < T, x of
// higher priority) with completed counts X = P + N and Y = P - N (the
// sparse wedges through non-hub mids, tallied here from the plan's hub
// runs, plus the block's wedges x - y - w through hub mids y, added by the
// matrix-core products of hub.hip), the block's wedges carry the credits of
// Lemma 1's pairing: a symmetric wedge lies in P - 1 balanced and N
// unbalanced butterflies of the pair, an asymmetric one in N - 1 and P.
// With s = Bm[x][y] B[w][y] the wedge's sign product, twice its balanced
// share is (X - 2) + s Y and twice its unbalanced share X - s Y.  Summed
// over the endpoints w of x through mid y,
//   2 bal(x, y) = |Bm[x][y]| (ZX - 2 Zc) + Bm[x][y] ZY,
//   2 unb(x, y) = |Bm[x][y]| ZX - Bm[x][y] ZY,
// with ZX = sum_w X[x][w] |B[w][y]| and ZY = sum_w Y[x][w] B[w][y] (w > x),
// Zc = #{w > x : B[w][y] != 0}: these are the credits of the pivot-mid edge
// (x, y), and their sums over x the mid y's.  Over the pivots x of w
// instead (x < w), with ZX' = sum_x X[x][w] |Bm[x][y]|, ZY' = sum_x
// Y[x][w] Bm[x][y] and Zc' = #{x < w : Bm[x][y] != 0}, the same algebra gives
// the end-mid edge (w, y):
//   2 bal(w, y) = |B[w][y]| (ZX' - 2 Zc') + B[w][y] ZY',
//   2 unb(w, y) = |B[w][y]| ZX' - B[w][y] ZY'.
// The products run on the int8 matrix cores: X and Y (up to a side's
// largest degree) are split into D signed 7-bit digits, v = sum_k d_k
// 2^(7 k), each digit's product accumulates exactly in int32 (at most
// T * 128 per entry), and each digit's share of the credits goes out
// scaled by 2^(7 k) (the shares of digit 0 are even: X and Y have the same
// parity).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"
#include "walk.h"

namespace dbbc {
namespace dev {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// Hub tally: one workgroup per hub item (a hub pivot x, or a part of a heavy
// one), 32-bit p and n per hub endpoint in LDS, the item's hub runs walked
// by its wavefronts, then its counts added into row x of the two planes
// (p + n, p - n) for the endpoints w in (x, T) (the planes start at zero).
constexpr int kHubTallyThreads = 256;
constexpr int kHubTallyWaves = kHubTallyThreads / kWave;

__global__ __launch_bounds__(kHubTallyThreads) void k_pv_hub_tally(HubTallyArgs a) {
  __shared__ uint32_t P[kMaxPVHubT], N[kMaxPVHubT];
  __shared__ __attribute__((aligned(16))) uint32_t mtab[kHubTallyWaves][kGather];
  __shared__ uint32_t mflag[kHubTallyWaves][kGather];
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  for (int i = tid; i < kMaxPVHubT; i += kHubTallyThreads) P[i] = N[i] = 0;
  for (int i = tid; i < kHubTallyWaves * static_cast<int>(kGather); i += kHubTallyThreads) (&mflag[0][0])[i] = 0;
  __syncthreads();
  const Marks<uint32_t> mk{mtab[wave], mflag[wave]};
  const uint32_t T = static_cast<uint32_t>(a.T);
  const size_t TT = static_cast<size_t>(T) * T;
  for (int32_t i = static_cast<int32_t>(blockIdx.x); i < a.n_items; i += static_cast<int32_t>(gridDim.x)) {
    const Item it = load_const(a.items, i);
    const uint32_t seg_end = it.seg_begin + it.seg_count;
    for (uint32_t k0 = it.seg_begin + wave * kWave; k0 < seg_end; k0 += kHubTallyThreads) {
      const uint32_t k1 = k0 + kWave < seg_end ? k0 + kWave : seg_end;
      walk_regs<4>(load_seg<false>(a.segs, k0, k1), a.other_adj, mk, a.long_len,
                   hash_tally([&](uint32_t e, uint32_t tag) {
                     const uint32_t key = e >> 1;  // a hub endpoint (x, T) by the plan
                     if (key < T) atomicAdd(((e ^ tag) & 1u) ? &N[key] : &P[key], 1u);
                   }));
    }
    __syncthreads();
    const uint32_t x = static_cast<uint32_t>(it.owner);
    int32_t* row = a.hub_xy + static_cast<size_t>(x) * T;
    for (uint32_t w = x + 1 + tid; w < T; w += kHubTallyThreads) {
      const uint32_t p = P[w], n = N[w];
      if (!(p | n)) continue;
      P[w] = 0;
      N[w] = 0;
      atomicAdd(&row[w], static_cast<int32_t>(p + n));
      atomicAdd(&row[TT + w], static_cast<int32_t>(p) - static_cast<int32_t>(n));
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Digits of the completed X and Y: one 64 x 64 tile per workgroup, written
// row-major (row x) and, through LDS, transposed (row w).
constexpr int kDigTile = 64;
constexpr int kMaxDigits = 5;  // 7-bit digits of values below 2^35

__global__ __launch_bounds__(256) void k_hub_digits(HubDigitArgs a) {
  __shared__ int8_t tile[2][kMaxDigits][kDigTile][kDigTile + 4];
  const int tr = static_cast<int>(blockIdx.y) * kDigTile, tc = static_cast<int>(blockIdx.x) * kDigTile;
  const size_t T = static_cast<size_t>(a.T), TT = T * T;
  const int D = a.D;
  for (int e = threadIdx.x; e < kDigTile * kDigTile; e += 256) {
    const int r = e / kDigTile, c = e % kDigTile;
#pragma unroll
    for (int xy = 0; xy < 2; ++xy) {
      const int32_t v = as_global(a.hub_xy)[xy * TT + (tr + r) * T + tc + c];
      for (int k = 0; k < D; ++k) {
        // low digits in [0, 128), the top digit signed
        const int32_t d = k == D - 1 ? (v >> (kHubDigitBits * k)) : ((v >> (kHubDigitBits * k)) & 127);
        const int8_t d8 = static_cast<int8_t>(d);
        as_global(a.rows)[(xy * D + k) * TT + (tr + r) * T + tc + c] = d8;
        tile[xy][k][r][c] = d8;
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kDigTile * kDigTile; e += 256) {
    const int r = e / kDigTile, c = e % kDigTile;  // r: w in the tile, c: x in the tile
#pragma unroll
    for (int xy = 0; xy < 2; ++xy)
      for (int k = 0; k < D; ++k) as_global(a.cols)[(xy * D + k) * TT + (tc + r) * T + tr + c] = tile[xy][k][c][r];
  }
}

// ---------------------------------------------------------------------------
// Credit products: one 128 x 128 tile (rows r, mids y) per workgroup, four
// wavefronts of 64 x 64, v_mfma_i32_32x32x32_i8.  Per digit, the digit
// planes of X and Y (rows r, contiguous in the contraction index t) and the
// transposed signs Bt (rows y, contiguous in t) stream through a ring of LDS
// stages filled by direct global-to-LDS loads; ZX accumulates with |Bt| and
// ZY with Bt.  The contraction skips the t that cannot hold a pair: t
// beyond the row tile (upper: t > r) or before it (t < r).
constexpr int kCrTile = 128;
constexpr int kCrThreads = 256;
constexpr int kCrKStep = 64;
constexpr int kCrStages = 3;
constexpr int kCrStage = kCrTile * kCrKStep;

__device__ __forceinline__ int cr_slot(int row, int c) {
  return row * kCrKStep + ((c ^ ((row >> 1) ^ (row >> 3))) & 3) * 16;
}

// Non-returning 64-bit add to global memory (two's complement: a negative
// digit share wraps and is made good by the other digits' shares).
__device__ __forceinline__ void add_u64(unsigned long long* p, int64_t v) {
  __hip_atomic_fetch_add(as_global(p), static_cast<unsigned long long>(v), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kCrThreads, 2) void k_hub_credit(HubCreditArgs a) {
  __shared__ __attribute__((aligned(16))) int8_t sm[kCrStages][3][kCrStage];
  // tiles heaviest first (the longest contractions: small row tiles when
  // contracting over t > r, large ones over t < r), so that the light ones
  // fill the last round; runs of consecutive tiles per XCD, as in the
  // count's block, would put the heavy tiles on few XCDs
  const int nrt = a.T / kCrTile, nct = a.K / kCrTile;
  const int heavy = static_cast<int>(blockIdx.x) / nct, tj = static_cast<int>(blockIdx.x) % nct;
  const int ti = a.upper ? heavy : nrt - 1 - heavy;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int row0 = ti * kCrTile + (wave >> 1) * 64;
  const int col0 = tj * kCrTile + (wave & 1) * 64;
  const int r = lane & 31;
  const size_t T = static_cast<size_t>(a.T), K = static_cast<size_t>(a.K), TT = T * T;
  const int t_lo = a.upper ? ti * kCrTile : 0;
  const int t_hi = a.upper ? a.T : (ti + 1) * kCrTile;
  const int nsteps = (t_hi - t_lo) / kCrKStep;
  const v4i ones = {0x01010101, 0x01010101, 0x01010101, 0x01010101};
  const int ar = (wave >> 1) * 64 + r, br = (wave & 1) * 64 + r;
  const int ch = lane >> 5;
  // edge credits of rows below nw take two words, the others one packed word
  const int32_t nw = !a.pos ? 0 : a.wide_all ? a.T : first_narrow_rank(a.off, a.n, a.max_deg_other);
  // the loads of one stage: each wavefront fills 2 x 1 KB of each operand
  int srow[2], scol[2], dst[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int part = wave * 2 + q;
    const int S = part * 64 + lane;
    srow[q] = S >> 2;
    scol[q] = (((S & 3) ^ ((srow[q] >> 1) ^ (srow[q] >> 3))) & 3) * 16;
    dst[q] = part * 1024;
  }
  for (int dg = 0; dg < a.D; ++dg) {
    const int8_t* src[3][2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      src[0][q] = a.A + static_cast<size_t>(dg) * TT + static_cast<size_t>(ti * kCrTile + srow[q]) * T + scol[q];
      src[1][q] = a.A + static_cast<size_t>(a.D + dg) * TT + static_cast<size_t>(ti * kCrTile + srow[q]) * T + scol[q];
      src[2][q] = a.Bt + static_cast<size_t>(tj * kCrTile + srow[q]) * T + scol[q];
    }
    auto issue = [&](int stage, int t) {
#pragma unroll
      for (int op = 0; op < 3; ++op)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src[op][q] + t),
                                           (__attribute__((address_space(3))) void*)(&sm[stage][op][dst[q]]), 16, 0,
                                           0);
    };
    // the previous digit's reads of the ring are done before it is refilled
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    v16i ZX[2][2], ZY[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 16; ++q) ZX[i][j][q] = ZY[i][j][q] = 0;
#pragma unroll
    for (int st = 0; st < kCrStages - 1; ++st)
      if (st < nsteps) issue(st, t_lo + st * kCrKStep);
    for (int step = 0; step < nsteps; ++step) {
      // this wavefront's loads of stage `step` are complete once at most the
      // loads of the later stage issued before this point are pending
      const int after = min(nsteps, step + kCrStages - 1) - step - 1;
      if (after >= 1)
        __builtin_amdgcn_s_waitcnt(0xF70 | 6);  // vmcnt(6): 6 loads per stage
      else
        __builtin_amdgcn_s_waitcnt(0xF70 | 0);
      // every wavefront's part of the stage is in LDS, and the stage read in
      // the previous step may be refilled (a bare barrier, as in k_hub)
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      const int nxt = step + kCrStages - 1;
      if (nxt < nsteps) issue(nxt % kCrStages, t_lo + nxt * kCrKStep);
      const int8_t* sX = sm[step % kCrStages][0];
      const int8_t* sY = sm[step % kCrStages][1];
      const int8_t* sB = sm[step % kCrStages][2];
#pragma unroll
      for (int kk = 0; kk < kCrKStep / 16; kk += 2) {
        const int c = kk + ch;
        const v4i X0 = *reinterpret_cast<const v4i*>(&sX[cr_slot(ar, c)]);
        const v4i X1 = *reinterpret_cast<const v4i*>(&sX[cr_slot(ar + 32, c)]);
        const v4i Y0 = *reinterpret_cast<const v4i*>(&sY[cr_slot(ar, c)]);
        const v4i Y1 = *reinterpret_cast<const v4i*>(&sY[cr_slot(ar + 32, c)]);
        const v4i B0 = *reinterpret_cast<const v4i*>(&sB[cr_slot(br, c)]);
        const v4i B1 = *reinterpret_cast<const v4i*>(&sB[cr_slot(br + 32, c)]);
        const v4i B0a = B0 & ones, B1a = B1 & ones;  // |s| of a sign in {-1, 0, 1}
        ZX[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(X0, B0a, ZX[0][0], 0, 0, 0);
        ZX[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(X0, B1a, ZX[0][1], 0, 0, 0);
        ZX[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(X1, B0a, ZX[1][0], 0, 0, 0);
        ZX[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(X1, B1a, ZX[1][1], 0, 0, 0);
        ZY[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Y0, B0, ZY[0][0], 0, 0, 0);
        ZY[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Y0, B1, ZY[0][1], 0, 0, 0);
        ZY[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Y1, B0, ZY[1][0], 0, 0, 0);
        ZY[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Y1, B1, ZY[1][1], 0, 0, 0);
      }
    }
    // Epilogue of this digit: credits scaled by 2^(7 dg).  Accumulator
    // layout: lane l, register q holds row 8 (q / 4) + 4 (l / 32) + q % 4
    // and column l % 32 of a 32 x 32 block.
    const int64_t scale = int64_t{1} << (kHubDigitBits * dg);
    int64_t mb[2] = {0, 0}, mu[2] = {0, 0};  // mid column sums per j
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int rr = row0 + i * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int y = col0 + j * 32 + (lane & 31);
          const size_t at = static_cast<size_t>(rr) * K + y;
          const int32_t e = as_global(a.E)[at];
          if (e == 0) continue;
          int64_t b2 = static_cast<int64_t>(ZX[i][j][q]) + e * static_cast<int64_t>(ZY[i][j][q]);
          const int64_t u2 = static_cast<int64_t>(ZX[i][j][q]) - e * static_cast<int64_t>(ZY[i][j][q]);
          if (dg == 0) b2 -= 2 * static_cast<int64_t>(as_global(a.Zc)[at]);
          // digit 0: the doubled shares are even; higher digits: scale / 2
          const int64_t bal = dg == 0 ? b2 / 2 : b2 * (scale >> 1);
          const int64_t unb = dg == 0 ? u2 / 2 : u2 * (scale >> 1);
          mb[j] += bal;
          mu[j] += unb;
          if (a.pos) {
            const int32_t pq = as_global(a.pos)[at];
            if (pq >= 0) {
              if (rr < nw) {
                if (bal) add_u64(a.ewb + pq, bal);
                if (unb) add_u64(a.ewu + pq, unb);
              } else if (bal | unb) {
                // the packed word is the integer sum of balanced + 2^32 x
                // unbalanced: negative digit shares wrap and are made good,
                // and both final sums are below 2^32 on this row
                add_u64(a.epack + pq,
                        static_cast<int64_t>(static_cast<uint64_t>(bal) + (static_cast<uint64_t>(unb) << 32)));
              }
            }
          }
        }
      }
    if (a.orig_mid) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        int64_t b = mb[j], u = mu[j];
        b += __shfl_xor(b, 32, 64);
        u += __shfl_xor(u, 32, 64);
        if (lane < 32) {
          const int y = col0 + j * 32 + lane;
          if (b | u) {
            const int32_t id = a.orig_mid[y];
            if (b) add_u64(a.bal_mid + id, b);
            if (u) add_u64(a.unb_mid + id, u);
          }
        }
      }
    }
  }
}

}  // namespace dev

hipError_t launch_pv_hub_tally(const HubTallyArgs* sides, int n, int grid, hipStream_t st) {
  for (int i = 0; i < n; ++i) {
    const HubTallyArgs& a = sides[i];
    if (a.n_items == 0) continue;
    if (a.T > kMaxPVHubT) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dev::k_pv_hub_tally, dim3(grid < a.n_items ? grid : a.n_items), dim3(dev::kHubTallyThreads), 0,
                       st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_hub_digits(const HubDigitArgs& a, hipStream_t st) {
  if (a.T <= 0) return hipSuccess;
  if (a.T % dev::kDigTile != 0 || a.D < 1 || a.D > dev::kMaxDigits) return hipErrorInvalidValue;
  const unsigned nt = static_cast<unsigned>(a.T / dev::kDigTile);
  hipLaunchKernelGGL(dev::k_hub_digits, dim3(nt, nt), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_hub_credit(const HubCreditArgs& a, hipStream_t st) {
  if (a.T <= 0 || a.K <= 0) return hipSuccess;
  if (a.T % dev::kCrTile != 0 || a.K % dev::kCrTile != 0 || a.D < 1 || a.D > dev::kMaxDigits)
    return hipErrorInvalidValue;
  const unsigned tiles = static_cast<unsigned>((a.T / dev::kCrTile) * (a.K / dev::kCrTile));
  hipLaunchKernelGGL(dev::k_hub_credit, dim3(tiles), dim3(dev::kCrThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace dbbc
