// Device ingestion of an edge list in text form: the one-GPU counterpart of
// the paper's Phase 1 (parallel loading, every range aligned to whole edge
// records) and Phase 2 (vertex identifiers made contiguous), ending in the
// device graph build.
//   1. every line start is found in parallel (a line starts at byte 0 or
//      after a newline), so each record is parsed whole by one thread: the
//      record alignment of Phase 1 at the finest grain;
//   2. each line is parsed into (u, v, sign) or marked blank / comment /
//      malformed; records keep their line order (duplicates: the last one
//      wins in the build, as in the paper's datasets);
//   3. per side, the raw ids are radix-sorted with their record index; a
//      run of equal ids is one vertex, numbered by its place among the
//      distinct ids (increasing raw id), which is the compact identifier of
//      Phase 2; the distinct raw ids are kept as the compact -> raw map.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <string>

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

// Line starts (byte 0, or the byte after a newline), flagged and counted.
__global__ void k_line_flags(const char* t, int64_t len, uint8_t* flag, unsigned long long* count) {
  unsigned long long c = 0;
  GRID_STRIDE(i, len) {
    const bool start = i == 0 || t[i - 1] == '\n';
    flag[i] = start ? 1 : 0;
    c += start ? 1 : 0;
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

// Line kinds.
enum : uint8_t { kRecord = 0, kSkip = 1, kBad = 2 };

__device__ __forceinline__ bool is_space(char c) { return c == ' ' || c == '\t' || c == ',' || c == '\r'; }

// One line [b, end of line): "u v s" with u, v decimal ids below 2^63 and s
// one of 1, +1 (positive), 0, -1 (negative); fields separated by spaces,
// tabs or commas; fields after the third are ignored.  Blank lines and lines
// whose first non-space character is '#' or '%' are skipped.
__global__ void k_parse(const char* t, int64_t len, const int64_t* starts, int64_t lines, uint64_t* ru,
                        uint64_t* rv, int8_t* rs, uint8_t* kind, unsigned long long* first_bad) {
  GRID_STRIDE(l, lines) {
    int64_t p = starts[l];
    auto at_end = [&]() { return p >= len || t[p] == '\n'; };
    auto skip_space = [&]() {
      while (!at_end() && is_space(t[p])) ++p;
    };
    auto number = [&](uint64_t& out) {
      if (at_end() || t[p] < '0' || t[p] > '9') return false;
      uint64_t x = 0;
      while (!at_end() && t[p] >= '0' && t[p] <= '9') {
        if (x > (~0ull >> 1) / 10) return false;  // beyond 2^63
        x = x * 10 + static_cast<uint64_t>(t[p] - '0');
        ++p;
      }
      if (x >> 63) return false;
      out = x;
      return at_end() || is_space(t[p]);
    };
    uint8_t k = kBad;
    skip_space();
    if (at_end() || t[p] == '#' || t[p] == '%') {
      k = kSkip;
    } else {
      uint64_t a = 0, b = 0, sv = 0;
      bool neg = false;
      bool ok = number(a);
      if (ok) {
        skip_space();
        ok = number(b);
      }
      if (ok) {
        skip_space();
        if (!at_end() && (t[p] == '-' || t[p] == '+')) {
          neg = t[p] == '-';
          ++p;
        }
        ok = number(sv) && (neg ? sv == 1 : sv <= 1);
      }
      if (ok) {
        ru[l] = a;
        rv[l] = b;
        rs[l] = (neg || sv == 0) ? int8_t(-1) : int8_t(1);
        k = kRecord;
      }
    }
    kind[l] = k;
    if (k == kBad) atomicMin(first_bad, static_cast<unsigned long long>(l));
  }
}

__global__ void k_is_record(const uint8_t* kind, int64_t n, uint8_t* flag) {
  GRID_STRIDE(i, n) flag[i] = kind[i] == kRecord ? 1 : 0;
}

__global__ void k_gather_records(const int64_t* lines, int64_t m, const uint64_t* ru, const uint64_t* rv,
                                 const int8_t* rs, uint64_t* u, uint64_t* v, int8_t* s, uint32_t* idx0,
                                 uint32_t* idx1) {
  GRID_STRIDE(i, m) {
    const int64_t l = lines[i];
    u[i] = ru[l];
    v[i] = rv[l];
    s[i] = rs[l];
    idx0[i] = static_cast<uint32_t>(i);
    idx1[i] = static_cast<uint32_t>(i);
  }
}

__global__ void k_run_heads(const uint64_t* sorted, int64_t m, uint32_t* head) {
  GRID_STRIDE(i, m) head[i] = (i == 0 || sorted[i] != sorted[i - 1]) ? 1u : 0u;
}

// After an inclusive scan of the run heads: record idx[i] gets compact id
// scan[i] - 1; the first element of each run writes the raw id to the map.
__global__ void k_assign_ids(const uint64_t* sorted, const uint32_t* idx, const uint32_t* head,
                             const uint32_t* scan, int64_t m, int32_t* id, int64_t* raw_of) {
  GRID_STRIDE(i, m) {
    const uint32_t c = scan[i] - 1u;
    id[idx[i]] = static_cast<int32_t>(c);
    if (head[i]) raw_of[c] = static_cast<int64_t>(sorted[i]);
  }
}

// Device memory of one step, freed on scope exit (at least 16 bytes, so
// that even an empty array has an address).
struct Tmp : DevBuf {
  hipError_t alloc(size_t bytes) { return DevBuf::alloc(std::max<size_t>(bytes, 16)); }
};

struct Fail {
  int status;
  std::string msg;
};

#define DEV_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw Fail{e_ == hipErrorOutOfMemory ? DBBC_E_OOM : DBBC_E_DEVICE,                \
                 std::string(#expr) + ": " + hipGetErrorString(e_)};                    \
  } while (0)

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
T to_host_one(const T* d, hipStream_t st) {
  T h{};
  DEV_TRY(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, st));
  DEV_TRY(hipStreamSynchronize(st));
  return h;
}

// Positions i in [0, n) with flag[i] set, in order, into out; returns count.
int64_t select_positions(CubTmp& ct, const uint8_t* flag, int64_t n, int64_t* out, int64_t* d_count, hipStream_t st) {
  hipcub::CountingInputIterator<int64_t> it(0);
  size_t need = 0;
  DEV_TRY(hipcub::DeviceSelect::Flagged(nullptr, need, it, flag, out, d_count, static_cast<int>(n), st));
  void* t = ct.get(need);
  DEV_TRY(hipcub::DeviceSelect::Flagged(t, need, it, flag, out, d_count, static_cast<int>(n), st));
  return to_host_one(d_count, st);
}

int bits_for_max(uint64_t mx) {
  int b = 1;
  while (b < 64 && (mx >> b) != 0) ++b;
  return b;
}

// Compact ids of one side: id[i] for record i, the raw id of each compact
// id into raw_of (ascending); returns the number of distinct ids.
int64_t compact_side(CubTmp& ct, uint64_t* keys, uint64_t* keys_alt, uint32_t* idx, uint32_t* idx_alt, int64_t m,
                     int32_t* id, IngestOut& out, int side, hipStream_t st) {
  size_t need = 0;
  uint64_t* d_max = keys_alt;  // scratch word before the sort uses it
  DEV_TRY(hipcub::DeviceReduce::Max(nullptr, need, keys, d_max, static_cast<int>(m), st));
  void* t = ct.get(need);
  DEV_TRY(hipcub::DeviceReduce::Max(t, need, keys, d_max, static_cast<int>(m), st));
  const int end_bit = bits_for_max(to_host_one(d_max, st));
  need = 0;
  DEV_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, need, keys, keys_alt, idx, idx_alt, static_cast<int>(m), 0,
                                             end_bit, st));
  t = ct.get(need);
  DEV_TRY(hipcub::DeviceRadixSort::SortPairs(t, need, keys, keys_alt, idx, idx_alt, static_cast<int>(m), 0, end_bit,
                                             st));
  Tmp head, scan;
  DEV_TRY(head.alloc(static_cast<size_t>(m) * 4));
  DEV_TRY(scan.alloc(static_cast<size_t>(m) * 4));
  hipLaunchKernelGGL(k_run_heads, dim3(grid_for(m)), dim3(kThreads), 0, st, keys_alt, m, head.as<uint32_t>());
  DEV_TRY(hipGetLastError());
  need = 0;
  DEV_TRY(hipcub::DeviceScan::InclusiveSum(nullptr, need, head.as<uint32_t>(), scan.as<uint32_t>(),
                                           static_cast<int>(m), st));
  t = ct.get(need);
  DEV_TRY(hipcub::DeviceScan::InclusiveSum(t, need, head.as<uint32_t>(), scan.as<uint32_t>(), static_cast<int>(m),
                                           st));
  const int64_t n = to_host_one(scan.as<uint32_t>() + (m - 1), st);
  DEV_TRY(out.raw[side].alloc(std::max<size_t>(static_cast<size_t>(n) * 8, 16)));
  out.raw[side].bytes = static_cast<size_t>(n) * 8;
  hipLaunchKernelGGL(k_assign_ids, dim3(grid_for(m)), dim3(kThreads), 0, st, keys_alt, idx_alt,
                     head.as<uint32_t>(), scan.as<uint32_t>(), m, id, out.raw[side].as<int64_t>());
  DEV_TRY(hipGetLastError());
  DEV_TRY(hipStreamSynchronize(st));
  return n;
}

void ingest(const char* text_in, int64_t len, uint32_t flags, hipStream_t st, HostGraph& g, DeviceCsr& csr,
            IngestOut& out) {
  CubTmp ct;
  Tmp dtext;
  const char* text = text_in;
  if (!(flags & DBBC_INPUT_DEVICE)) {
    DEV_TRY(dtext.alloc(static_cast<size_t>(len)));
    if (len) DEV_TRY(hipMemcpyAsync(dtext.p, text_in, static_cast<size_t>(len), hipMemcpyHostToDevice, st));
    text = dtext.as<char>();
  }
  Tmp flag, starts, count, bad;
  DEV_TRY(flag.alloc(static_cast<size_t>(len)));
  DEV_TRY(count.alloc(8));
  DEV_TRY(bad.alloc(8));
  DEV_TRY(launch_fill_u64(bad.as<unsigned long long>(), 1, ~0ull, st));
  int64_t lines = 0;
  if (len) {
    // the lines are counted first: the start list is sized to them
    DEV_TRY(launch_fill_u64(count.as<unsigned long long>(), 1, 0ull, st));
    hipLaunchKernelGGL(k_line_flags, dim3(grid_for(len)), dim3(kThreads), 0, st, text, len, flag.as<uint8_t>(),
                       count.as<unsigned long long>());
    DEV_TRY(hipGetLastError());
    lines = static_cast<int64_t>(to_host_one(count.as<unsigned long long>(), st));
    DEV_TRY(starts.alloc(static_cast<size_t>(lines) * 8));
    if (select_positions(ct, flag.as<uint8_t>(), len, starts.as<int64_t>(), count.as<int64_t>(), st) != lines)
      throw Fail{DBBC_E_DEVICE, "line count mismatch"};
  }
  Tmp ru, rv, rs, kind;
  DEV_TRY(ru.alloc(static_cast<size_t>(lines) * 8));
  DEV_TRY(rv.alloc(static_cast<size_t>(lines) * 8));
  DEV_TRY(rs.alloc(static_cast<size_t>(lines)));
  DEV_TRY(kind.alloc(static_cast<size_t>(lines)));
  if (lines) {
    hipLaunchKernelGGL(k_parse, dim3(grid_for(lines)), dim3(kThreads), 0, st, text, len, starts.as<int64_t>(), lines,
                       ru.as<uint64_t>(), rv.as<uint64_t>(), rs.as<int8_t>(), kind.as<uint8_t>(),
                       bad.as<unsigned long long>());
    DEV_TRY(hipGetLastError());
  }
  const unsigned long long first_bad = to_host_one(bad.as<unsigned long long>(), st);
  if (first_bad != ~0ull)
    throw Fail{DBBC_E_PARSE, "line " + std::to_string(first_bad + 1) +
                                 ": expected \"u v s\" with ids below 2^63 and s in {1, 0, -1, +1}"};
  // the records, in line order
  Tmp rec_lines;
  DEV_TRY(rec_lines.alloc(static_cast<size_t>(lines) * 8));
  int64_t m = 0;
  if (lines) {
    hipLaunchKernelGGL(k_is_record, dim3(grid_for(lines)), dim3(kThreads), 0, st, kind.as<uint8_t>(), lines,
                       flag.as<uint8_t>());
    DEV_TRY(hipGetLastError());
    m = select_positions(ct, flag.as<uint8_t>(), lines, rec_lines.as<int64_t>(), count.as<int64_t>(), st);
  }
  if (m >= (int64_t(1) << 31) - 1) throw Fail{DBBC_E_TOO_LARGE, "more than 2^31 - 2 edge records"};
  out.lines = lines;
  out.records = m;
  if (m == 0) throw Fail{DBBC_E_INVALID_ARG, "the text holds no edge record"};
  Tmp ku, kv, kalt, ss, i0, i1, i2, iu, iv;
  const size_t M = static_cast<size_t>(m);
  DEV_TRY(ku.alloc(M * 8));
  DEV_TRY(kv.alloc(M * 8));
  DEV_TRY(kalt.alloc(M * 8));
  DEV_TRY(ss.alloc(M));
  DEV_TRY(i0.alloc(M * 4));
  DEV_TRY(i1.alloc(M * 4));
  DEV_TRY(i2.alloc(M * 4));
  DEV_TRY(iu.alloc(M * 4));
  DEV_TRY(iv.alloc(M * 4));
  hipLaunchKernelGGL(k_gather_records, dim3(grid_for(m)), dim3(kThreads), 0, st, rec_lines.as<int64_t>(), m,
                     ru.as<uint64_t>(), rv.as<uint64_t>(), rs.as<int8_t>(), ku.as<uint64_t>(), kv.as<uint64_t>(),
                     ss.as<int8_t>(), i0.as<uint32_t>(), i1.as<uint32_t>());
  DEV_TRY(hipGetLastError());
  // free the per-line arrays before the sorts
  DEV_TRY(hipStreamSynchronize(st));
  (void)ru.alloc(0);
  (void)rv.alloc(0);
  (void)starts.alloc(0);
  (void)flag.alloc(0);
  const int64_t n_u = compact_side(ct, ku.as<uint64_t>(), kalt.as<uint64_t>(), i0.as<uint32_t>(), i2.as<uint32_t>(),
                                   m, iu.as<int32_t>(), out, 0, st);
  const int64_t n_v = compact_side(ct, kv.as<uint64_t>(), kalt.as<uint64_t>(), i1.as<uint32_t>(), i2.as<uint32_t>(),
                                   m, iv.as<int32_t>(), out, 1, st);
  if (n_u + n_v >= (int64_t(1) << 30)) throw Fail{DBBC_E_TOO_LARGE, "n_u + n_v must be below 2^30"};
  std::string err;
  const int rc = build_device_graph(static_cast<int32_t>(n_u), static_cast<int32_t>(n_v), m, iu.as<int32_t>(),
                                    iv.as<int32_t>(), ss.as<int8_t>(), (flags & ~DBBC_INPUT_DEVICE) | DBBC_INPUT_DEVICE,
                                    st, g, csr, err);
  if (rc != DBBC_OK) throw Fail{rc, err};
}

}  // namespace

int ingest_text(const char* text, int64_t len, uint32_t flags, hipStream_t st, HostGraph& g, DeviceCsr& csr,
                IngestOut& out, std::string& err) {
  if (len < 0 || (len > 0 && !text)) {
    err = "text must not be NULL and len must be non-negative";
    return DBBC_E_INVALID_ARG;
  }
  if (len >= (int64_t(1) << 31) - 1) {
    err = "text longer than 2^31 - 2 bytes";
    return DBBC_E_TOO_LARGE;
  }
  auto drop_maps = [&]() {
    (void)hipStreamSynchronize(st);
    for (int s = 0; s < 2; ++s) out.raw[s].release();
  };
  try {
    ingest(text, len, flags, st, g, csr, out);
  } catch (const Fail& f) {
    err = f.msg;
    drop_maps();
    return f.status;
  } catch (const std::bad_alloc&) {
    err = "host allocation failed while reading the text";
    drop_maps();
    return DBBC_E_OOM;
  }
  return DBBC_OK;
}

}  // namespace dbbc
