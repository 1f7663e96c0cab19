// Device memory of libdbbc.  Every device allocation the library makes goes
// through a DevBuf, which takes its memory from the allocator of the entry
// point that is running on the calling thread (the caller's dbbc_allocator,
// or hipMalloc / hipFree by default) and gives it back to the same allocator.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <utility>

#include "../../include/dbbc.h"

namespace dbbc {

// An allocator and the stream its memory is handed out for.
struct DevAlloc {
  dbbc_allocator a{nullptr, nullptr, nullptr};  // a.alloc == NULL: hipMalloc / hipFree
  void* stream = nullptr;

  hipError_t get(void** p, size_t n) const {
    *p = nullptr;
    if (!a.alloc) return hipMalloc(p, n);
    *p = a.alloc(n, stream, a.ctx);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  void put(void* p) const {
    if (!p) return;
    if (!a.alloc) {
      (void)hipFree(p);
    } else {
      a.free(p, stream, a.ctx);
    }
  }
};

// The calling thread's current allocator (hipMalloc outside any AllocScope).
inline thread_local DevAlloc g_current_alloc;

inline const DevAlloc& current_alloc() { return g_current_alloc; }

// Within its lifetime, allocations of the calling thread go to a (handed out
// for stream st); the previous allocator comes back at the end.
class AllocScope {
 public:
  AllocScope(const DevAlloc& a, void* st) : prev_(g_current_alloc) {
    g_current_alloc = a;
    g_current_alloc.stream = st;
  }
  ~AllocScope() { g_current_alloc = prev_; }
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;

 private:
  DevAlloc prev_;
};

// Owned device memory; freed (to the allocator it came from) on destruction.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevAlloc from;

  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), from(o.from) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      from = o.from;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }

  void release() {
    from.put(p);
    p = nullptr;
    bytes = 0;
  }
  // n bytes (at least 16 when n > 0) from the current allocator; n == 0
  // leaves the buffer empty
  hipError_t alloc(size_t n) {
    release();
    if (n == 0) return hipSuccess;
    from = current_alloc();
    hipError_t e = from.get(&p, std::max<size_t>(n, 16));
    if (e == hipSuccess) bytes = n;
    return e;
  }
  // keep the allocation if it is already large enough
  hipError_t reserve(size_t n) {
    if (n <= bytes && (p || n == 0)) return hipSuccess;
    return alloc(n);
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

}  // namespace dbbc
