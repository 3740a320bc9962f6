// Stream-ordered caching allocator behind DBuf.
//
// A solver's setup makes a few hundred device allocations and frees about
// half of them again, and every hipFree waits for the whole device; a solver
// destroyed after its solve frees gigabytes (the Krylov bases).  Freed blocks
// are therefore kept per device and handed out again.  A block freed while an
// API call runs on stream s is tagged with s: work queued on s later runs
// after every earlier use of the block, so the block may be reused on s at
// once.  Reuse on another stream first waits for the device; a block becomes
// free for any stream once its stream has been synchronised (solver destroy,
// stream change).  Outside an API call (no stream known) blocks go straight
// back to the runtime.  The cache holds at most a fixed share of the device's
// memory; a failed hipMalloc releases it and tries again.
#include <map>
#include <mutex>
#include <unordered_map>

#include "gmg_internal.h"

namespace gmg {

namespace {

struct FreeBlock {
  void* p;
  hipStream_t s;
  bool idle;  // its stream has been synchronised since it was freed
};

struct DevPool {
  std::mutex mu;
  std::multimap<size_t, FreeBlock> free_by_size;
  std::unordered_map<void*, size_t> size_of;  // every block handed out by the pool
  size_t cached = 0;                           // bytes in free_by_size
  size_t cap = 0;                              // most bytes kept
};

thread_local bool t_has_stream = false;
thread_local hipStream_t t_stream = nullptr;

DevPool& pool_of_current_device() {
  // never destroyed: freeing device memory during process teardown may
  // outlive the runtime
  static std::mutex mu;
  static std::map<int, DevPool*>* pools = new std::map<int, DevPool*>();
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(mu);
  DevPool*& d = (*pools)[dev];
  if (!d) {
    d = new DevPool();
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      tot = (size_t)16 << 30;
    }
    d->cap = tot / 8;
    if (const char* e = std::getenv("GMG_POOL_MB")) d->cap = (size_t)std::max(0LL, std::atoll(e)) << 20;
  }
  return *d;
}

size_t round_size(size_t bytes) {
  const size_t g = bytes < ((size_t)1 << 20) ? 256 : ((size_t)2 << 20);
  return (bytes + g - 1) / g * g;
}

// under d.mu
void release_cached(DevPool& d) {
  if (d.free_by_size.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : d.free_by_size) {
    (void)hipFree(kv.second.p);
    d.size_of.erase(kv.second.p);
  }
  d.free_by_size.clear();
  d.cached = 0;
}

}  // namespace

PoolStream::PoolStream(hipStream_t s) : had_(t_has_stream), prev_(t_stream) {
  t_has_stream = true;
  t_stream = s;
}
PoolStream::~PoolStream() {
  t_has_stream = had_;
  t_stream = prev_;
}

void* pool_alloc(size_t bytes) {
  if (bytes == 0) return nullptr;
  DevPool& d = pool_of_current_device();
  const size_t rb = round_size(bytes);
  std::lock_guard<std::mutex> g(d.mu);
  if (t_has_stream) {
    // the smallest cached block that fits with at most a quarter to spare
    const size_t most = rb + rb / 4;
    auto pick = d.free_by_size.end();
    bool other_stream = false;
    for (auto it = d.free_by_size.lower_bound(rb); it != d.free_by_size.end() && it->first <= most; ++it) {
      if (it->second.idle || it->second.s == t_stream) {
        pick = it;
        break;
      }
      if (pick == d.free_by_size.end()) { pick = it; other_stream = true; }
    }
    if (pick != d.free_by_size.end()) {
      if (other_stream) {
        // last used on another stream: wait for the device, then every
        // cached block is free for any stream
        (void)hipDeviceSynchronize();
        for (auto& kv : d.free_by_size) kv.second.idle = true;
      }
      void* p = pick->second.p;
      d.cached -= pick->first;
      d.free_by_size.erase(pick);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, rb) != hipSuccess) {
    (void)hipGetLastError();
    release_cached(d);
    if (hipMalloc(&p, rb) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  d.size_of[p] = rb;
  return p;
}

void pool_free(void* p) {
  if (!p) return;
  DevPool& d = pool_of_current_device();
  std::lock_guard<std::mutex> g(d.mu);
  auto it = d.size_of.find(p);
  if (it == d.size_of.end()) {
    (void)hipFree(p);
    return;
  }
  const size_t sz = it->second;
  if (!t_has_stream || d.cached + sz > d.cap) {
    d.size_of.erase(it);
    (void)hipFree(p);
    return;
  }
  d.free_by_size.emplace(sz, FreeBlock{p, t_stream, false});
  d.cached += sz;
}

void pool_idle(hipStream_t s) {
  DevPool& d = pool_of_current_device();
  std::lock_guard<std::mutex> g(d.mu);
  for (auto& kv : d.free_by_size)
    if (kv.second.s == s) kv.second.idle = true;
}

}  // namespace gmg
