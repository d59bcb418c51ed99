// Device memory cache of the library.  Problems, preconditioners and sequences
// come and go once per job; hipMalloc costs tens of microseconds and hipFree
// synchronises the whole device, so released blocks are kept and handed out
// again.  Stream order makes reuse safe: a block released on stream s is
// given out again at once on s (every earlier use on s precedes the new one),
// and on another stream once the event recorded at its release has completed.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace pmor {
namespace {

struct Cached {
  void* p;
  int device;
  hipStream_t stream;
  hipEvent_t done;
};

struct Cache {
  std::mutex mu;
  std::multimap<size_t, Cached> free_blocks;  // by size
  std::map<void*, size_t> live;               // size of every block handed out
  std::map<int, std::vector<hipEvent_t>> events;  // spare events per device
  size_t cached_bytes = 0;
};

Cache& cache() {
  static Cache* c = new Cache();  // never destroyed: the HIP runtime may be gone at exit
  return *c;
}

size_t round_size(size_t b) { return ((b < 256 ? 256 : b) + 255) & ~size_t(255); }

// every cached block back to the runtime (the device is synchronised first)
void trim_locked(Cache& c) {
  (void)hipDeviceSynchronize();
  for (auto& kv : c.free_blocks) {
    (void)hipFree(kv.second.p);
    c.events[kv.second.device].push_back(kv.second.done);
  }
  c.free_blocks.clear();
  c.cached_bytes = 0;
}

}  // namespace

hipError_t dmalloc(void** p, size_t bytes, hipStream_t s) {
  Cache& c = cache();
  const size_t need = round_size(bytes);
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(c.mu);
  // a cached block of at least the size, at most twice it (or 1 MiB more)
  const size_t hi = std::max(2 * need, need + ((size_t)1 << 20));
  auto first = c.free_blocks.lower_bound(need);
  auto end = c.free_blocks.upper_bound(hi);
  for (int pass = 0; pass < 2; ++pass) {
    for (auto it = first; it != end; ++it) {
      if (it->second.device != dev) continue;
      const bool ok = pass == 0 ? it->second.stream == s : hipEventQuery(it->second.done) == hipSuccess;
      if (!ok) continue;
      *p = it->second.p;
      c.live[*p] = it->first;
      c.cached_bytes -= it->first;
      c.events[dev].push_back(it->second.done);
      c.free_blocks.erase(it);
      return hipSuccess;
    }
  }
  hipError_t e = hipMalloc(p, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim_locked(c);
    e = hipMalloc(p, need);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return e;
    }
  }
  c.live[*p] = need;
  return hipSuccess;
}

void dfree(void* p, hipStream_t s) {
  if (!p) return;
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) {  // not from the cache
    (void)hipFree(p);
    return;
  }
  const size_t sz = it->second;
  c.live.erase(it);
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipEvent_t ev = nullptr;
  auto& spare = c.events[dev];
  if (!spare.empty()) {
    ev = spare.back();
    spare.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    (void)hipFree(p);
    return;
  }
  if (hipEventRecord(ev, s) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    (void)hipFree(p);
    spare.push_back(ev);
    return;
  }
  c.free_blocks.insert({sz, Cached{p, dev, s, ev}});
  c.cached_bytes += sz;
}

void dtrim() {
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  trim_locked(c);
}

}  // namespace pmor
