// Device memory cache of the library.  Problems, preconditioners and sequences
// come and go once per job; hipMalloc costs tens of microseconds and hipFree
// synchronises the whole device, so released blocks are kept and handed out
// again.  Stream order makes reuse safe: a block released on stream s is
// given out again at once on s (every earlier use on s precedes the new one),
// and on another stream once the event recorded at its release has completed
// (a block whose stream was retired, see dstream_retire, is free for any).
// New blocks of up to SLAB_BLOCK bytes are cut from slabs of SLAB bytes (one
// hipMalloc per slab instead of one per block: setting up hundreds of systems
// at once asks for thousands of small arrays); a slab goes back to the runtime
// when every block cut from it has been released and trimmed.
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

constexpr size_t SLAB = (size_t)256 << 20;
constexpr size_t SLAB_BLOCK = (size_t)16 << 20;

struct Slab {
  void* base;
  size_t used;     // bytes cut so far (blocks are cut in order, never merged)
  int64_t blocks;  // blocks cut from it that are live or cached
  int device;
};

struct Cache {
  std::mutex mu;
  std::multimap<size_t, Cached> free_blocks;  // by size
  std::map<void*, size_t> live;               // size of every block handed out
  std::map<int, std::vector<hipEvent_t>> events;  // spare events per device
  std::map<void*, Slab*> owner;               // slab of every block cut from one
  std::map<int, Slab*> open;                  // the slab new blocks are cut from, per device
  size_t cached_bytes = 0;
};

Cache& cache() {
  static Cache* c = new Cache();  // never destroyed: the HIP runtime may be gone at exit
  return *c;
}

size_t round_size(size_t b) { return ((b < 256 ? 256 : b) + 255) & ~size_t(255); }

// a block cut from a slab is dropped: the slab is freed once none of its blocks is left
void drop_slab_block(Cache& c, std::map<void*, Slab*>::iterator it) {
  Slab* s = it->second;
  c.owner.erase(it);
  if (--s->blocks > 0) return;
  auto op = c.open.find(s->device);
  if (op != c.open.end() && op->second == s) c.open.erase(op);
  (void)hipFree(s->base);
  delete s;
}

// every cached block back to the runtime (the device is synchronised first)
void trim_locked(Cache& c) {
  (void)hipDeviceSynchronize();
  for (auto& kv : c.free_blocks) {
    auto ow = c.owner.find(kv.second.p);
    if (ow != c.owner.end()) drop_slab_block(c, ow);
    else (void)hipFree(kv.second.p);
    if (kv.second.done) c.events[kv.second.device].push_back(kv.second.done);
  }
  c.free_blocks.clear();
  c.cached_bytes = 0;
}

// a block no stream uses any more, back to the runtime (or dropped from its slab)
void release_now(Cache& c, void* p) {
  auto ow = c.owner.find(p);
  if (ow != c.owner.end()) drop_slab_block(c, ow);
  else (void)hipFree(p);
}

// a new block of `need` bytes (a multiple of 256) on device dev: cut from the
// device's open slab, a new slab when it is full, or its own hipMalloc when
// larger than SLAB_BLOCK or when no slab can be had
hipError_t fresh_locked(Cache& c, void** p, size_t need, int dev) {
  if (need <= SLAB_BLOCK) {
    Slab* s = c.open.count(dev) ? c.open[dev] : nullptr;
    if (!s || s->used + need > SLAB) {
      void* base = nullptr;
      if (hipMalloc(&base, SLAB) == hipSuccess) {
        s = new Slab{base, 0, 0, dev};
        c.open[dev] = s;  // the old slab stays until its blocks are dropped
      } else {
        (void)hipGetLastError();
        s = nullptr;
      }
    }
    if (s) {
      *p = static_cast<char*>(s->base) + s->used;
      s->used += need;
      ++s->blocks;
      c.owner[*p] = s;
      return hipSuccess;
    }
  }
  return hipMalloc(p, need);
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
      const bool ok = pass == 0 ? (it->second.stream == s && it->second.done != nullptr)
                                : (it->second.done == nullptr || hipEventQuery(it->second.done) == hipSuccess);
      if (!ok) continue;
      *p = it->second.p;
      c.live[*p] = it->first;
      c.cached_bytes -= it->first;
      if (it->second.done) c.events[dev].push_back(it->second.done);
      c.free_blocks.erase(it);
      return hipSuccess;
    }
  }
  hipError_t e = fresh_locked(c, p, need, dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim_locked(c);
    e = fresh_locked(c, p, need, dev);
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
    release_now(c, p);
    return;
  }
  if (hipEventRecord(ev, s) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    release_now(c, p);
    spare.push_back(ev);
    return;
  }
  c.free_blocks.insert({sz, Cached{p, dev, s, ev}});
  c.cached_bytes += sz;
}

// stream s is complete and about to be destroyed: its cached blocks no longer
// name it, and their release events (recorded on it) go back to the spare pool,
// so that no later call queries an event of a destroyed stream
void dstream_retire(hipStream_t s) {
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  for (auto& kv : c.free_blocks) {
    Cached& b = kv.second;
    if (b.stream != s || !b.done) continue;
    c.events[b.device].push_back(b.done);
    b.done = nullptr;  // free for any stream
    b.stream = nullptr;
  }
}

void dtrim() {
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  trim_locked(c);
}

}  // namespace pmor
