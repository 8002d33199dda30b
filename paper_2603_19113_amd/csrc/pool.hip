// Caching allocators of libmfs: device blocks with stream-ordered reuse, and pinned host blocks.
//
// A scene's tables, pair partial sums and Krylov basis are large and short-lived under a request
// loop.  hipMalloc and hipFree are slow and hipFree waits for the device, which would stall every
// other request running on it.  Freed blocks therefore stay on the device in a size-ordered cache.
// A block returned with pool_free carries an event recorded on the stream of its last use; the next
// owner makes its own stream wait for that event (or waits on the host when it has no stream), so
// reuse is ordered without any device-wide synchronisation.  The cache is bounded; when hipMalloc
// runs out of memory the cache of that device is released and the allocation retried once.
#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "mfs_internal.h"

namespace mfs {
namespace {

struct Cached {
  void* p;
  size_t bytes;
  int dev;
  hipEvent_t ready;  // recorded after the last use; null when none is needed
};

struct DevicePool {
  std::mutex mu;
  std::multimap<size_t, Cached> free_;
  size_t cached = 0;
  size_t live = 0;
  size_t limit = size_t(64) << 30;
  int64_t hits = 0, misses = 0;
};

struct HostPool {
  std::mutex mu;
  std::multimap<size_t, void*> free_;
  size_t cached = 0;
  size_t limit = size_t(256) << 20;
};

// Never destroyed: blocks may be returned from static destructors of callers.
DevicePool& dpool() {
  static DevicePool* p = new DevicePool();
  return *p;
}
HostPool& hpool() {
  static HostPool* p = new HostPool();
  return *p;
}

size_t round_size(size_t b) {
  const size_t small = size_t(1) << 20, big = size_t(2) << 20;
  if (b < small) return (b + 511) / 512 * 512;
  return (b + big - 1) / big * big;
}

// Release cached blocks of device `dev` (-1: every device).  Caller holds the lock.
void release_cached(DevicePool& P, int dev) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto it = P.free_.begin(); it != P.free_.end();) {
    Cached& c = it->second;
    if (dev >= 0 && c.dev != dev) {
      ++it;
      continue;
    }
    if (c.ready) {
      (void)hipEventSynchronize(c.ready);
      (void)hipEventDestroy(c.ready);
    }
    if (c.dev != cur) (void)hipSetDevice(c.dev);
    (void)hipFree(c.p);
    if (c.dev != cur) (void)hipSetDevice(cur);
    P.cached -= c.bytes;
    it = P.free_.erase(it);
  }
}

}  // namespace

void* pool_alloc(size_t bytes, hipStream_t st, size_t* got, hipError_t* err) {
  *err = hipSuccess;
  const size_t b = round_size(std::max<size_t>(bytes, 1));
  int dev = 0;
  (void)hipGetDevice(&dev);
  DevicePool& P = dpool();
  Cached hit{nullptr, 0, 0, nullptr};
  {
    std::lock_guard<std::mutex> lk(P.mu);
    // smallest cached block that fits, wasting at most half of it
    for (auto it = P.free_.lower_bound(b); it != P.free_.end() && it->first <= 2 * b; ++it) {
      if (it->second.dev != dev) continue;
      hit = it->second;
      P.free_.erase(it);
      P.cached -= hit.bytes;
      P.live += hit.bytes;
      ++P.hits;
      break;
    }
  }
  if (hit.p) {
    if (hit.ready) {
      hipError_t e = st ? hipStreamWaitEvent(st, hit.ready, 0) : hipEventSynchronize(hit.ready);
      (void)hipEventDestroy(hit.ready);
      if (e != hipSuccess) {
        *err = e;
        pool_free(hit.p, hit.bytes, nullptr);
        return nullptr;
      }
    }
    *got = hit.bytes;
    return hit.p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, b);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(P.mu);
      release_cached(P, dev);
    }
    e = hipMalloc(&p, b);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *err = e;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(P.mu);
  P.live += b;
  ++P.misses;
  *got = b;
  return p;
}

void pool_free(void* p, size_t bytes, hipStream_t last) {
  if (!p) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
    if (hipEventRecord(ev, last) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipEventDestroy(ev);
      ev = nullptr;
    }
  } else {
    (void)hipGetLastError();
    ev = nullptr;
  }
  DevicePool& P = dpool();
  std::lock_guard<std::mutex> lk(P.mu);
  P.live -= std::min(P.live, bytes);
  if (!ev || P.cached + bytes > P.limit) {  // not cacheable: free for good after its last use
    if (ev) {
      (void)hipEventSynchronize(ev);
      (void)hipEventDestroy(ev);
    } else {
      (void)hipStreamSynchronize(last);
    }
    (void)hipFree(p);
    return;
  }
  P.free_.emplace(bytes, Cached{p, bytes, dev, ev});
  P.cached += bytes;
}

void* pinned_alloc(size_t bytes, size_t* got, hipError_t* err) {
  *err = hipSuccess;
  const size_t b = round_size(std::max<size_t>(bytes, 1));
  HostPool& H = hpool();
  {
    std::lock_guard<std::mutex> lk(H.mu);
    auto it = H.free_.lower_bound(b);
    if (it != H.free_.end() && it->first <= 4 * b) {
      void* p = it->second;
      *got = it->first;
      H.cached -= it->first;
      H.free_.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *err = e;
    return nullptr;
  }
  *got = b;
  return p;
}

void pinned_free(void* p, size_t bytes) {
  if (!p) return;
  HostPool& H = hpool();
  std::lock_guard<std::mutex> lk(H.mu);
  if (H.cached + bytes > H.limit) {
    (void)hipHostFree(p);
    return;
  }
  H.free_.emplace(bytes, p);
  H.cached += bytes;
}

void pool_query(int64_t* hits, int64_t* misses, int64_t* cached, int64_t* live, int64_t* limit) {
  DevicePool& P = dpool();
  std::lock_guard<std::mutex> lk(P.mu);
  *hits = P.hits;
  *misses = P.misses;
  *cached = (int64_t)P.cached;
  *live = (int64_t)P.live;
  *limit = (int64_t)P.limit;
}

void pool_trim() {
  DevicePool& P = dpool();
  std::lock_guard<std::mutex> lk(P.mu);
  release_cached(P, -1);
}

void pool_set_limit(size_t bytes) {
  DevicePool& P = dpool();
  std::lock_guard<std::mutex> lk(P.mu);
  P.limit = bytes;
  if (P.cached > P.limit) release_cached(P, -1);
}

// One non-blocking stream per host thread and device for the library's own synchronous work
// (scene packing), so that it neither waits for nor blocks other streams.
namespace {
struct ThreadStreams {
  std::vector<hipStream_t> s;
  ~ThreadStreams() {
    for (hipStream_t x : s)
      if (x) (void)hipStreamDestroy(x);
  }
};
}  // namespace

hipStream_t private_stream(hipError_t* err) {
  thread_local ThreadStreams ts;
  std::vector<hipStream_t>& streams = ts.s;
  *err = hipSuccess;
  int dev = 0;
  (void)hipGetDevice(&dev);
  if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
  if (!streams[dev]) {
    hipError_t e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *err = e;
      streams[dev] = nullptr;
      return nullptr;
    }
  }
  return streams[dev];
}

// The block size pool_alloc takes from HIP for a request of `bytes` (what a fresh allocation costs).
size_t pool_block_size(size_t bytes) { return round_size(std::max<size_t>(bytes, 1)); }

}  // namespace mfs
