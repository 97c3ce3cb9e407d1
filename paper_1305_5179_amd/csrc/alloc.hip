// Device memory of the library: a caching allocator.
//
// hipMallocAsync / hipFreeAsync cost tens to hundreds of microseconds per
// call on this platform, and a setup or a solve makes dozens of them, so
// blocks are kept by the library once allocated and handed out again:
//   * a block freed during an API call (stream-ordered, the call's kernels
//     may still be queued) goes back to the free list of (device, stream)
//     and is reused only by later allocations on that same stream, which
//     run after every use enqueued before the free;
//   * a block freed after a device-wide synchronisation (rbf_destroy) goes
//     to the device's list for any stream.
// A miss calls hipMalloc; when that fails for lack of memory the device is
// synchronised, every cached block of it is returned to HIP and the
// allocation is tried once more.  Cached memory otherwise stays with the
// library until the process ends.
#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>

#include "common.h"

namespace rbf {

namespace {

struct Live {
  int dev;
  size_t bytes;
};

struct Cache {
  std::mutex mu;
  std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void*>> per_stream;
  std::map<int, std::multimap<size_t, void*>> any_stream;
  std::unordered_map<void*, Live> live;
};

Cache& cache() {
  static Cache* c = new Cache();   // never destroyed: blocks outlive static destructors
  return *c;
}

// Size classes: 512-byte steps below 1 MiB, 2 MiB steps above.
size_t size_class(size_t bytes) {
  if (bytes == 0) bytes = 1;
  const size_t step = bytes < (size_t(1) << 20) ? 512 : (size_t(2) << 20);
  return (bytes + step - 1) / step * step;
}

// Best fit no larger than 5/4 of the request (twice for small blocks).
void* take(std::multimap<size_t, void*>& m, size_t bytes) {
  auto it = m.lower_bound(bytes);
  const size_t limit = bytes < (size_t(1) << 20) ? 2 * bytes : bytes + bytes / 4;
  if (it == m.end() || it->first > limit) return nullptr;
  void* p = it->second;
  m.erase(it);
  return p;
}

thread_local bool t_synced_release = false;

}  // namespace

hipStream_t& temp_stream() {
  static thread_local hipStream_t s = nullptr;
  return s;
}

SyncedRelease::SyncedRelease() : prev(t_synced_release) { t_synced_release = true; }
SyncedRelease::~SyncedRelease() { t_synced_release = prev; }

void* temp_alloc_bytes(size_t bytes) {
  int dev = 0;
  RBF_HIP(hipGetDevice(&dev));
  const size_t sz = size_class(bytes);
  const hipStream_t s = temp_stream();
  Cache& c = cache();
  {
    std::lock_guard<std::mutex> lock(c.mu);
    void* p = nullptr;
    auto ps = c.per_stream.find({dev, s});
    if (ps != c.per_stream.end()) p = take(ps->second, sz);
    if (!p) {
      auto as = c.any_stream.find(dev);
      if (as != c.any_stream.end()) p = take(as->second, sz);
    }
    if (p) return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    // return every cached block of the device to HIP and try once more
    RBF_HIP(hipDeviceSynchronize());
    std::vector<void*> drop;
    {
      std::lock_guard<std::mutex> lock(c.mu);
      for (auto& kv : c.per_stream)
        if (kv.first.first == dev) {
          for (auto& b : kv.second) drop.push_back(b.second);
          kv.second.clear();
        }
      auto as = c.any_stream.find(dev);
      if (as != c.any_stream.end()) {
        for (auto& b : as->second) drop.push_back(b.second);
        as->second.clear();
      }
      for (void* q : drop) c.live.erase(q);
    }
    for (void* q : drop) (void)hipFree(q);
    e = hipMalloc(&p, sz);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error{e == hipErrorOutOfMemory ? RBF_ENOMEM : RBF_EDEVICE,
                std::string("hipMalloc(") + std::to_string(sz) + " bytes): " + hipGetErrorString(e)};
  }
  std::lock_guard<std::mutex> lock(c.mu);
  c.live[p] = Live{dev, sz};
  return p;
}

void temp_free(void* p) {
  if (!p) return;
  Cache& c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;   // not ours: nothing to do
  const Live b = it->second;
  if (t_synced_release)
    c.any_stream[b.dev].emplace(b.bytes, p);
  else
    c.per_stream[{b.dev, temp_stream()}].emplace(b.bytes, p);
}

}  // namespace rbf
