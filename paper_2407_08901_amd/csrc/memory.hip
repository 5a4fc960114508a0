// memory.hip - device and pinned host memory of the library.
//
// Every device buffer of the library (context arrays, setup temporaries) comes from a
// process-wide cache.  A freed block stays mapped and goes back to the next request of the same
// rounded size on the same device, so repeated setups of one problem size call hipMalloc and
// hipFree only the first time.  Both calls stall the host (hipFree also waits for the whole
// device), and a block of recently freed VRAM is cleared by the driver before hipMalloc returns
// it, which costs about a second per 100 GB.
//
// Reuse is ordered by the callers: a block goes back to the cache only after the stream that
// last used it has been synchronised.  The cache holds at most 3/4 of the device's memory; a
// block beyond that is freed at once, and a hipMalloc that runs out of memory empties the cache
// of its device and tries once more.  sppc_release_cached_memory() empties it on demand.
#include "common.h"

#include <map>
#include <mutex>
#include <tuple>
#include <unordered_map>
#include <vector>

namespace sppc {

namespace {

struct Block {
  size_t size;
  int dev;
  bool host;
};

std::mutex g_mu;
std::unordered_map<void*, Block> g_live;                        // handed out
std::multimap<std::tuple<int, bool, size_t>, void*> g_cache;   // (device, host, size) -> block
std::map<int, size_t> g_cached;  // cached bytes per device
std::map<int, size_t> g_cap;  // per device

size_t rounded(size_t bytes) {
  const size_t g = bytes >= ((size_t)1 << 20) ? ((size_t)2 << 20) : (size_t)512;
  return (std::max<size_t>(bytes, 1) + g - 1) / g * g;
}

size_t cap_of(int dev) {  // called with g_mu held and dev current on the first call
  auto it = g_cap.find(dev);
  if (it != g_cap.end()) return it->second;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    tot = 0;
  }
  return g_cap[dev] = tot / 4 * 3;
}

void release_raw(void* p, bool host) {
  if (host) (void)hipHostFree(p); else (void)hipFree(p);
}

// frees every cached block of one device (dev < 0: of all devices); returns the bytes freed
size_t trim(int dev) {
  std::vector<std::pair<void*, bool>> out;
  size_t bytes = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
      if (dev < 0 || std::get<0>(it->first) == dev) {
        out.push_back({it->second, std::get<1>(it->first)});
        bytes += std::get<2>(it->first);
        g_cached[std::get<0>(it->first)] -= std::get<2>(it->first);
        it = g_cache.erase(it);
      } else {
        ++it;
      }
    }
  }
  for (auto& b : out) release_raw(b.first, b.second);
  return bytes;
}

hipError_t take(void** out, size_t bytes, bool host) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t sz = rounded(bytes);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    (void)cap_of(dev);
    auto it = g_cache.find(std::make_tuple(dev, host, sz));
    if (it != g_cache.end()) {
      *out = it->second;
      g_cache.erase(it);
      g_cached[dev] -= sz;
      g_live[*out] = Block{sz, dev, host};
      return hipSuccess;
    }
  }
  void* p = nullptr;
  e = host ? hipHostMalloc(&p, sz, hipHostMallocDefault) : hipMalloc(&p, sz);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    if (trim(dev) > 0) e = host ? hipHostMalloc(&p, sz, hipHostMallocDefault) : hipMalloc(&p, sz);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_live[p] = Block{sz, dev, host};
  *out = p;
  return hipSuccess;
}

void give_back(void* p) {
  if (!p) return;
  bool free_now = false, host = false;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;  // not from this cache
    const Block b = it->second;
    g_live.erase(it);
    host = b.host;
    if (g_cached[b.dev] + b.size > cap_of(b.dev)) {
      free_now = true;
    } else {
      g_cache.insert({std::make_tuple(b.dev, b.host, b.size), p});
      g_cached[b.dev] += b.size;
    }
  }
  if (free_now) release_raw(p, host);
}

}  // namespace

hipError_t dev_alloc(void** p, size_t bytes) { return take(p, bytes, false); }
void dev_free(void* p) { give_back(p); }
hipError_t pinned_alloc(void** p, size_t bytes) { return take(p, bytes, true); }
void pinned_free(void* p) { give_back(p); }
size_t release_cached(void) { return trim(-1); }

}  // namespace sppc

extern "C" size_t sppc_release_cached_memory(void) { return sppc::release_cached(); }
