// memory.hip - device and pinned host memory of the library.
//
// Device memory comes from one of two places:
//   * a caller's workspace (sppc_setup with a workspace): every device array of the context, its
//     setup temporaries included, is carved from that block.  Persistent arrays grow from its
//     bottom and setup temporaries from its top; a freed block is returned when it is the last one
//     of its end (freed blocks below it are returned with it), so the bytes sppc_workspace_size
//     adds up (the persistent arrays plus the largest set of temporaries alive at once) suffice.
//   * the library itself: hipMalloc on request and hipFree when the array is given back.  An
//     optional process-wide cache (sppc_set_memory_cache) keeps freed blocks for the next request
//     of the same rounded size on the same device instead: hipMalloc/hipFree stall the host
//     (hipFree also waits for the whole device) and recently freed VRAM is cleared by the driver
//     before it is handed out again.  The cache is off unless enabled; a block goes back to it
//     only after the stream that last used it has been synchronised.
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
size_t g_cache_limit = 0;     // bytes per device the cache may keep (0: no cache)

size_t rounded(size_t bytes) {
  const size_t g = bytes >= ((size_t)1 << 20) ? ((size_t)2 << 20) : (size_t)512;
  return (std::max<size_t>(bytes, 1) + g - 1) / g * g;
}

size_t cap_of(int dev) {  // called with g_mu held and dev current on the first call
  if (g_cache_limit == 0) return 0;
  auto it = g_cap.find(dev);
  if (it != g_cap.end()) return std::min(it->second, g_cache_limit);
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    tot = 0;
  }
  return std::min(g_cap[dev] = tot / 4 * 3, g_cache_limit);
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

// ---------------------------------------------------------------- caller workspace
struct Workspace {
  struct Blk {
    size_t off, size;
    bool freed;
  };
  char* base = nullptr;
  size_t size = 0;
  size_t lo = 0;    // bottom end in use: [0, lo)
  size_t hi = 0;    // top end in use: [hi, size)
  size_t peak = 0;  // largest lo + (size - hi) seen
  std::vector<Blk> bottom, top;

  static size_t al(size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; }
  void* alloc(size_t bytes, bool temp) {
    const size_t b = al(bytes);
    if (b > hi - lo) return nullptr;
    size_t off;
    if (temp) {
      hi -= b;
      off = hi;
      top.push_back({off, b, false});
    } else {
      off = lo;
      lo += b;
      bottom.push_back({off, b, false});
    }
    peak = std::max(peak, lo + (size - hi));
    return base + off;
  }
  bool owns(const void* p) const { return p >= (const void*)base && p < (const void*)(base + size); }
  void release(void* p) {
    const size_t off = (size_t)((char*)p - base);
    for (auto* v : {&bottom, &top})
      for (auto& bk : *v)
        if (bk.off == off && !bk.freed) {
          bk.freed = true;
          while (!bottom.empty() && bottom.back().freed) {
            lo = bottom.back().off;
            bottom.pop_back();
          }
          while (!top.empty() && top.back().freed) {
            hi = top.back().off + top.back().size;
            top.pop_back();
          }
          return;
        }
  }
};

namespace {
thread_local Workspace* t_ws = nullptr;  // the workspace of the context an entry point works on
}

Workspace* ws_create(void* base, size_t bytes) {
  Workspace* w = new Workspace();
  const uintptr_t a = ((uintptr_t)base + 255) & ~(uintptr_t)255;  // 256-byte aligned start
  w->base = (char*)a;
  w->size = bytes > (size_t)(a - (uintptr_t)base) ? (bytes - (size_t)(a - (uintptr_t)base)) / 256 * 256 : 0;
  w->lo = 0;
  w->hi = w->size;
  return w;
}
void ws_destroy(Workspace* w) { delete w; }
size_t ws_peak(const Workspace* w) { return w ? w->peak : 0; }
WsScope::WsScope(Workspace* w) : prev(t_ws) { t_ws = w; }
WsScope::~WsScope() { t_ws = prev; }

static hipError_t ws_take(void** p, size_t bytes, bool temp) {
  *p = t_ws->alloc(bytes, temp);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t dev_alloc(void** p, size_t bytes) { return t_ws ? ws_take(p, bytes, false) : take(p, bytes, false); }
hipError_t dev_alloc_tmp(void** p, size_t bytes) { return t_ws ? ws_take(p, bytes, true) : take(p, bytes, false); }
void dev_free(void* p) {
  if (!p) return;
  if (t_ws && t_ws->owns(p)) {
    t_ws->release(p);
    return;
  }
  give_back(p);
}
hipError_t pinned_alloc(void** p, size_t bytes) { return take(p, bytes, true); }
void pinned_free(void* p) { give_back(p); }
size_t release_cached(void) { return trim(-1); }

}  // namespace sppc

extern "C" size_t sppc_release_cached_memory(void) { return sppc::release_cached(); }

extern "C" size_t sppc_set_memory_cache(size_t bytes_per_device) {
  size_t prev;
  {
    std::lock_guard<std::mutex> lk(sppc::g_mu);
    prev = sppc::g_cache_limit;
    sppc::g_cache_limit = bytes_per_device;
  }
  if (bytes_per_device == 0) sppc::release_cached();
  return prev;
}
