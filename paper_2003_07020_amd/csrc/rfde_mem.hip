// Device-memory cache for plan and batch buffers.  Mapping fresh device memory costs roughly
// 10-20 ms per GB here (measured: a 70 GB plan spent 1-2 s in allocation when the memory was not
// already mapped, 2 ms when it was), which would dominate the setup of every plan.  Freed
// blocks are therefore kept per device and handed out again for a request of at most their size
// and at least three quarters of it.  A failed hipMalloc releases the cache and retries once;
// rfde_release_cached_memory() releases it on demand.
#include <map>
#include <mutex>

#include "rfde_internal.hpp"

namespace rfde {
namespace {

struct Block {
  size_t bytes;
  int device;
};

std::mutex g_mu;
std::map<void*, Block> g_live;                      // handed out
std::multimap<size_t, std::pair<void*, int>> g_free;  // cached: size -> (pointer, device)

size_t round_size(size_t b) {
  const size_t q = b >= ((size_t)1 << 20) ? ((size_t)2 << 20) : 256;
  return (b + q - 1) / q * q;
}

size_t release_locked(int device) {  // device < 0: every device
  size_t n = 0;
  for (auto it = g_free.begin(); it != g_free.end();) {
    if (device < 0 || it->second.second == device) {
      (void)hipFree(it->second.first);
      n += it->first;
      it = g_free.erase(it);
    } else {
      ++it;
    }
  }
  return n;
}

}  // namespace

int dev_alloc(void** ptr, size_t bytes) {
  int dev = 0;
  RFDE_HIP(hipGetDevice(&dev));
  const size_t want = round_size(bytes == 0 ? 1 : bytes);
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto it = g_free.lower_bound(want); it != g_free.end() && it->first <= want + want / 3;
       ++it) {
    if (it->second.second != dev) continue;
    *ptr = it->second.first;
    g_live[*ptr] = Block{it->first, dev};
    g_free.erase(it);
    return RFDE_OK;
  }
  hipError_t e = hipMalloc(ptr, want);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    release_locked(dev);
    e = hipMalloc(ptr, want);
  }
  if (e != hipSuccess) {
    *ptr = nullptr;
    return hip_fail(e, "hipMalloc", __FILE__, __LINE__);
  }
  g_live[*ptr] = Block{want, dev};
  return RFDE_OK;
}

void dev_free(void* ptr) {
  if (!ptr) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_live.find(ptr);
  if (it == g_live.end()) {
    (void)hipFree(ptr);
    return;
  }
  g_free.emplace(it->second.bytes, std::make_pair(ptr, it->second.device));
  g_live.erase(it);
}

size_t dev_cached_bytes(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  size_t n = 0;
  for (const auto& kv : g_free)
    if (kv.second.second == device) n += kv.first;
  return n;
}

}  // namespace rfde

extern "C" size_t rfde_release_cached_memory(void) {
  std::lock_guard<std::mutex> lk(rfde::g_mu);
  return rfde::release_locked(-1);
}
