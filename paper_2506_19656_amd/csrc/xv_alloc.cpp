// xv_alloc.cpp -- caching device allocator of libxv.
//
// Every device buffer of the library (encoded cubes, coding work buffers,
// decode buffers) comes from here.  A freed block is not returned to the
// runtime: it is kept with the stream it was last used on and an event
// recorded on that stream at the free.  A later allocation on the same
// stream may take it at once (stream order makes the old work finish first);
// an allocation on another stream takes it only once that event has
// completed.  hipMalloc runs only when no cached block fits, and hipFree only
// when an allocation fails for lack of memory or on xv_cache_release.  This
// keeps both runtime calls off the per-request path, where the stream-ordered
// pool of the runtime costs hundreds of microseconds of host time per free.
//
// Size classes: requests are rounded up to a power of two below 1 MiB and to
// a multiple of 2 MiB above; a cached block is reused for a request of at
// least four fifths of its size, so a reused block wastes at most a quarter
// of the request.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "xv_internal.h"

namespace xv {
namespace {

struct Cached {
  void* p;
  size_t bytes;
  int dev;
  hipStream_t stream;  // stream of the last use; kNoStream once retired
  hipEvent_t ev;       // recorded on that stream at the free
};

struct Live {
  size_t bytes;
  int dev;
};

const hipStream_t kNoStream = reinterpret_cast<hipStream_t>(~(uintptr_t)0);

std::mutex g_mu;
std::multimap<size_t, Cached> g_free;      // by size
std::unordered_map<void*, Live> g_live;    // handed out
std::vector<hipEvent_t> g_events;          // idle events for reuse
size_t g_cached_bytes = 0, g_live_bytes = 0, g_peak_bytes = 0;

size_t round_size(size_t n) {
  if (n == 0) n = 1;
  if (n < (1u << 20)) {
    size_t r = 512;
    while (r < n) r <<= 1;
    return r;
  }
  const size_t g = 2u << 20;
  return (n + g - 1) / g * g;
}

hipEvent_t take_event() {
  if (!g_events.empty()) {
    hipEvent_t e = g_events.back();
    g_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Releases cached blocks back to the runtime.  With wait, blocks whose last
// use has not completed are waited for; without, they are kept.
size_t release_locked(bool wait) {
  size_t freed = 0;
  for (auto it = g_free.begin(); it != g_free.end();) {
    Cached& c = it->second;
    bool done = !c.ev || hipEventQuery(c.ev) == hipSuccess;
    if (!done && wait) done = hipEventSynchronize(c.ev) == hipSuccess;
    if (!done) {
      ++it;
      continue;
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != c.dev) (void)hipSetDevice(c.dev);
    (void)hipFree(c.p);
    if (cur != c.dev) (void)hipSetDevice(cur);
    if (c.ev) g_events.push_back(c.ev);
    freed += c.bytes;
    g_cached_bytes -= c.bytes;
    it = g_free.erase(it);
  }
  return freed;
}

}  // namespace

hipError_t dev_alloc(void** out, size_t bytes, hipStream_t s) {
  *out = nullptr;
  const size_t want = round_size(bytes);
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return he;
  std::lock_guard<std::mutex> lk(g_mu);
  // best fit among blocks no more than a quarter larger than the request
  const size_t limit = want + want / 4;
  for (auto it = g_free.lower_bound(want); it != g_free.end() && it->first <= limit; ++it) {
    Cached& c = it->second;
    if (c.dev != dev) continue;
    if (c.stream != s && c.ev && hipEventQuery(c.ev) != hipSuccess) continue;
    *out = c.p;
    g_live[c.p] = Live{c.bytes, dev};
    g_cached_bytes -= c.bytes;
    g_live_bytes += c.bytes;
    if (g_live_bytes > g_peak_bytes) g_peak_bytes = g_live_bytes;
    if (c.ev) g_events.push_back(c.ev);
    g_free.erase(it);
    return hipSuccess;
  }
  he = hipMalloc(out, want);
  if (he == hipErrorOutOfMemory || he == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    release_locked(false);
    he = hipMalloc(out, want);
    if (he == hipErrorOutOfMemory || he == hipErrorMemoryAllocation) {
      (void)hipGetLastError();
      release_locked(true);
      he = hipMalloc(out, want);
    }
  }
  if (he != hipSuccess) {
    *out = nullptr;
    return he;
  }
  g_live[*out] = Live{want, dev};
  g_live_bytes += want;
  if (g_live_bytes > g_peak_bytes) g_peak_bytes = g_live_bytes;
  return hipSuccess;
}

void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) return;  // not ours: ignore rather than corrupt the cache
  const Live l = it->second;
  g_live.erase(it);
  g_live_bytes -= l.bytes;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != l.dev) (void)hipSetDevice(l.dev);
  hipEvent_t ev = take_event();
  if (ev && hipEventRecord(ev, s) != hipSuccess) {
    (void)hipGetLastError();
    // without an event the block can only be reused after a full wait
    (void)hipStreamSynchronize(s);
    g_events.push_back(ev);
    ev = nullptr;
  }
  if (cur != l.dev) (void)hipSetDevice(cur);
  g_free.emplace(l.bytes, Cached{p, l.bytes, l.dev, s, ev});
  g_cached_bytes += l.bytes;
}

void dev_stream_retired(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_free)
    if (kv.second.stream == s) kv.second.stream = kNoStream;
}

size_t dev_cache_release() {
  std::lock_guard<std::mutex> lk(g_mu);
  return release_locked(true);
}

void dev_cache_stats(size_t* live, size_t* cached, size_t* peak) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (live) *live = g_live_bytes;
  if (cached) *cached = g_cached_bytes;
  if (peak) *peak = g_peak_bytes;
}

}  // namespace xv
