// Library plumbing: error details, status strings, stream-ordered scratch,
// and per-kernel timing with HIP events.
#include "ddm_internal.h"

#include <cstdio>
#include <cstring>
#include <map>
#include <unordered_map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

namespace ddm {

static thread_local std::string g_detail;

void set_detail(const std::string& s) { g_detail = s; }

ddm_status hip_fail(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  g_detail = buf;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return DDM_E_NOMEM;
  return DDM_E_DEVICE;
}

// ---------------------------------------------------------------------------
// device memory cache
//
// Blocks come from hipMalloc and are cached when freed.  A freed block
// remembers the stream that freed it and an event recorded on that stream at
// the free: the same stream may reuse the block at once (stream order),
// another stream only once the event has completed.  Reuse is best fit
// among cached blocks at most 25% (+1 MiB) larger than asked; sizes above
// 1 MiB are rounded up to one of 8 steps per power of two so that requests
// of similar size share blocks.  The cached bytes are bounded: beyond
// kCacheLimit, the largest cached blocks whose last use has completed are
// returned to the driver.
// ---------------------------------------------------------------------------
struct CachedBlock {
  char* p;
  size_t size;
  hipStream_t s;
  hipEvent_t ev;
  int dev;
};

static std::mutex g_mem_mu;
static std::multimap<size_t, CachedBlock>* g_free = new std::multimap<size_t, CachedBlock>();
static std::map<char*, std::pair<size_t, int>>* g_live = new std::map<char*, std::pair<size_t, int>>();
static std::vector<hipEvent_t>* g_events = new std::vector<hipEvent_t>();

// events without timing, from a pool (creating one per use is slow)
hipEvent_t pooled_event() {
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    if (!g_events->empty()) {
      hipEvent_t e = g_events->back();
      g_events->pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void release_event(hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_events->push_back(e);
}

static size_t round_bytes(size_t b) {
  if (b <= (1u << 20)) return (b + 255) & ~size_t(255);
  // (8 + i) * 2^(e-3), i < 8: at most 12.5% above the request
  int e = 63 - __builtin_clzll((unsigned long long)b);
  const size_t step = size_t(1) << (e - 3);
  return (b + step - 1) & ~(step - 1);
}

// about a fifth of one GPU's 288 GB of HBM: the slot arena of a large
// learned match (tens of GB) stays cached from one step to the next instead
// of going back to the driver and being mapped again (seconds at that size);
// an allocation that fails gives the cache back and retries
constexpr size_t kCacheLimit = size_t(64) << 30;
static size_t g_cached = 0;  // bytes in g_free
// bytes handed out by dev_alloc and not yet freed, and the test hook's cap
// on them (0: none), beyond which dev_alloc fails as the driver's would
static size_t g_live_bytes = 0;
static size_t g_alloc_cap = 0;

// Frees cached blocks, largest first, whose last use has completed, until
// the cache is within its limit.  Called with g_mem_mu held; returns the
// blocks to free outside the lock.
static void trim_cache(std::vector<CachedBlock>* out) {
  for (auto it = g_free->end(); g_cached > kCacheLimit && it != g_free->begin();) {
    --it;
    CachedBlock& b = it->second;
    bool idle = false;
    if (b.ev) {
      const hipError_t q = hipEventQuery(b.ev);
      idle = q == hipSuccess;
      if (q != hipSuccess && q != hipErrorNotReady) (void)hipGetLastError();
    }
    if (!idle) continue;
    out->push_back(b);
    g_cached -= b.size;
    it = g_free->erase(it);
  }
}

char* dev_alloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 256;
  bytes = round_bytes(bytes);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    if (g_alloc_cap && g_live_bytes + bytes > g_alloc_cap) return nullptr;
    const size_t cap = bytes + bytes / 4 + (1u << 20);
    for (auto it = g_free->lower_bound(bytes); it != g_free->end() && it->first <= cap; ++it) {
      CachedBlock& b = it->second;
      if (b.dev != dev) continue;
      bool ok = b.s == s;
      if (!ok && b.ev) {
        const hipError_t q = hipEventQuery(b.ev);
        ok = q == hipSuccess;
        if (q != hipSuccess && q != hipErrorNotReady) (void)hipGetLastError();
      }
      if (!ok) continue;
      char* p = b.p;
      const size_t sz = b.size;
      if (b.ev) g_events->push_back(b.ev);
      g_cached -= sz;
      g_free->erase(it);
      (*g_live)[p] = {sz, dev};
      g_live_bytes += sz;
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // give the cached blocks of this device back to the driver and retry
    std::vector<CachedBlock> drop;
    {
      std::lock_guard<std::mutex> lk(g_mem_mu);
      for (auto it = g_free->begin(); it != g_free->end();) {
        if (it->second.dev == dev) {
          drop.push_back(it->second);
          g_cached -= it->second.size;
          it = g_free->erase(it);
        } else {
          ++it;
        }
      }
    }
    (void)hipDeviceSynchronize();
    for (auto& b : drop) {
      (void)hipFree(b.p);
      release_event(b.ev);
    }
    (void)hipGetLastError();
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  std::lock_guard<std::mutex> lk(g_mem_mu);
  (*g_live)[(char*)p] = {bytes, dev};
  g_live_bytes += bytes;
  return (char*)p;
}

void dev_free(char* p, hipStream_t s) {
  if (!p) return;
  size_t sz = 0;
  int dev = 0;
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_live->find(p);
    if (it == g_live->end()) return;
    sz = it->second.first;
    dev = it->second.second;
    g_live->erase(it);
    g_live_bytes -= sz;
  }
  hipEvent_t ev = pooled_event();
  if (ev) (void)hipEventRecord(ev, s);
  // without an event only the freeing stream may reuse the block
  std::vector<CachedBlock> drop;
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_free->insert({sz, CachedBlock{p, sz, s, ev, dev}});
    g_cached += sz;
    if (g_cached > kCacheLimit) trim_cache(&drop);
  }
  if (drop.empty()) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& b : drop) {
    if (b.dev != cur) (void)hipSetDevice(b.dev);
    (void)hipFree(b.p);
    if (b.dev != cur) (void)hipSetDevice(cur);
    release_event(b.ev);
  }
  (void)hipGetLastError();
}

ddm_status scratch_overrun(const char* where) {
  set_detail(std::string(where) + ": scratch takes exceed the reserved block");
  return DDM_E_DEVICE;
}

Scratch::~Scratch() {
  if (base_ && !ext_ && !dry_) dev_free(base_, s_);
}

bool Scratch::commit() {
  if (want_ == 0) want_ = 256;
  if (dry_) {
    base_ = reinterpret_cast<char*>(uintptr_t(1) << 40);
    used_ = 0;
    return true;
  }
  if (ext_) {
    if (want_ > ext_cap_) {
      set_detail("scratch needs " + std::to_string(want_) + " bytes, the fixed scratch holds " +
                 std::to_string(ext_cap_));
      return false;
    }
    base_ = ext_;
    used_ = 0;
    return true;
  }
  base_ = dev_alloc(want_, s_);
  if (!base_) {
    set_detail("device scratch allocation failed");
    return false;
  }
  used_ = 0;
  return true;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
static thread_local bool g_prof_on = false;
static thread_local std::string g_prof_focus;  // empty: record every kernel
static thread_local std::vector<ProfRec> g_prof;
static thread_local std::vector<hipEvent_t> g_free_events;
static thread_local std::map<std::string, std::pair<double, uint64_t>> g_prof_acc;

static hipEvent_t get_event() {
  if (!g_free_events.empty()) {
    hipEvent_t e = g_free_events.back();
    g_free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

ProfScope::ProfScope(const char* name, hipStream_t s) : name_(name), s_(s) {
  ev_[0] = ev_[1] = nullptr;
  if (!g_prof_on) return;
  if (!g_prof_focus.empty() && g_prof_focus != name) return;
  // events recorded during graph capture would become graph nodes
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return;
  }
  hipEvent_t a = get_event();
  if (!a) return;
  ev_[0] = a;
  (void)hipEventRecord(a, s);
}

ProfScope::~ProfScope() {
  if (!ev_[0]) return;
  hipEvent_t b = get_event();
  if (!b) return;
  (void)hipEventRecord(b, s_);
  g_prof.push_back(ProfRec{name_, (hipEvent_t)ev_[0], b});
}

static void prof_collect() {
  for (auto& r : g_prof) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& acc = g_prof_acc[r.name];
      acc.first += ms;
      acc.second += 1;
    }
    (void)hipGetLastError();
    g_free_events.push_back(r.a);
    g_free_events.push_back(r.b);
  }
  g_prof.clear();
}

}  // namespace ddm

using namespace ddm;

extern "C" const char* ddm_strerror(ddm_status s) {
  switch (s) {
    case DDM_OK: return "success";
    case DDM_E_INVALID_ARG: return "invalid argument";
    case DDM_E_INVALID_INPUT: return "invalid input coordinates (NaN/inf or lo > hi)";
    case DDM_E_CAPACITY: return "output capacity too small";
    case DDM_E_NOMEM: return "out of memory";
    case DDM_E_DEVICE: return "HIP runtime error";
  }
  return "unknown status";
}

extern "C" const char* ddm_last_error_detail(void) { return g_detail.c_str(); }

extern "C" uint64_t ddm_debug_alloc_cap(uint64_t bytes) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_alloc_cap = (size_t)bytes;
  return g_live_bytes;
}

extern "C" void ddm_prof_enable(int on) {
  if (!on) prof_collect();
  g_prof_on = on != 0;
}

extern "C" void ddm_prof_focus(const char* name) { g_prof_focus = name ? name : ""; }

extern "C" uint64_t ddm_prof_read(char* buf, uint64_t size) {
  prof_collect();
  std::string js = "{";
  bool first = true;
  for (auto& kv : g_prof_acc) {
    char item[256];
    snprintf(item, sizeof(item), "%s\"%s\": [%.6f, %llu]", first ? "" : ", ", kv.first.c_str(),
             kv.second.first, (unsigned long long)kv.second.second);
    js += item;
    first = false;
  }
  js += "}";
  g_prof_acc.clear();
  if (buf && size) {
    size_t c = js.size() < size - 1 ? js.size() : (size_t)(size - 1);
    memcpy(buf, js.data(), c);
    buf[c] = 0;
  }
  return js.size();
}
