// Library plumbing: error details, status strings, stream-ordered scratch,
// and per-kernel timing with HIP events.
#include "ddm_internal.h"

#include <cstdio>
#include <cstring>
#include <map>
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

// Keep memory released by hipFreeAsync in the device's default pool instead
// of returning it to the driver, so repeated builds and matches reuse it.
void ensure_pool(int device) {
  static std::mutex mu;
  static std::set<int> done;
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(device)) return;
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
    uint64_t thr = ~0ull;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  (void)hipGetLastError();
  done.insert(device);
}

Scratch::~Scratch() {
  if (base_) (void)hipFreeAsync(base_, s_);
}

bool Scratch::commit() {
  if (want_ == 0) want_ = 256;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) ensure_pool(dev);
  void* p = nullptr;
  hipError_t e = hipMallocAsync(&p, want_, s_);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    set_detail("device scratch allocation failed");
    return false;
  }
  base_ = (char*)p;
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
