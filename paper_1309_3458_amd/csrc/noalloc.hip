// The match without allocation, for callers that cannot allocate device
// memory (code under stream capture, tight serving loops): the plain
// count -> scan -> fill path of ddm_match with every piece of scratch carved
// from one static device array.
//
// Each device that runs the entry point holds its own copy of the array
// (DDM_NOALLOC_SCRATCH_MB MiB) until the process ends.  The array's name in
// host code is a host-side stand-in, not a device address: its address on
// the current device is looked up once per device with hipGetSymbolAddress,
// and only that address reaches kernels.  Every call on a device shares the
// device's array: calls that overlap on one device (on different streams or
// from different threads) race.  The match's kernels set every counter they
// read before they read it, so nothing is left over from the previous call.
#include "ddm_internal.h"

#include <mutex>

namespace ddm {

constexpr size_t kNoAllocScratchBytes = size_t(DDM_NOALLOC_SCRATCH_MB) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
struct DeviceScratch {
  std::once_flag once;
  char* ptr = nullptr;
  hipError_t err = hipSuccess;
};
DeviceScratch g_scratch[kMaxDevices];
}  // namespace

// the array's address on the current device (looked up on first use there)
static ddm_status device_scratch(char** out) {
  int dev = -1;
  DDM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_detail("ddm_match_noalloc: device index beyond the scratch table");
    return DDM_E_INVALID_ARG;
  }
  DeviceScratch& slot = g_scratch[dev];
  std::call_once(slot.once, [&slot] {
    void* p = nullptr;
    slot.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (slot.err == hipSuccess) slot.ptr = static_cast<char*>(p);
  });
  if (slot.err != hipSuccess)
    return hip_fail(slot.err, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
  if (!slot.ptr) {
    set_detail("ddm_match_noalloc: no device address for the static scratch");
    return DDM_E_DEVICE;
  }
  *out = slot.ptr;
  return DDM_OK;
}

}  // namespace ddm

using namespace ddm;

extern "C" ddm_status ddm_match_noalloc(const ddm_tree* t, const float* upd_lo,
                                        const float* upd_hi, uint32_t m, uint64_t* out_pairs,
                                        uint64_t capacity, uint64_t* out_count, void* stream) {
  set_detail("");
  if (out_count) *out_count = 0;
  if (!t) {
    set_detail("tree is NULL");
    return DDM_E_INVALID_ARG;
  }
  char* base = nullptr;
  ddm_status r = device_scratch(&base);
  if (r != DDM_OK) return r;
  return match_external_scratch(t, upd_lo, upd_hi, m, out_pairs, capacity, out_count,
                                (hipStream_t)stream, base, kNoAllocScratchBytes,
                                "ddm_match_noalloc");
}
