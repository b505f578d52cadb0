// Internal declarations shared by the libddm translation units (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>

#include "ddm.h"

namespace ddm {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
void set_detail(const std::string& s);
ddm_status hip_fail(hipError_t e, const char* what, const char* file, int line);

#define DDM_HIP(call)                                                        \
  do {                                                                       \
    hipError_t _e = (call);                                                  \
    if (_e != hipSuccess) return ::ddm::hip_fail(_e, #call, __FILE__, __LINE__); \
  } while (0)

#define DDM_LAUNCHED(name)                                                   \
  do {                                                                       \
    hipError_t _e = hipGetLastError();                                       \
    if (_e != hipSuccess) return ::ddm::hip_fail(_e, name, __FILE__, __LINE__); \
  } while (0)

// ---------------------------------------------------------------------------
// kernel timing (HIP events on the launching stream)
// ---------------------------------------------------------------------------
struct ProfScope {
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
  const char* name_;
  hipStream_t s_;
  void* ev_[2];
};

// ---------------------------------------------------------------------------
// stream-ordered scratch
// ---------------------------------------------------------------------------
struct Scratch {
  explicit Scratch(hipStream_t s) : s_(s) {}
  ~Scratch();
  // commit() returns false on failure (detail set); 256-byte aligned
  // sub-allocations are carved from one cached block by reserve()/take();
  // the block returns to the cache, ordered on the stream, at destruction.
  void reserve(size_t bytes) { want_ += (bytes + 255) & ~size_t(255); }
  bool commit();
  // Carve from caller-owned device memory instead (base 256-byte aligned,
  // `cap` bytes): commit() then fails, with the detail set, when the
  // reservations exceed `cap`, and nothing is freed at destruction.
  void use_external(char* base, size_t cap) {
    ext_ = base;
    ext_cap_ = cap;
  }
  // Host-only layout check: commit() at a fixed dummy address without any
  // memory behind it, so that take() and fits() can be exercised on a CPU.
  // The pointers handed out must never be dereferenced.
  void dry_run() { dry_ = true; }
  // Every take() must have its own reserve() of the same size, in any
  // order; fits() tells whether the takes so far stay inside the block and
  // must be checked before any kernel uses the memory.
  template <class T>
  T* take(size_t count) {
    size_t b = (count * sizeof(T) + 255) & ~size_t(255);
    char* p = base_ + used_;
    used_ += b;
    return reinterpret_cast<T*>(p);
  }
  bool fits() const { return used_ <= want_; }
  hipStream_t s_;
  char* base_ = nullptr;
  size_t want_ = 0, used_ = 0;
  char* ext_ = nullptr;
  size_t ext_cap_ = 0;
  bool dry_ = false;
};

// error for a scratch layout whose takes exceed its reservations (a
// programming error caught before any kernel touches the memory)
ddm_status scratch_overrun(const char* where);

// stream-aware device memory cache and event pool (api.hip)
char* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(char* p, hipStream_t s);
hipEvent_t pooled_event();
void release_event(hipEvent_t e);

// ---------------------------------------------------------------------------
// device-side data layout
// ---------------------------------------------------------------------------
// One radix-sort array (ping-pong buffers; v may be null for keys only).
struct SortArr {
  uint32_t* k[2];
  uint32_t* v[2];
  uint32_t n;
  uint32_t tile0;  // first tile of this array in the launch
};

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;  // 2048 keys per tile

// Per-dimension flat interval tree (positions 1..P, P = 2^H - 1 >= n).
//   rec[k]    (n+1) records of 2d floats; record p (1 <= p <= n) holds the
//             p-th segment in lower-bound order: lo_k, hi_k, then lo, hi of
//             every other dimension in increasing order.
//   maxhi[k]  P+1 floats, maxhi[k][p] = max upper bound in subtree(p).
//   id[k]     n+1 uint32, subscription id at position p.
//   skey_lo[k], skey_hi[k]: n sorted order-preserving keys of lo_k / hi_k.
//   bmax[k]   C = max(1, (P+1)/64) floats: bmax[k][c] = max upper bound over
//             positions 64c .. 64c+63 (position 64c and the height-5 subtree
//             rooted at 64c+32), the tree's augmentation cut at height 5.
//   maxlen[k] one float >= every (hi - lo) in dimension k.
struct TreeDev {
  const float* rec[DDM_MAX_D];
  const float* maxhi[DDM_MAX_D];
  const uint32_t* id[DDM_MAX_D];
  const uint32_t* skey_lo[DDM_MAX_D];
  const uint32_t* skey_hi[DDM_MAX_D];
  const float* bmax[DDM_MAX_D];
  const float* maxlen;
  // every 64th sorted key: sidx_lo[k][c] = skey_lo[k][64c], c < ns
  const uint32_t* sidx_lo[DDM_MAX_D];
  const uint32_t* sidx_hi[DDM_MAX_D];  // d == 1 only (upper bounds sorted)
  // kQuant quantiles of the sorted lower-bound keys: quant[k][i] =
  // skey_lo[k][floor(i n / kQuant)]
  const uint32_t* quant[DDM_MAX_D];
  uint32_t n, d, H, ns;
};

constexpr uint32_t kQuant = 4096;

constexpr uint32_t kBlockLog = 6;  // 64 positions per block of bmax

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
// Order-preserving map float32 -> uint32 (-0.0 is folded onto +0.0 so that
// key order equals float order, equalities included).
__device__ __forceinline__ uint32_t f2key(float f) {
  uint32_t b = __float_as_uint(f);
  if ((b & 0x7fffffffu) == 0u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ bool valid_extent(float lo, float hi) {
  return isfinite(lo) && isfinite(hi) && lo <= hi;
}

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of `mask` below this lane
__device__ __forceinline__ uint32_t mask_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// lanes of the wave whose 8-bit digit equals this lane's (restricted to `active`)
__device__ __forceinline__ uint64_t match_digit8(uint32_t dig, uint64_t active) {
  uint64_t peers = active;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    bool bit = (dig >> b) & 1u;
    uint64_t m = ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ float uniform_f32(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// first index in sorted keys[0..n) with keys[i] >= x
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ keys, uint32_t n,
                                                    uint32_t x) {
  uint32_t lo = 0, len = n;
  while (len > 0) {
    uint32_t half = len >> 1;
    if (keys[lo + half] < x) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo;
}

// first index in sorted keys[0..n) with keys[i] > x
__device__ __forceinline__ uint32_t upper_bound_u32(const uint32_t* __restrict__ keys, uint32_t n,
                                                    uint32_t x) {
  uint32_t lo = 0, len = n;
  while (len > 0) {
    uint32_t half = len >> 1;
    if (keys[lo + half] <= x) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo;
}

// Two-level searches over sorted keys[0..n) with samples idx[c] = keys[64c]
// (c < ns = ceil(n/64)): a binary search over the samples (small, cache
// resident) picks one 64-key window, a second one finishes inside it.
// number of keys <= x
__device__ __forceinline__ uint32_t upper_bound_2l(const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ idx, uint32_t n,
                                                   uint32_t ns, uint32_t x) {
  const uint32_t g = upper_bound_u32(idx, ns, x);
  if (g == 0) return 0;
  const uint32_t lo = (g - 1) << 6;
  const uint32_t hi = min(g << 6, n);
  return lo + 1 + upper_bound_u32(keys + lo + 1, hi - lo - 1, x);
}
// number of keys < x
__device__ __forceinline__ uint32_t lower_bound_2l(const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ idx, uint32_t n,
                                                   uint32_t ns, uint32_t x) {
  const uint32_t g = lower_bound_u32(idx, ns, x);
  if (g == 0) return 0;
  const uint32_t lo = (g - 1) << 6;
  const uint32_t hi = min(g << 6, n);
  return lo + 1 + lower_bound_u32(keys + lo + 1, hi - lo - 1, x);
}

// NS independent two-level counts run in lockstep, so that the loads of the
// different searches overlap: res[i] = #{keys_i < x_i} (upper[i] false) or
// #{keys_i <= x_i} (upper[i] true).  Binary lifting with a trip count fixed
// by ns keeps all searches on the same step.
template <int NS>
__device__ __forceinline__ void count_2l(const uint32_t* const (&keys)[NS],
                                         const uint32_t* const (&idx)[NS],
                                         const uint32_t (&x)[NS], const bool (&upper)[NS],
                                         uint32_t n, uint32_t ns, uint32_t (&res)[NS]) {
  uint32_t g[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) g[i] = 0;
  uint32_t top = 1;
  while ((top << 1) <= ns) top <<= 1;
  for (uint32_t step = top; step > 0; step >>= 1) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const uint32_t c = g[i] + step;
      if (c <= ns) {
        const uint32_t v = idx[i][c - 1];
        if (upper[i] ? (v <= x[i]) : (v < x[i])) g[i] = c;
      }
    }
  }
  uint32_t lo[NS], w[NS], pos[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    lo[i] = g[i] ? ((g[i] - 1) << 6) : 0u;
    const uint32_t hi = g[i] ? min(g[i] << 6, n) : 0u;
    w[i] = g[i] ? hi - lo[i] - 1 : 0u;
    pos[i] = 0;
  }
#pragma unroll
  for (uint32_t step = 32; step > 0; step >>= 1) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const uint32_t c = pos[i] + step;
      if (c <= w[i]) {
        const uint32_t v = keys[i][lo[i] + c];
        if (upper[i] ? (v <= x[i]) : (v < x[i])) pos[i] = c;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) res[i] = g[i] ? lo[i] + 1 + pos[i] : 0u;
}

// ---------------------------------------------------------------------------
// learned sizing (learn.hip)
// ---------------------------------------------------------------------------
constexpr int kFeatures = 18;
constexpr int kFeatBins = 64;
constexpr int kParams = 5441;  // 18*64 + 64 + 64*64 + 64 + 64 + 1

// inputs of the per-tree feature statistics
struct FeatArgs {
  const float* rec[DDM_MAX_D];
  const float* maxhi[DDM_MAX_D];
  const uint32_t* skey_lo[DDM_MAX_D];
  const uint32_t* sidx_lo[DDM_MAX_D];
  uint32_t n, d, ns, root;
  float* fstat;    // [DDM_MAX_D][4]: min lower bound, width, mean length, 0
  uint32_t* fcum;  // [DDM_MAX_D][2][kFeatBins + 1] prefix counts of lo / hi
  uint32_t* sat;   // kSatWords: d-dimensional prefix counts of lower corners
};
struct FeatDev {
  const float* fstat;
  const uint32_t* fcum;
  const uint32_t* sat;
  uint32_t n, d;
};
// grid cells per dimension of the joint lower-corner histogram (d <= 3)
__host__ __device__ constexpr uint32_t sat_grid(uint32_t d) {
  return d == 1 ? 256u : (d == 2 ? 64u : 16u);
}
constexpr uint32_t kSatWords = 17u * 17u * 17u;  // max over d of (G+1)^d
ddm_status enqueue_feature_stats(const FeatArgs& A, hipStream_t s);
ddm_status launch_features(const FeatDev& F, uint32_t d, const float* ulo, const float* uhi,
                           uint32_t m, float* X, hipStream_t s);
ddm_status launch_mlp_forward(const float* params, const float* X, uint32_t N, int out_mode,
                              float delta, uint32_t capmax, float* yhat, uint32_t* cap,
                              hipStream_t s);
ddm_status launch_mlp_grad(const float* params, const float* X, const float* Y, uint32_t N,
                           float* grad, float* loss, hipStream_t s);

// ---------------------------------------------------------------------------
// launchers implemented in the .hip files (all enqueue on `s`)
// ---------------------------------------------------------------------------
// radix sort of `narr` arrays described by device descriptors; 4 passes of 8
// bits; results end in k[0]/v[0].  hist: ntiles*256 uint32 scratch.
ddm_status radix_sort_batch(const SortArr* arrs_dev, uint32_t narr, const uint32_t* tile_map,
                            uint32_t ntiles, uint32_t* hist, int first_pass, int npasses,
                            hipStream_t s);
// fills descriptors + tile map on the device from host values (<= 8 arrays)
ddm_status sort_setup_small(const SortArr* host_arrs, uint32_t narr, SortArr* arrs_dev,
                            uint32_t* tile_map, uint32_t ntiles, hipStream_t s);

// one-sweep radix sort (stable LSD, 8-bit digits) of 1..kOsMaxArrays arrays
// whose sizes the host knows (host_arrs: k[0]/v[0] hold the input, k[1]/v[1]
// the second buffers; v may be null): one zeroing and one histogram kernel,
// then one kernel per pass; the result ends in k[npasses & 1] / v[...].
// scratch: radix_onesweep_scratch_bytes(...) bytes of device memory; err: a
// device word that receives kFlagSortTimeout if a look-back wait gave up
// (the order is then wrong).
constexpr uint32_t kOsMaxArrays = 2 * DDM_MAX_D;
constexpr int32_t kFlagSortTimeout = 0x40000000;
size_t radix_onesweep_scratch_bytes(const SortArr* host_arrs, uint32_t narr, int npasses);
ddm_status radix_sort_onesweep(const SortArr* host_arrs, uint32_t narr, int npasses,
                               void* scratch, int32_t* err, hipStream_t s);

// per-segment sort of the pairs in place (segments off[j] .. off[j+1]);
// ids must be below 2^20.  lists: 2m+2 uint32 scratch (last two words are
// counters, zeroed by the caller beforehand).
ddm_status sort_segments_inplace(const uint64_t* off, uint32_t m, uint64_t* out, uint32_t n,
                                 uint32_t* lists, uint32_t* lists_count, hipStream_t s);

// The plain match (count -> scan -> fill, no stash) with all its scratch in
// caller-provided device memory [base, base + cap) and the count read back
// into pageable host memory, so that it allocates nothing (match.hip; `who`
// names the caller in error details).
ddm_status match_external_scratch(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                                  uint32_t m, uint64_t* out_pairs, uint64_t capacity,
                                  uint64_t* out_count, hipStream_t s, char* base, size_t cap,
                                  const char* who);

// The learned single pass (as ddm_match_learned_begin) for a caller that
// accounts device memory: once the predicted number of slots is known, and
// before the slot arena is allocated, grant(predicted) is called (it may
// block) and returns the number of slots granted; the arena holds at most
// that many, and updates beyond it overflow into the exact fill.
// Returning kArenaRefused makes the match return DDM_E_NOMEM before it
// allocates anything more.
using ArenaGrant = std::function<uint64_t(uint64_t)>;
constexpr uint64_t kArenaRefused = ~0ull;
ddm_status match_learned_begin_granted(const ddm_tree* t, const float* upd_lo,
                                       const float* upd_hi, uint32_t m,
                                       const ddm_predictor* pred, uint64_t* out_count,
                                       hipStream_t s, const ddm_match_opts* opts,
                                       ddm_pending** out_pending, const ArenaGrant& grant);

// the same for K pairs and any n (ids above 2^20 are sorted from a copy)
ddm_status sort_segments_keys(const uint64_t* off, uint32_t m, uint64_t* out, uint64_t K,
                              uint32_t n, uint32_t* lists, uint32_t* lists_count, hipStream_t s);

// exclusive scan of u32 counts into u64 offsets out[0..m], out[m] = total.
// tmp: scan_tmp_words(m) uint64 scratch.  maxout (optional, zeroed by the
// caller): receives the largest count.
size_t scan_tmp_words(uint32_t m);
ddm_status scan_u32_u64(const uint32_t* in, uint64_t* out, uint32_t m, uint64_t* tmp,
                        hipStream_t s, uint32_t* maxout = nullptr);

}  // namespace ddm
