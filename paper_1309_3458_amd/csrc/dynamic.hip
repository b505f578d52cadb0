// Dynamic DDM: both extent sets, both interval trees and the current result
// stay resident on the device, and moving extents recomputes only the pairs
// of the moved extents (the paper's dynamic scenario, Sec. IV and Sec. VI:
// one tree over the subscriptions T_S and one over the updates T_U; a moved
// update needs one query of T_S, a moved subscription one query of T_U).
//
// A move of c extents of one set:
//   1. the moved ids are sorted (their new extents follow), marked in a
//      bitmap (a repeated id is refused) and their tree is refitted or
//      rebuilt (ddm_tree_update, which also validates the new extents);
//   2. their new extents overwrite the resident copy of the set;
//   3. the moved extents query the other set's tree: moved updates give
//      their columns of M directly (keys in update order); moved
//      subscriptions give their rows, which a stable radix sort of the
//      update ids turns into (update, subscription) key order;
//   4. the resident result drops every pair of a moved id (one pass with the
//      bitmap and a compaction) and merges the recomputed pairs in (both
//      lists are sorted and disjoint: each element's place is its index plus
//      the number of smaller elements of the other list).
// The result is always exactly the pairs of the current sets, sorted.
#include "ddm_internal.h"

#include <algorithm>
#include <new>

struct ddm_dynamic {
  int device = 0;
  uint32_t n = 0, m = 0, d = 0;
  float* s_lo = nullptr;  // resident copies, dimension-major
  float* s_hi = nullptr;
  float* u_lo = nullptr;
  float* u_hi = nullptr;
  ddm_tree* ts = nullptr;  // tree over the subscriptions
  ddm_tree* tu = nullptr;  // tree over the updates
  uint64_t* pairs = nullptr;  // current result (device)
  uint64_t K = 0, cap = 0;
  hipStream_t home = nullptr;  // stream of the last call (for frees)
};

namespace ddm {

__global__ void dyn_iota_kernel(uint32_t* __restrict__ v, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) v[i] = i;
}

__global__ void dyn_zero_kernel(uint32_t* __restrict__ p, uint64_t count) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

// marks the moved ids; flag[0] |= 1 for an id out of range, |= 2 for a
// repeated id
__global__ void dyn_mark_kernel(const uint32_t* __restrict__ ids, uint32_t count,
                                uint32_t limit, uint32_t* __restrict__ bits,
                                int32_t* __restrict__ flag) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  const uint32_t id = ids[c];
  if (id >= limit) {
    atomicOr(flag, 1);
    return;
  }
  const uint32_t old = atomicOr(&bits[id >> 5], 1u << (id & 31));
  if (old & (1u << (id & 31))) atomicOr(flag, 2);
}

// sorted moved ids (with their positions in the caller's arrays) -> the new
// extents in that order, and written into the resident copy of the set
__global__ void dyn_gather_scatter_kernel(const uint32_t* __restrict__ sid,
                                          const uint32_t* __restrict__ spos, uint32_t count,
                                          uint32_t d, const float* __restrict__ new_lo,
                                          const float* __restrict__ new_hi,
                                          float* __restrict__ glo, float* __restrict__ ghi,
                                          float* __restrict__ set_lo, float* __restrict__ set_hi,
                                          uint32_t set_count) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  const uint32_t id = sid[c], p = spos[c];
  for (uint32_t k = 0; k < d; ++k) {
    const float lo = new_lo[(size_t)k * count + p], hi = new_hi[(size_t)k * count + p];
    glo[(size_t)k * count + c] = lo;
    ghi[(size_t)k * count + c] = hi;
    set_lo[(size_t)k * set_count + id] = lo;
    set_hi[(size_t)k * set_count + id] = hi;
  }
}

// columns of moved updates: (local << 32) | s -> (update id << 32) | s
__global__ void dyn_remap_cols_kernel(uint64_t* __restrict__ keys, uint64_t K,
                                      const uint32_t* __restrict__ sid) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const uint64_t k = keys[i];
  keys[i] = ((uint64_t)sid[k >> 32] << 32) | (k & 0xffffffffull);
}

// rows of moved subscriptions: (local << 32) | u -> update id, subscription
// id (split for the stable sort by update id)
__global__ void dyn_split_rows_kernel(const uint64_t* __restrict__ keys, uint64_t K,
                                      const uint32_t* __restrict__ sid,
                                      uint32_t* __restrict__ upd, uint32_t* __restrict__ sub) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const uint64_t k = keys[i];
  upd[i] = (uint32_t)k;
  sub[i] = sid[k >> 32];
}

__global__ void dyn_join_kernel(const uint32_t* __restrict__ upd, const uint32_t* __restrict__ sub,
                                uint64_t K, uint64_t* __restrict__ keys) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) keys[i] = ((uint64_t)upd[i] << 32) | sub[i];
}

// keep[i] = 1 if pair i involves no moved id (of the moved set)
__global__ void dyn_keep_kernel(const uint64_t* __restrict__ keys, uint64_t K,
                                const uint32_t* __restrict__ bits, int rows,
                                uint32_t* __restrict__ keep) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const uint64_t k = keys[i];
  const uint32_t id = rows ? (uint32_t)k : (uint32_t)(k >> 32);
  keep[i] = (bits[id >> 5] >> (id & 31)) & 1u ? 0u : 1u;
}

__global__ void dyn_compact_kernel(const uint64_t* __restrict__ keys, uint64_t K,
                                   const uint32_t* __restrict__ keep,
                                   const uint64_t* __restrict__ pos, uint64_t* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K && keep[i]) out[pos[i]] = keys[i];
}

// number of elements of sorted v[0..len) below x
__device__ __forceinline__ uint64_t count_below(const uint64_t* __restrict__ v, uint64_t len,
                                                uint64_t x) {
  uint64_t lo = 0, hi = len;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (v[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// merge of two sorted, disjoint lists A (a elements) and B (b elements)
__global__ void dyn_merge_kernel(const uint64_t* __restrict__ A, uint64_t a,
                                 const uint64_t* __restrict__ B, uint64_t b,
                                 uint64_t* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a) {
    out[i + count_below(B, b, A[i])] = A[i];
  } else if (i < a + b) {
    const uint64_t jb = i - a;
    out[jb + count_below(A, a, B[jb])] = B[jb];
  }
}

static unsigned blocks(uint64_t count) { return (unsigned)((count + 255) / 256); }

// stable LSD radix sort of `count` (key, value) u32 pairs by the key's
// passes (8 bits each); the result lands in buffer index passes & 1
static ddm_status sort_pairs(uint32_t* const (&k)[2], uint32_t* const (&v)[2], uint32_t count,
                             uint32_t passes, hipStream_t s) {
  if (passes == 0 || count == 0) return DDM_OK;
  const uint32_t ntiles = (count + kSortTile - 1) / kSortTile;
  Scratch sc(s);
  sc.reserve(sizeof(SortArr));
  sc.reserve(sizeof(uint32_t) * ntiles);
  sc.reserve(sizeof(uint32_t) * 256 * (size_t)ntiles);
  if (!sc.commit()) return DDM_E_NOMEM;
  SortArr* arr = sc.take<SortArr>(1);
  uint32_t* tile_map = sc.take<uint32_t>(ntiles);
  uint32_t* hist = sc.take<uint32_t>(256 * (size_t)ntiles);
  if (!sc.fits()) return scratch_overrun("dynamic sort");
  SortArr h{{k[0], k[1]}, {v[0], v[1]}, count, 0};
  ddm_status r = sort_setup_small(&h, 1, arr, tile_map, ntiles, s);
  if (r != DDM_OK) return r;
  return radix_sort_batch(arr, 1, tile_map, ntiles, hist, 0, (int)passes, s);
}

static uint32_t passes_for(uint32_t max_value) {
  uint32_t p = 0;
  for (uint32_t v = max_value; v; v >>= 8) ++p;
  return p;
}

// the pairs of the sorted moved extents (glo/ghi, `count` of them, ids
// sid) against the other set's tree, as (update << 32) | subscription keys
// sorted ascending; rows: the moved extents are subscriptions
static ddm_status recompute(ddm_dynamic* dy, bool rows, const uint32_t* sid, const float* glo,
                            const float* ghi, uint32_t count, uint64_t** out, uint64_t* outK,
                            char** block, hipStream_t s) {
  const ddm_tree* other = rows ? dy->tu : dy->ts;
  uint64_t K = 0;
  ddm_pending* pend = nullptr;
  ddm_status r = ddm_match_begin(other, glo, ghi, count, &K, s, nullptr, &pend);
  if (r != DDM_OK) return r;
  *outK = K;
  *out = nullptr;
  *block = nullptr;
  if (K == 0) return ddm_match_finish(pend, nullptr, 0);
  if (K >= (1ull << 32)) {
    ddm_match_abort(pend);
    set_detail("dynamic move: more than 2^32 - 1 recomputed pairs");
    return DDM_E_INVALID_ARG;
  }
  const size_t bytes = sizeof(uint64_t) * K + (rows ? 4 * sizeof(uint32_t) * K + 1024 : 0);
  char* mem = dev_alloc(bytes, s);
  if (!mem) {
    ddm_match_abort(pend);
    set_detail("dynamic move: device allocation failed");
    return DDM_E_NOMEM;
  }
  uint64_t* keys = (uint64_t*)mem;
  r = ddm_match_finish(pend, keys, K);
  if (r != DDM_OK) {
    dev_free(mem, s);
    return r;
  }
  if (!rows) {
    dyn_remap_cols_kernel<<<blocks(K), 256, 0, s>>>(keys, K, sid);
    DDM_LAUNCHED("dyn_remap_cols_kernel");
  } else {
    // (subscription, update) order -> (update, subscription) order: a stable
    // sort by update id keeps each update's subscriptions ascending
    uint32_t* base = (uint32_t*)(mem + sizeof(uint64_t) * K);
    uint32_t* const ku[2] = {base, base + K};
    uint32_t* const vs[2] = {base + 2 * K, base + 3 * K};
    dyn_split_rows_kernel<<<blocks(K), 256, 0, s>>>(keys, K, sid, ku[0], vs[0]);
    DDM_LAUNCHED("dyn_split_rows_kernel");
    const uint32_t passes = passes_for(dy->m - 1);
    r = sort_pairs(ku, vs, (uint32_t)K, passes, s);
    if (r != DDM_OK) {
      dev_free(mem, s);
      return r;
    }
    dyn_join_kernel<<<blocks(K), 256, 0, s>>>(ku[passes & 1], vs[passes & 1], K, keys);
    DDM_LAUNCHED("dyn_join_kernel");
  }
  *out = keys;
  *block = mem;
  return DDM_OK;
}

}  // namespace ddm

using namespace ddm;

extern "C" ddm_status ddm_dynamic_create(const float* sub_lo, const float* sub_hi, uint32_t n,
                                         const float* upd_lo, const float* upd_hi, uint32_t m,
                                         uint32_t d, void* stream, ddm_dynamic** out) {
  set_detail("");
  if (!out || d < 1 || d > DDM_MAX_D || (n && (!sub_lo || !sub_hi)) ||
      (m && (!upd_lo || !upd_hi)) || n >= 0x80000000u || m >= 0x80000000u) {
    set_detail("ddm_dynamic_create: bad argument");
    return DDM_E_INVALID_ARG;
  }
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  ddm_dynamic* dy = new (std::nothrow) ddm_dynamic();
  if (!dy) return DDM_E_NOMEM;
  DDM_HIP(hipGetDevice(&dy->device));
  dy->n = n;
  dy->m = m;
  dy->d = d;
  dy->home = s;
  const size_t sb = sizeof(float) * d * (size_t)std::max(n, 1u);
  const size_t ub = sizeof(float) * d * (size_t)std::max(m, 1u);
  dy->s_lo = (float*)dev_alloc(sb, s);
  dy->s_hi = (float*)dev_alloc(sb, s);
  dy->u_lo = (float*)dev_alloc(ub, s);
  dy->u_hi = (float*)dev_alloc(ub, s);
  auto fail = [&](ddm_status r) {
    ddm_dynamic_free(dy);
    return r;
  };
  if (!dy->s_lo || !dy->s_hi || !dy->u_lo || !dy->u_hi) {
    set_detail("ddm_dynamic_create: device allocation failed");
    return fail(DDM_E_NOMEM);
  }
  if (n) {
    DDM_HIP(hipMemcpyAsync(dy->s_lo, sub_lo, sizeof(float) * d * (size_t)n,
                           hipMemcpyDeviceToDevice, s));
    DDM_HIP(hipMemcpyAsync(dy->s_hi, sub_hi, sizeof(float) * d * (size_t)n,
                           hipMemcpyDeviceToDevice, s));
  }
  if (m) {
    DDM_HIP(hipMemcpyAsync(dy->u_lo, upd_lo, sizeof(float) * d * (size_t)m,
                           hipMemcpyDeviceToDevice, s));
    DDM_HIP(hipMemcpyAsync(dy->u_hi, upd_hi, sizeof(float) * d * (size_t)m,
                           hipMemcpyDeviceToDevice, s));
  }
  ddm_status r = ddm_build(dy->s_lo, dy->s_hi, n, d, stream, &dy->ts);
  if (r != DDM_OK) return fail(r);
  r = ddm_build(dy->u_lo, dy->u_hi, m, d, stream, &dy->tu);
  if (r != DDM_OK) return fail(r);
  r = ddm_tree_check(dy->tu);
  if (r != DDM_OK) return fail(r);
  uint64_t K = 0;
  ddm_pending* pend = nullptr;
  r = ddm_match_begin(dy->ts, dy->u_lo, dy->u_hi, m, &K, stream, nullptr, &pend);
  if (r != DDM_OK) return fail(r);
  dy->cap = std::max<uint64_t>(K, 1);
  dy->pairs = (uint64_t*)dev_alloc(sizeof(uint64_t) * dy->cap, s);
  if (!dy->pairs) {
    ddm_match_abort(pend);
    set_detail("ddm_dynamic_create: device allocation failed");
    return fail(DDM_E_NOMEM);
  }
  r = ddm_match_finish(pend, dy->pairs, dy->cap);
  if (r != DDM_OK) return fail(r);
  dy->K = K;
  *out = dy;
  return DDM_OK;
}

extern "C" ddm_status ddm_dynamic_move(ddm_dynamic* dy, uint32_t set, const uint32_t* ids,
                                       const float* new_lo, const float* new_hi, uint32_t count,
                                       void* stream, uint64_t* out_count) {
  set_detail("");
  if (!dy || set > DDM_DYNAMIC_UPDATES || (count && (!ids || !new_lo || !new_hi))) {
    set_detail("ddm_dynamic_move: bad argument");
    return DDM_E_INVALID_ARG;
  }
  if (out_count) *out_count = dy->K;
  if (count == 0) return DDM_OK;
  int cur = -1;
  DDM_HIP(hipGetDevice(&cur));
  if (cur != dy->device) {
    set_detail("ddm_dynamic_move: the current device is not the object's device");
    return DDM_E_INVALID_ARG;
  }
  const bool rows = set == DDM_DYNAMIC_SUBSCRIPTIONS;
  const uint32_t limit = rows ? dy->n : dy->m;
  if (count > limit) {
    set_detail("ddm_dynamic_move: more moves than extents in the set");
    return DDM_E_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  dy->home = s;
  const uint32_t d = dy->d;
  const uint64_t words = ((uint64_t)limit + 31) / 32;
  // scratch: sorted ids and positions (two buffers each), bitmap, flag, the
  // moved extents in sorted order
  Scratch sc(s);
  for (int i = 0; i < 4; ++i) sc.reserve(sizeof(uint32_t) * count);
  sc.reserve(sizeof(uint32_t) * words);
  sc.reserve(sizeof(int32_t));
  sc.reserve(sizeof(float) * d * (size_t)count);
  sc.reserve(sizeof(float) * d * (size_t)count);
  if (!sc.commit()) return DDM_E_NOMEM;
  uint32_t* const kid[2] = {sc.take<uint32_t>(count), sc.take<uint32_t>(count)};
  uint32_t* const kpos[2] = {sc.take<uint32_t>(count), sc.take<uint32_t>(count)};
  uint32_t* bits = sc.take<uint32_t>(words);
  int32_t* flag = sc.take<int32_t>(1);
  float* glo = sc.take<float>((size_t)d * count);
  float* ghi = sc.take<float>((size_t)d * count);
  if (!sc.fits()) return scratch_overrun("ddm_dynamic_move");
  // 1. mark the ids (range, repeats), sort them with their positions
  dyn_zero_kernel<<<blocks(words + 1), 256, 0, s>>>(bits, words);
  DDM_LAUNCHED("dyn_zero_kernel");
  dyn_zero_kernel<<<1, 64, 0, s>>>((uint32_t*)flag, 1);
  DDM_LAUNCHED("dyn_zero_kernel");
  dyn_mark_kernel<<<blocks(count), 256, 0, s>>>(ids, count, limit, bits, flag);
  DDM_LAUNCHED("dyn_mark_kernel");
  int32_t hflag = 0;
  DDM_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  DDM_HIP(hipStreamSynchronize(s));
  if (hflag) {
    set_detail(hflag & 1 ? "ddm_dynamic_move: id out of range"
                         : "ddm_dynamic_move: an id appears more than once");
    return DDM_E_INVALID_INPUT;
  }
  DDM_HIP(hipMemcpyAsync(kid[0], ids, sizeof(uint32_t) * count, hipMemcpyDeviceToDevice, s));
  dyn_iota_kernel<<<blocks(count), 256, 0, s>>>(kpos[0], count);
  DDM_LAUNCHED("dyn_iota_kernel");
  const uint32_t passes = passes_for(limit - 1);
  ddm_status r = sort_pairs(kid, kpos, count, passes, s);
  if (r != DDM_OK) return r;
  const uint32_t* sid = kid[passes & 1];
  const uint32_t* spos = kpos[passes & 1];
  // 2. refit (validates the new extents; nothing changes on error), then
  // write the new extents into the resident copy, in sorted order
  r = ddm_tree_update(rows ? dy->ts : dy->tu, ids, new_lo, new_hi, count, stream, nullptr);
  if (r != DDM_OK) return r;
  dyn_gather_scatter_kernel<<<blocks(count), 256, 0, s>>>(
      sid, spos, count, d, new_lo, new_hi, glo, ghi, rows ? dy->s_lo : dy->u_lo,
      rows ? dy->s_hi : dy->u_hi, limit);
  DDM_LAUNCHED("dyn_gather_scatter_kernel");
  // 3. the moved extents' pairs against the other set's tree
  uint64_t* fresh = nullptr;
  uint64_t F = 0;
  char* fresh_mem = nullptr;
  r = recompute(dy, rows, sid, glo, ghi, count, &fresh, &F, &fresh_mem, s);
  if (r != DDM_OK) return r;
  // 4. drop the moved ids' old pairs, merge the new ones in
  const uint64_t K = dy->K;
  if (K >= (1ull << 32)) {
    if (fresh_mem) dev_free(fresh_mem, s);
    set_detail("ddm_dynamic_move: more than 2^32 - 1 resident pairs");
    return DDM_E_INVALID_ARG;
  }
  Scratch sk(s);
  sk.reserve(sizeof(uint32_t) * std::max<uint64_t>(K, 1));
  sk.reserve(sizeof(uint64_t) * (K + 1));
  sk.reserve(sizeof(uint64_t) * scan_tmp_words((uint32_t)K));
  sk.reserve(sizeof(uint64_t) * std::max<uint64_t>(K, 1));
  if (!sk.commit()) {
    if (fresh_mem) dev_free(fresh_mem, s);
    return DDM_E_NOMEM;
  }
  uint32_t* keep = sk.take<uint32_t>(std::max<uint64_t>(K, 1));
  uint64_t* pos = sk.take<uint64_t>(K + 1);
  uint64_t* stmp = sk.take<uint64_t>(scan_tmp_words((uint32_t)K));
  uint64_t* kept = sk.take<uint64_t>(std::max<uint64_t>(K, 1));
  if (!sk.fits()) {
    if (fresh_mem) dev_free(fresh_mem, s);
    return scratch_overrun("ddm_dynamic_move");
  }
  uint64_t A = 0;
  if (K) {
    dyn_keep_kernel<<<blocks(K), 256, 0, s>>>(dy->pairs, K, bits, rows ? 1 : 0, keep);
    DDM_LAUNCHED("dyn_keep_kernel");
    r = scan_u32_u64(keep, pos, (uint32_t)K, stmp, s);
    if (r != DDM_OK) {
      if (fresh_mem) dev_free(fresh_mem, s);
      return r;
    }
    dyn_compact_kernel<<<blocks(K), 256, 0, s>>>(dy->pairs, K, keep, pos, kept);
    DDM_LAUNCHED("dyn_compact_kernel");
    DDM_HIP(hipMemcpyAsync(&A, pos + K, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    DDM_HIP(hipStreamSynchronize(s));
  }
  const uint64_t total = A + F;
  if (total > dy->cap) {
    uint64_t* grown = (uint64_t*)dev_alloc(sizeof(uint64_t) * total, s);
    if (!grown) {
      if (fresh_mem) dev_free(fresh_mem, s);
      set_detail("ddm_dynamic_move: device allocation failed");
      return DDM_E_NOMEM;
    }
    dev_free((char*)dy->pairs, s);
    dy->pairs = grown;
    dy->cap = total;
  }
  if (total) {
    dyn_merge_kernel<<<blocks(total), 256, 0, s>>>(kept, A, fresh, F, dy->pairs);
    DDM_LAUNCHED("dyn_merge_kernel");
  }
  dy->K = total;
  if (fresh_mem) dev_free(fresh_mem, s);
  if (out_count) *out_count = total;
  return DDM_OK;
}

extern "C" ddm_status ddm_dynamic_result(const ddm_dynamic* dy, const uint64_t** pairs,
                                         uint64_t* count) {
  if (!dy || !pairs || !count) return DDM_E_INVALID_ARG;
  *pairs = dy->pairs;
  *count = dy->K;
  return DDM_OK;
}

extern "C" void ddm_dynamic_free(ddm_dynamic* dy) {
  if (!dy) return;
  if (dy->ts) ddm_tree_free(dy->ts);
  if (dy->tu) ddm_tree_free(dy->tu);
  hipStream_t s = dy->home;
  if (dy->pairs) dev_free((char*)dy->pairs, s);
  if (dy->s_lo) dev_free((char*)dy->s_lo, s);
  if (dy->s_hi) dev_free((char*)dy->s_hi, s);
  if (dy->u_lo) dev_free((char*)dy->u_lo, s);
  if (dy->u_hi) dev_free((char*)dy->u_hi, s);
  delete dy;
}
