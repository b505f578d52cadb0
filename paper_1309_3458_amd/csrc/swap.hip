// Matching two sets given together, with the tree on the smaller one.
//
// Sec. IV notes that n <= m may be assumed without loss of generality,
// swapping the roles of S and U otherwise: intersection is symmetric, so the
// pairs of a tree built on the updates and queried with the subscriptions
// are the same pairs with their two ids exchanged.  The swapped match yields
// (subscription << 32) | update keys grouped by subscription; a stable radix
// sort of the update ids, with the subscription ids as payload, regroups
// them by update while keeping each group's subscriptions in order, which is
// exactly the key order of ddm_match.  Only the digits an update id can have
// are sorted (one pass per 8 bits of m - 1).
#include "ddm_internal.h"

namespace ddm {

__global__ void swap_split_kernel(const uint64_t* __restrict__ keys, uint64_t K,
                                  uint32_t* __restrict__ upd, uint32_t* __restrict__ sub) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const uint64_t k = keys[i];
  upd[i] = (uint32_t)k;
  sub[i] = (uint32_t)(k >> 32);
}

__global__ void swap_join_kernel(const uint32_t* __restrict__ upd,
                                 const uint32_t* __restrict__ sub, uint64_t K,
                                 uint64_t* __restrict__ keys) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  keys[i] = ((uint64_t)upd[i] << 32) | sub[i];
}

}  // namespace ddm

using namespace ddm;

extern "C" ddm_status ddm_match_sets(const float* sub_lo, const float* sub_hi, uint32_t n,
                                     const float* upd_lo, const float* upd_hi, uint32_t m,
                                     uint32_t d, int swap_policy, uint64_t* out_pairs,
                                     uint64_t capacity, uint64_t* out_count, int* out_swapped,
                                     void* stream) {
  set_detail("");
  if (out_swapped) *out_swapped = 0;
  if (!out_count) {
    set_detail("ddm_match_sets: out_count is NULL");
    return DDM_E_INVALID_ARG;
  }
  *out_count = 0;
  if (swap_policy < DDM_SWAP_AUTO || swap_policy > DDM_SWAP_ALWAYS) {
    set_detail("ddm_match_sets: swap_policy must be DDM_SWAP_AUTO, _NEVER or _ALWAYS");
    return DDM_E_INVALID_ARG;
  }
  // the transposition sorts K < 2^32 pairs; a capacity below 2^32 bounds
  // every K that is ever written
  const bool small_cap = capacity < (1ull << 32);
  bool swap = false;
  if (swap_policy == DDM_SWAP_ALWAYS) {
    if (!small_cap) {
      set_detail("ddm_match_sets: the role swap needs capacity < 2^32");
      return DDM_E_INVALID_ARG;
    }
    swap = true;
  } else if (swap_policy == DDM_SWAP_AUTO) {
    // measured: with d <= 2 the per-update work and the transposition cost
    // more than the larger tree saves; with d >= 3 the larger tree's long
    // candidate ranges dominate
    swap = n > m && d >= 3 && small_cap;
  }
  hipStream_t s = (hipStream_t)stream;
  ddm_tree* t = nullptr;
  ddm_status r = swap ? ddm_build(upd_lo, upd_hi, m, d, stream, &t)
                      : ddm_build(sub_lo, sub_hi, n, d, stream, &t);
  if (r != DDM_OK) return r;
  uint64_t K = 0;
  r = swap ? ddm_match(t, sub_lo, sub_hi, n, out_pairs, capacity, &K, stream)
           : ddm_match(t, upd_lo, upd_hi, m, out_pairs, capacity, &K, stream);
  ddm_tree_free(t);
  *out_count = K;
  if (r != DDM_OK || !swap) return r;
  if (out_swapped) *out_swapped = 1;
  if (K == 0) return DDM_OK;
  uint32_t passes = 0;
  for (uint32_t v = m - 1; v; v >>= 8) ++passes;
  const uint32_t ntiles = (uint32_t)((K + kSortTile - 1) / kSortTile);
  Scratch sc(s);
  for (int i = 0; i < 4; ++i) sc.reserve(sizeof(uint32_t) * K);
  sc.reserve(sizeof(SortArr));
  sc.reserve(sizeof(uint32_t) * ntiles);
  sc.reserve(sizeof(uint32_t) * 256 * (size_t)ntiles);
  if (!sc.commit()) return DDM_E_NOMEM;
  uint32_t* ku[2] = {sc.take<uint32_t>(K), sc.take<uint32_t>(K)};
  uint32_t* vs[2] = {sc.take<uint32_t>(K), sc.take<uint32_t>(K)};
  SortArr* arr = sc.take<SortArr>(1);
  uint32_t* tile_map = sc.take<uint32_t>(ntiles);
  uint32_t* hist = sc.take<uint32_t>(256 * (size_t)ntiles);
  if (!sc.fits()) return scratch_overrun("ddm_match_sets");
  const unsigned grid = (unsigned)((K + 255) / 256);
  {
    ProfScope ps("swap_transpose", s);
    swap_split_kernel<<<grid, 256, 0, s>>>(out_pairs, K, ku[0], vs[0]);
    DDM_LAUNCHED("swap_split_kernel");
  }
  if (passes) {
    SortArr h{{ku[0], ku[1]}, {vs[0], vs[1]}, (uint32_t)K, 0};
    r = sort_setup_small(&h, 1, arr, tile_map, ntiles, s);
    if (r != DDM_OK) return r;
    r = radix_sort_batch(arr, 1, tile_map, ntiles, hist, 0, (int)passes, s);
    if (r != DDM_OK) return r;
  }
  {
    ProfScope ps("swap_transpose", s);
    swap_join_kernel<<<grid, 256, 0, s>>>(ku[passes & 1], vs[passes & 1], K, out_pairs);
    DDM_LAUNCHED("swap_join_kernel");
  }
  return DDM_OK;
}
