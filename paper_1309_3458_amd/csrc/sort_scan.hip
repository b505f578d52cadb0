// Device radix sort (stable LSD, 8-bit digits, many arrays per launch) and
// exclusive scan (u32 counts -> u64 offsets) for gfx950 wave64.
//
// Sort: per pass three kernels -- tile histograms, per-array scan of the
// (tile, digit) counts, stable scatter.  A tile is 256 threads x 16 rounds.
// Within a round, a lane's rank among equal digits comes from eight wavefront
// ballots (lanes with the same digit), and the four waves of the workgroup
// are ordered through LDS counters, which keeps the sort stable.
#include "ddm_internal.h"

namespace ddm {

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void rs_hist_kernel(const SortArr* __restrict__ arrs,
                                                               const uint32_t* __restrict__ tile_map,
                                                               uint32_t* __restrict__ hist, int pass) {
  __shared__ uint32_t h[256];
  const uint32_t t = blockIdx.x;
  const uint32_t tid = threadIdx.x;
  h[tid] = 0;
  const SortArr A = arrs[tile_map[t]];
  const uint32_t lt = t - A.tile0;
  const uint32_t* __restrict__ src = A.k[pass & 1];
  const uint32_t base = lt * kSortTile;
  const uint32_t end = min(A.n, base + kSortTile);
  const int shift = pass * 8;
  // all loads first, so the tile costs one memory latency
  uint32_t key[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t i = base + r * kSortThreads + tid;
    key[r] = (i < end) ? src[i] : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t i = base + r * kSortThreads + tid;
    const bool valid = i < end;
    const uint32_t dig = (key[r] >> shift) & 255u;
    const uint64_t peers = match_digit8(dig, ballot(valid));
    if (valid && mask_rank(peers) == 0) atomicAdd(&h[dig], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  hist[(size_t)t * 256 + tid] = h[tid];
}

// One workgroup per array: exclusive offsets of digit b in tile lt equal
// (all keys of smaller digits) + (keys of digit b in earlier tiles).  The
// 1024 threads are 256 digits x 4 quarters of the array's tiles.
constexpr int kScanQ = 4;

__global__ __launch_bounds__(256 * kScanQ) void rs_scan_kernel(const SortArr* __restrict__ arrs,
                                                               uint32_t* __restrict__ hist) {
  __shared__ uint32_t part[kScanQ][256];
  __shared__ uint32_t base[256];
  __shared__ uint32_t wtot[256 / kWave];
  const SortArr A = arrs[blockIdx.x];
  const uint32_t tid = threadIdx.x;
  const uint32_t b = tid & 255u, q = tid >> 8;
  const uint32_t T = (A.n + kSortTile - 1) / kSortTile;
  const uint32_t lt0 = (uint32_t)(((uint64_t)T * q) / kScanQ);
  const uint32_t lt1 = (uint32_t)(((uint64_t)T * (q + 1)) / kScanQ);
  uint32_t* __restrict__ h = hist + (size_t)A.tile0 * 256 + b;
  uint32_t sum = 0;
#pragma unroll 8
  for (uint32_t lt = lt0; lt < lt1; ++lt) sum += h[(size_t)lt * 256];
  part[q][b] = sum;
  __syncthreads();
  uint32_t excl = 0;
  if (q == 0) {
    uint32_t tot = 0;
#pragma unroll
    for (int qq = 0; qq < kScanQ; ++qq) tot += part[qq][b];
    const uint32_t lane = lane_id();
    uint32_t inc = tot;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t2 = __shfl_up(inc, o, kWave);
      if (lane >= (uint32_t)o) inc += t2;
    }
    if (lane == kWave - 1) wtot[b / kWave] = inc;
    excl = inc - tot;
  }
  __syncthreads();
  if (q == 0) {
    for (uint32_t w = 0; w < b / kWave; ++w) excl += wtot[w];
    base[b] = excl;
  }
  __syncthreads();
  uint32_t run = base[b];
  for (uint32_t qq = 0; qq < q; ++qq) run += part[qq][b];
#pragma unroll 8
  for (uint32_t lt = lt0; lt < lt1; ++lt) {
    const uint32_t v = h[(size_t)lt * 256];
    h[(size_t)lt * 256] = run;
    run += v;
  }
}

__global__ __launch_bounds__(kSortThreads) void rs_scatter_kernel(const SortArr* __restrict__ arrs,
                                                                  const uint32_t* __restrict__ tile_map,
                                                                  const uint32_t* __restrict__ hist,
                                                                  int pass) {
  __shared__ uint32_t doff[256];
  __shared__ uint32_t wc[kSortThreads / kWave][256];
  const uint32_t t = blockIdx.x;
  const uint32_t tid = threadIdx.x;
  const uint32_t wave = tid / kWave;
  const SortArr A = arrs[tile_map[t]];
  const uint32_t lt = t - A.tile0;
  const uint32_t* __restrict__ ks = A.k[pass & 1];
  uint32_t* __restrict__ kd = A.k[(pass & 1) ^ 1];
  const uint32_t* __restrict__ vs = A.v[pass & 1];
  uint32_t* __restrict__ vd = A.v[(pass & 1) ^ 1];
  const uint32_t base = lt * kSortTile;
  const uint32_t end = min(A.n, base + kSortTile);
  const int shift = pass * 8;
  doff[tid] = hist[(size_t)t * 256 + tid];
  uint32_t key[kSortItems], val[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t i = base + r * kSortThreads + tid;
    const bool valid = i < end;
    key[r] = valid ? ks[i] : 0u;
    val[r] = (valid && vs) ? vs[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (base + r * kSortThreads >= end) break;
    const uint32_t i = base + r * kSortThreads + tid;
    const bool valid = i < end;
    const uint32_t dig = (key[r] >> shift) & 255u;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; ++w) wc[w][tid] = 0;
    __syncthreads();
    const uint64_t peers = match_digit8(dig, ballot(valid));
    const uint32_t rank = mask_rank(peers);
    if (valid && rank == 0) wc[wave][dig] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = doff[dig] + rank;
      for (uint32_t w = 0; w < wave; ++w) pos += wc[w][dig];
      kd[pos] = key[r];
      if (vd) vd[pos] = val[r];
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; ++w) add += wc[w][tid];
    doff[tid] += add;
  }
}

ddm_status radix_sort_batch(const SortArr* arrs_dev, uint32_t narr, const uint32_t* tile_map,
                            uint32_t ntiles, uint32_t* hist, int first_pass, int npasses,
                            hipStream_t s) {
  if (ntiles == 0 || narr == 0) return DDM_OK;
  for (int p = first_pass; p < first_pass + npasses; ++p) {
    {
      ProfScope ps("radix_hist", s);
      rs_hist_kernel<<<ntiles, kSortThreads, 0, s>>>(arrs_dev, tile_map, hist, p);
      DDM_LAUNCHED("rs_hist_kernel");
    }
    {
      ProfScope ps("radix_scan", s);
      rs_scan_kernel<<<narr, 256 * kScanQ, 0, s>>>(arrs_dev, hist);
      DDM_LAUNCHED("rs_scan_kernel");
    }
    {
      ProfScope ps("radix_scatter", s);
      rs_scatter_kernel<<<ntiles, kSortThreads, 0, s>>>(arrs_dev, tile_map, hist, p);
      DDM_LAUNCHED("rs_scatter_kernel");
    }
  }
  return DDM_OK;
}

struct SmallSortDesc {
  SortArr a[2 * DDM_MAX_D];
  uint32_t narr;
};

__global__ void sort_setup_kernel(SmallSortDesc D, SortArr* __restrict__ out,
                                  uint32_t* __restrict__ tile_map, uint32_t ntiles) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < D.narr) out[t] = D.a[t];
  if (t < ntiles) {
    uint32_t a = 0;
    for (uint32_t q = 1; q < D.narr; ++q)
      if (D.a[q].tile0 <= t) a = q;
    tile_map[t] = a;
  }
}

ddm_status sort_setup_small(const SortArr* host_arrs, uint32_t narr, SortArr* arrs_dev,
                            uint32_t* tile_map, uint32_t ntiles, hipStream_t s) {
  if (narr > 2 * DDM_MAX_D) {
    set_detail("sort_setup_small: too many arrays");
    return DDM_E_INVALID_ARG;
  }
  SmallSortDesc D{};
  for (uint32_t i = 0; i < narr; ++i) D.a[i] = host_arrs[i];
  D.narr = narr;
  const uint32_t cnt = ntiles > narr ? ntiles : narr;
  sort_setup_kernel<<<(cnt + 255) / 256, 256, 0, s>>>(D, arrs_dev, tile_map, ntiles);
  DDM_LAUNCHED("sort_setup_kernel");
  return DDM_OK;
}

// ---------------------------------------------------------------------------
// exclusive scan u32 -> u64 (three kernels: tile sums, scan of sums, tiles)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    uint64_t o = __shfl_up(v, off, kWave);
    if (lane >= (uint32_t)off) v += o;
  }
  return v;
}

// block-wide exclusive scan of one u64 per thread (256 threads); returns the
// exclusive prefix, *total receives the block sum.
__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t v, uint64_t* total) {
  __shared__ uint64_t wsum[kScanThreads / kWave];
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  const uint64_t inc = wave_incl_scan_u64(v);
  if (lane == kWave - 1) wsum[wave] = inc;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    if ((uint32_t)w < wave) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_tile_sums(const uint32_t* __restrict__ in,
                                                               uint32_t m,
                                                               uint64_t* __restrict__ sums) {
  const uint32_t base = blockIdx.x * kScanTile;
  uint64_t acc = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t i = base + r * kScanThreads + threadIdx.x;
    if (i < m) acc += in[i];
  }
  uint64_t tot;
  (void)block_excl_scan_u64(acc, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(uint64_t* __restrict__ sums,
                                                                 uint32_t nt) {
  uint64_t carry = 0;
  for (uint32_t base = 0; base < nt; base += kScanThreads) {
    const uint32_t i = base + threadIdx.x;
    const uint64_t v = (i < nt) ? sums[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_excl_scan_u64(v, &tot);
    if (i < nt) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) sums[nt] = carry;
}

__global__ __launch_bounds__(kScanThreads) void scan_tiles_kernel(const uint32_t* __restrict__ in,
                                                                  uint32_t m,
                                                                  const uint64_t* __restrict__ sums,
                                                                  uint64_t* __restrict__ out) {
  // each thread owns kScanItems consecutive elements (blocked arrangement)
  const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint64_t acc = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t i = base + r;
    v[r] = (i < m) ? in[i] : 0u;
    acc += v[r];
  }
  uint64_t tot;
  uint64_t run = sums[blockIdx.x] + block_excl_scan_u64(acc, &tot);
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t i = base + r;
    if (i < m) out[i] = run;
    run += v[r];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[m] = sums[gridDim.x];
}

size_t scan_tmp_words(uint32_t m) { return (size_t)(m + kScanTile - 1) / kScanTile + 1; }

ddm_status scan_u32_u64(const uint32_t* in, uint64_t* out, uint32_t m, uint64_t* tmp,
                        hipStream_t s) {
  const uint32_t nt = (m + kScanTile - 1) / kScanTile;
  if (nt == 0) {
    // m == 0: out[0] = 0 (a kernel rather than a memset node, so that the
    // sequence stays safe to capture into a graph)
    scan_sums_kernel<<<1, kScanThreads, 0, s>>>(out, 0);
    DDM_LAUNCHED("scan_sums_kernel");
    return DDM_OK;
  }
  ProfScope ps("scan", s);
  scan_tile_sums<<<nt, kScanThreads, 0, s>>>(in, m, tmp);
  DDM_LAUNCHED("scan_tile_sums");
  scan_sums_kernel<<<1, kScanThreads, 0, s>>>(tmp, nt);
  DDM_LAUNCHED("scan_sums_kernel");
  scan_tiles_kernel<<<nt, kScanThreads, 0, s>>>(in, m, tmp, out);
  DDM_LAUNCHED("scan_tiles_kernel");
  return DDM_OK;
}

}  // namespace ddm
