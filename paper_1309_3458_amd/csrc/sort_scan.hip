// Device radix sort (stable LSD, 8-bit digits, many arrays per launch) and
// exclusive scan (u32 counts -> u64 offsets) for gfx950 wave64.
//
// Sort: per pass three kernels -- tile histograms, per-array scan of the
// (tile, digit) counts, stable scatter.  A tile is 256 threads x 16 rounds.
// Within a round, a lane's rank among equal digits comes from eight wavefront
// ballots (lanes with the same digit), and the four waves of the workgroup
// are ordered through LDS counters, which keeps the sort stable.
#include "ddm_internal.h"

#include <algorithm>
#include <atomic>

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
  // each wavefront ranks a contiguous run of kSortItems * 64 keys of the
  // tile (key base + w * run + r * 64 + lane) against its own digit
  // counters, round after round without a barrier; one scan over the
  // wavefronts then places every run (stable: runs and rounds in key order)
  constexpr uint32_t NW = kSortThreads / kWave;
  constexpr uint32_t RUN = kSortItems * kWave;
  __shared__ uint32_t wc[NW][256];
  __shared__ uint32_t woff[NW][256];
  const uint32_t t = blockIdx.x;
  const uint32_t tid = threadIdx.x;
  const uint32_t wave = tid / kWave, lane = lane_id();
  const SortArr A = arrs[tile_map[t]];
  const uint32_t lt = t - A.tile0;
  const uint32_t* __restrict__ ks = A.k[pass & 1];
  uint32_t* __restrict__ kd = A.k[(pass & 1) ^ 1];
  const uint32_t* __restrict__ vs = A.v[pass & 1];
  uint32_t* __restrict__ vd = A.v[(pass & 1) ^ 1];
  const uint32_t base = lt * kSortTile + wave * RUN;
  const uint32_t end = min(A.n, lt * kSortTile + kSortTile);
  const int shift = pass * 8;
#pragma unroll
  for (uint32_t w = 0; w < NW; ++w) wc[w][tid] = 0;
  uint32_t key[kSortItems], val[kSortItems], loc[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t i = base + r * kWave + lane;
    const bool valid = i < end;
    key[r] = valid ? ks[i] : 0u;
    val[r] = (valid && vs) ? vs[i] : 0u;
  }
  __syncthreads();  // counters clear
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const bool valid = base + r * kWave + lane < end;
    const uint32_t dig = (key[r] >> shift) & 255u;
    const uint64_t peers = match_digit8(dig, ballot(valid));
    const uint32_t rk = mask_rank(peers);
    const uint32_t c = valid ? wc[wave][dig] : 0u;
    loc[r] = c + rk;
    if (valid && rk == 0) wc[wave][dig] = c + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // thread tid owns digit tid: the tile's offset of the digit (from the
  // scan of the tile histograms) plus the runs of the wavefronts before
  {
    uint32_t run = hist[(size_t)t * 256 + tid];
#pragma unroll
    for (uint32_t w = 0; w < NW; ++w) {
      woff[w][tid] = run;
      run += wc[w][tid];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (base + r * kWave + lane >= end) continue;
    const uint32_t pos = woff[wave][(key[r] >> shift) & 255u] + loc[r];
    kd[pos] = key[r];
    if (vd) vd[pos] = val[r];
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
// one-sweep radix sort of a few arrays with host-known sizes
//
// The digit totals of every pass come from one histogram kernel (they do not
// depend on the order of the keys).  Each pass is then one kernel: a tile
// (4096 or 8192 keys, 512 per wavefront in order) ranks its keys with
// per-wavefront digit counters (no workgroup barrier per round), publishes
// its digit counts, and takes the counts of the tiles before it in the same
// array by decoupled look-back: each digit walks back over the tiles'
// published (flag, count) words until one holds an inclusive prefix.  The
// look-back reads grow with the square of the tiles per array, and every
// tile runs its phases one after another (load, rank, look-back, stage,
// write), so few large tiles with many wavefronts each are faster than many
// small ones, as long as there are compute units for more of them.  When
// the device holds every tile at once a tile takes its index from its
// workgroup; otherwise from a counter in the order tiles start, so every
// tile they wait for has started and publishes without waiting on later
// tiles.  A wait longer than kOsSpinLimit sleeps gives up, raises
// kFlagSortTimeout in *err and goes on with a wrong offset, so that every
// wave still exits.
// ---------------------------------------------------------------------------
constexpr uint32_t kOsHistKeys = 4096;  // keys per workgroup of the histogram kernel
constexpr uint32_t kOsWindow = 8;       // predecessor tiles read together in a look-back step
// tiles of a pass: 4096 keys and 512 threads while one tile per compute
// unit covers the arrays, otherwise 8192 keys and 1024 threads (8 keys per
// lane either way)
constexpr uint32_t kOsTileSmall = 4096, kOsThreadsSmall = 512;
constexpr uint32_t kOsTileLarge = 8192, kOsThreadsLarge = 1024;
constexpr uint64_t kOsAgg = 1ull << 32, kOsIncl = 2ull << 32;
constexpr uint32_t kOsSpinLimit = 1u << 22;

struct OsDesc {
  SortArr a[kOsMaxArrays];
  uint32_t narr;
  uint32_t hblk0[kOsMaxArrays + 1];  // first histogram workgroup of each array
  uint32_t tile0[kOsMaxArrays + 1];  // first tile of each array
};

__device__ __forceinline__ uint32_t os_array(const uint32_t* first, uint32_t narr, uint32_t x) {
  uint32_t a = 0;
  for (uint32_t q = 1; q < narr; ++q)
    if (first[q] <= x) a = q;
  return a;
}

__global__ void os_zero_kernel(uint32_t* __restrict__ ghist, uint32_t nh,
                               uint32_t* __restrict__ ctr, uint64_t* __restrict__ status,
                               size_t nstatus) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = g; i < nh; i += stride) ghist[i] = 0;
  for (size_t i = g; i < nstatus; i += stride) status[i] = 0;
  if (g < 4) ctr[g] = 0;
}

__global__ __launch_bounds__(kSortThreads) void os_hist_kernel(OsDesc D, uint32_t* __restrict__ ghist,
                                                               int npasses) {
  __shared__ uint32_t h[4][256];
  const uint32_t tid = threadIdx.x;
#pragma unroll
  for (int p = 0; p < 4; ++p) h[p][tid] = 0;
  __syncthreads();
  const uint32_t a = os_array(D.hblk0, D.narr, blockIdx.x);
  const SortArr& A = D.a[a];
  const uint32_t begin = (blockIdx.x - D.hblk0[a]) * kOsHistKeys;
  const uint32_t end = min(A.n, begin + kOsHistKeys);
  const uint32_t* __restrict__ src = A.k[0];
  // all of this thread's keys are loaded before any is counted, so that the
  // loads are in flight together
  constexpr uint32_t R = kOsHistKeys / kSortThreads;
  uint32_t key[R];
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t i = begin + r * kSortThreads + tid;
    key[r] = i < end ? src[i] : 0u;
  }
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    if (begin + r * kSortThreads + tid >= end) break;
    for (int p = 0; p < npasses; ++p) atomicAdd(&h[p][(key[r] >> (8 * p)) & 255u], 1u);
  }
  __syncthreads();
  for (int p = 0; p < npasses; ++p) {
    const uint32_t c = h[p][tid];
    if (c) atomicAdd(&ghist[((size_t)a * 4 + p) * 256 + tid], c);
  }
}

template <uint32_t kOsThreads, uint32_t kOsTile>
__global__ __launch_bounds__(kOsThreads) void os_pass_kernel(OsDesc D,
                                                            const uint32_t* __restrict__ ghist,
                                                            uint32_t* __restrict__ ctr,
                                                            uint64_t* __restrict__ status,
                                                            uint32_t ntiles, int pass,
                                                            int32_t* __restrict__ err,
                                                            uint32_t direct) {
  constexpr uint32_t W = kOsThreads / kWave;  // wavefronts ranking the tile
  constexpr uint32_t DW = 256 / kWave;        // wavefronts that own one digit per lane
  constexpr uint32_t R = kOsTile / kOsThreads;  // keys per lane
  __shared__ uint32_t s_t;
  __shared__ uint32_t wcnt[W][256];
  __shared__ uint32_t woff[W][256];
  __shared__ uint32_t wsum[2][DW];
  __shared__ uint32_t ldst[256];  // first slot of each digit in the tile's staged order
  __shared__ uint32_t gpos[256];  // where that run starts in the output
  __shared__ uint32_t lkey[kOsTile];
  __shared__ uint32_t lval[kOsTile];
  const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
  if (!direct && tid == 0) s_t = atomicAdd(ctr + pass, 1u);
  for (uint32_t i = lane; i < 256; i += kWave) wcnt[wave][i] = 0;
  __syncthreads();
  const uint32_t t = direct ? blockIdx.x : s_t;
  const uint32_t a = os_array(D.tile0, D.narr, t);
  const SortArr& A = D.a[a];
  const uint32_t lt = t - D.tile0[a];
  const uint32_t* __restrict__ ks = A.k[pass & 1];
  uint32_t* __restrict__ kd = A.k[(pass & 1) ^ 1];
  const uint32_t* __restrict__ vs = A.v[pass & 1];
  uint32_t* __restrict__ vd = A.v[(pass & 1) ^ 1];
  const uint32_t tbase = lt * kOsTile;
  const uint32_t tn = min(kOsTile, A.n - tbase);  // keys in this tile
  const uint32_t base = tbase + wave * (R * kWave);
  const uint32_t shift = 8u * (uint32_t)pass;
  // the first DW wavefronts own one digit per lane in the scans below
  const bool owner = tid < 256;
  const uint32_t d = tid & 255u;
  const uint32_t g = owner ? ghist[((size_t)a * 4 + pass) * 256 + d] : 0u;
  uint32_t key[R], val[R], loc[R];
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t i = base + r * kWave + lane;
    const bool valid = i < A.n;
    key[r] = valid ? ks[i] : 0u;
    val[r] = (valid && vs) ? vs[i] : 0u;
  }
  // ranks inside the wavefront's R * 64 keys, in key order (stable)
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    const bool valid = base + r * kWave + lane < A.n;
    const uint32_t dig = (key[r] >> shift) & 255u;
    const uint64_t peers = match_digit8(dig, ballot(valid));
    const uint32_t rk = mask_rank(peers);
    const uint32_t b = valid ? wcnt[wave][dig] : 0u;
    loc[r] = b + rk;
    if (valid && rk == 0) wcnt[wave][dig] = b + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // digit owners: the tile's count of digit d, the digit's base in the array
  // and in the tile (scans over the digits), and the count of digit d in the
  // array's earlier tiles (look-back)
  uint32_t inc = 0, inc2 = 0, tc = 0, excl = 0;
  if (owner) {
#pragma unroll
    for (uint32_t w = 0; w < W; ++w) tc += wcnt[w][d];
    inc = g;
    inc2 = tc;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t x = (uint32_t)__shfl_up((int)inc, o, kWave);
      const uint32_t y = (uint32_t)__shfl_up((int)inc2, o, kWave);
      if (lane >= (uint32_t)o) {
        inc += x;
        inc2 += y;
      }
    }
    if (lane == kWave - 1) {
      wsum[0][wave] = inc;
      wsum[1][wave] = inc2;
    }
    uint64_t* __restrict__ st = status + (size_t)pass * ntiles * 256;
    if (lt == 0) {
      __hip_atomic_store(st + (size_t)t * 256 + d, kOsIncl | tc, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(st + (size_t)t * 256 + d, kOsAgg | tc, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      // tiles j-1, j-2, ... down to the array's first tile, kOsWindow at a
      // time (their loads are in flight together); a tile that has not
      // published yet is read again
      const uint32_t first = D.tile0[a];
      uint32_t j = t, spin = 0;
      bool done = false;
      while (!done) {
        uint64_t v[kOsWindow];
#pragma unroll
        for (uint32_t q = 0; q < kOsWindow; ++q)
          v[q] = (j - first > q) ? __hip_atomic_load(st + (size_t)(j - 1 - q) * 256 + d,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : 0ull;
        uint32_t used = 0;
        bool wait = false;
#pragma unroll
        for (uint32_t q = 0; q < kOsWindow; ++q) {
          if (done || wait || j - first <= q) continue;
          if ((v[q] >> 32) == 0) {
            wait = true;
            continue;
          }
          excl += (uint32_t)v[q];
          ++used;
          if (v[q] & kOsIncl) done = true;
        }
        j -= used;
        if (!done && j == first) done = true;  // never: the first tile is inclusive
        if (wait && !done) {
          if (++spin > kOsSpinLimit) {
            atomicOr(err, kFlagSortTimeout);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __hip_atomic_store(st + (size_t)t * 256 + d, kOsIncl | (excl + tc), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  if (owner) {
    uint32_t gb = inc - g, lb = inc2 - tc;
    for (uint32_t w = 0; w < wave; ++w) {
      gb += wsum[0][w];
      lb += wsum[1][w];
    }
    ldst[d] = lb;
    gpos[d] = gb + excl;
    uint32_t run = lb;
#pragma unroll
    for (uint32_t w = 0; w < W; ++w) {
      woff[w][d] = run;
      run += wcnt[w][d];
    }
  }
  __syncthreads();
  // stage the tile in digit order in LDS, then write each digit's run to
  // consecutive output slots (neighbouring lanes write neighbouring words)
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    if (base + r * kWave + lane < A.n) {
      const uint32_t lp = woff[wave][(key[r] >> shift) & 255u] + loc[r];
      if (lp < kOsTile) {
        lkey[lp] = key[r];
        lval[lp] = val[r];
      }
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < tn; i += kOsThreads) {
    const uint32_t k = lkey[i];
    const uint32_t dig = (k >> shift) & 255u;
    const uint32_t pos = gpos[dig] + (i - ldst[dig]);
    if (pos < A.n) {  // always, unless a look-back wait gave up
      kd[pos] = k;
      if (vd) vd[pos] = lval[i];
    }
  }
}

// compute units of the current device (0 if the runtime cannot say); and
// workgroups of a pass kernel the device holds at once (0 if unknown, which
// keeps the counter); each asked once per device
constexpr int kOsDevs = 64;

static uint32_t os_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return ~0u;
  }
  return dev >= 0 && dev < kOsDevs ? (uint32_t)dev : ~0u;
}

static uint32_t os_cus() {
  static std::atomic<uint32_t> cache[kOsDevs];  // value + 1, 0 = not asked yet
  const uint32_t dev = os_device();
  if (dev == ~0u) return 0;
  const uint32_t c = cache[dev].load(std::memory_order_relaxed);
  if (c) return c - 1;
  int cus = 0;
  uint32_t r = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, (int)dev) == hipSuccess)
    r = (uint32_t)std::max(0, cus);
  else
    (void)hipGetLastError();
  cache[dev].store(r + 1, std::memory_order_relaxed);
  return r;
}

template <uint32_t THREADS, uint32_t TILE>
static uint32_t os_resident_blocks() {
  static std::atomic<uint32_t> cache[kOsDevs];  // value + 1, 0 = not asked yet
  const uint32_t dev = os_device();
  if (dev == ~0u) return 0;
  const uint32_t c = cache[dev].load(std::memory_order_relaxed);
  if (c) return c - 1;
  int per = 0;
  uint32_t r = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, (const void*)os_pass_kernel<THREADS, TILE>, THREADS, 0) == hipSuccess)
    r = os_cus() * (uint32_t)std::max(0, per);
  else
    (void)hipGetLastError();
  cache[dev].store(r + 1, std::memory_order_relaxed);
  return r;
}

static uint32_t os_tiles(const SortArr* host_arrs, uint32_t narr, uint32_t tile) {
  uint32_t tl = 0;
  for (uint32_t i = 0; i < narr; ++i) tl += (host_arrs[i].n + tile - 1) / tile;
  return tl;
}

// the tile size of a sort of these arrays
static uint32_t os_tile_keys(const SortArr* host_arrs, uint32_t narr) {
  return os_tiles(host_arrs, narr, kOsTileSmall) <= os_cus() ? kOsTileSmall : kOsTileLarge;
}

static void os_layout(const SortArr* host_arrs, uint32_t narr, uint32_t tile, OsDesc* D,
                      uint32_t* nhblk, uint32_t* ntiles) {
  uint32_t hb = 0, tl = 0;
  *D = OsDesc{};
  D->narr = narr;
  for (uint32_t i = 0; i < narr; ++i) {
    D->a[i] = host_arrs[i];
    D->hblk0[i] = hb;
    D->tile0[i] = tl;
    hb += (host_arrs[i].n + kOsHistKeys - 1) / kOsHistKeys;
    tl += (host_arrs[i].n + tile - 1) / tile;
  }
  D->hblk0[narr] = hb;
  D->tile0[narr] = tl;
  *nhblk = hb;
  *ntiles = tl;
}

size_t radix_onesweep_scratch_bytes(const SortArr* host_arrs, uint32_t narr, int npasses) {
  OsDesc D;
  uint32_t hb, tl;
  // the smaller tiles bound the status words of either tile size
  os_layout(host_arrs, narr, kOsTileSmall, &D, &hb, &tl);
  return 256 + sizeof(uint32_t) * 1024 * (size_t)narr + sizeof(uint64_t) * 256 * (size_t)tl *
                                                            (size_t)(npasses > 0 ? npasses : 1);
}

ddm_status radix_sort_onesweep(const SortArr* host_arrs, uint32_t narr, int npasses,
                               void* scratch, int32_t* err, hipStream_t s) {
  if (narr == 0 || narr > kOsMaxArrays || npasses < 0 || npasses > 4) {
    set_detail("radix_sort_onesweep: 1..8 arrays, 0..4 passes");
    return DDM_E_INVALID_ARG;
  }
  if (npasses == 0) return DDM_OK;
  OsDesc D;
  uint32_t hb, tl;
  os_layout(host_arrs, narr, os_tile_keys(host_arrs, narr), &D, &hb, &tl);
  if (tl == 0) return DDM_OK;
  uint32_t* ctr = (uint32_t*)scratch;  // 4 counters, padded to 256 bytes
  uint32_t* ghist = (uint32_t*)((char*)scratch + 256);
  uint64_t* status = (uint64_t*)(ghist + 1024 * (size_t)narr);
  const size_t nstatus = 256 * (size_t)tl * (size_t)npasses;
  {
    ProfScope ps("radix_hist", s);
    const size_t work = std::max<size_t>(nstatus, 1024 * (size_t)narr);
    const unsigned zb = (unsigned)std::min<size_t>((work + 255) / 256, 2048);
    os_zero_kernel<<<zb, 256, 0, s>>>(ghist, 1024 * narr, ctr, status, nstatus);
    DDM_LAUNCHED("os_zero_kernel");
    os_hist_kernel<<<hb, kSortThreads, 0, s>>>(D, ghist, npasses);
    DDM_LAUNCHED("os_hist_kernel");
  }
  // when every workgroup of a pass fits on the device at once, a tile takes
  // its index from its workgroup (every tile it waits for is running);
  // otherwise from a counter in start order
  const bool small = os_tile_keys(host_arrs, narr) == kOsTileSmall;
  const uint32_t resident = small ? os_resident_blocks<kOsThreadsSmall, kOsTileSmall>()
                                  : os_resident_blocks<kOsThreadsLarge, kOsTileLarge>();
  const uint32_t direct = tl <= resident ? 1u : 0u;
  for (int p = 0; p < npasses; ++p) {
    ProfScope ps("radix_scatter", s);
    if (small)
      os_pass_kernel<kOsThreadsSmall, kOsTileSmall>
          <<<tl, kOsThreadsSmall, 0, s>>>(D, ghist, ctr, status, tl, p, err, direct);
    else
      os_pass_kernel<kOsThreadsLarge, kOsTileLarge>
          <<<tl, kOsThreadsLarge, 0, s>>>(D, ghist, ctr, status, tl, p, err, direct);
    DDM_LAUNCHED("os_pass_kernel");
  }
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
                                                               uint64_t* __restrict__ sums,
                                                               uint32_t* __restrict__ maxout) {
  const uint32_t base = blockIdx.x * kScanTile;
  uint64_t acc = 0;
  uint32_t mx = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t i = base + r * kScanThreads + threadIdx.x;
    if (i < m) {
      const uint32_t v = in[i];
      acc += v;
      mx = max(mx, v);
    }
  }
  uint64_t tot;
  (void)block_excl_scan_u64(acc, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
  if (maxout) {
    // one atomic per workgroup (the device-scope atomics on one word queue)
    __shared__ uint32_t wmax[kScanThreads / kWave];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, kWave));
    if (lane_id() == 0) wmax[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t b = 0;
      for (uint32_t w = 0; w < kScanThreads / kWave; ++w) b = max(b, wmax[w]);
      if (b) atomicMax(maxout, b);
    }
  }
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

// scan_tiles_kernel with the tile's base computed in the workgroup from the
// tile sums before it (for few tiles: saves the pass over the sums)
constexpr uint32_t kScanFusedTiles = 2048;

__global__ __launch_bounds__(kScanThreads) void scan_tiles_fused_kernel(
    const uint32_t* __restrict__ in, uint32_t m, const uint64_t* __restrict__ sums,
    uint64_t* __restrict__ out) {
  uint64_t prev = 0;
  for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanThreads) prev += sums[i];
  uint64_t tbase;
  (void)block_excl_scan_u64(prev, &tbase);
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
  uint64_t run = tbase + block_excl_scan_u64(acc, &tot);
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t i = base + r;
    if (i < m) out[i] = run;
    run += v[r];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[m] = tbase + tot;
}

size_t scan_tmp_words(uint32_t m) { return (size_t)(m + kScanTile - 1) / kScanTile + 1; }

ddm_status scan_u32_u64(const uint32_t* in, uint64_t* out, uint32_t m, uint64_t* tmp,
                        hipStream_t s, uint32_t* maxout) {
  const uint32_t nt = (m + kScanTile - 1) / kScanTile;
  if (nt == 0) {
    // m == 0: out[0] = 0 (a kernel rather than a memset node, so that the
    // sequence stays safe to capture into a graph)
    scan_sums_kernel<<<1, kScanThreads, 0, s>>>(out, 0);
    DDM_LAUNCHED("scan_sums_kernel");
    return DDM_OK;
  }
  ProfScope ps("scan", s);
  scan_tile_sums<<<nt, kScanThreads, 0, s>>>(in, m, tmp, maxout);
  DDM_LAUNCHED("scan_tile_sums");
  if (nt <= kScanFusedTiles) {
    scan_tiles_fused_kernel<<<nt, kScanThreads, 0, s>>>(in, m, tmp, out);
    DDM_LAUNCHED("scan_tiles_fused_kernel");
    return DDM_OK;
  }
  scan_sums_kernel<<<1, kScanThreads, 0, s>>>(tmp, nt);
  DDM_LAUNCHED("scan_sums_kernel");
  scan_tiles_kernel<<<nt, kScanThreads, 0, s>>>(in, m, tmp, out);
  DDM_LAUNCHED("scan_tiles_kernel");
  return DDM_OK;
}

}  // namespace ddm
