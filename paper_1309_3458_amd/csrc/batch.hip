// Many independent DDM instances matched together (an addition to the
// paper's method; each instance is the problem of Sec. III solved as in
// Algorithm 5).
//
// Every step handles all instances in the same launches: one key kernel, one
// radix sort over all arrays, one pass of tree kernels over all trees, one
// probe kernel, one counting sort of all updates by (instance, probe
// dimension, position), one persistent traversal for the counts, one scan,
// one persistent traversal for the fill and one segment sort.  The two
// traversals are persistent kernels: a fixed grid of wavefronts takes work
// items (instance, probe dimension, tile of updates) from an atomic ticket
// until none are left.  The sequence has no host synchronization and no
// allocation, so it is captured once into a hipGraph and replayed.
//
// The updates of all instances are numbered globally in instance order, so a
// single exclusive scan of the per-update counts gives every instance's
// output range: instance i owns out[off[qbase_i] .. off[qbase_i + m_i]).
#include <algorithm>
#include <new>
#include <vector>

#include "ddm_internal.h"
#include "traverse.h"
#include "tree_dev.h"

namespace ddm {

struct BInst {
  TreeDev T;
  const float* s_lo;
  const float* s_hi;
  const float* u_lo;
  const float* u_hi;
  uint32_t n, m, d;
  uint32_t qbase;  // first global update index
  uint32_t bbase;  // first bucket
  uint32_t nb;     // buckets per dimension
  uint32_t qpt;    // updates per traversal work item
  uint64_t ebase;  // first element of the key kernel (d * n elements)
  int32_t* flag;   // nonzero: invalid coordinates
  uint32_t* klo;   // d * n lower keys (tree k: klo + k n)
  uint32_t* khi;   // n upper keys (d == 1), else null
  uint32_t* idb;   // d * (n + 1) payload / ids
};

constexpr uint32_t kProbeThreads = 1024;
// trees are a grid dimension of the index kernel (at most 65535)
constexpr uint32_t kBatchMaxInstances = DDM_BATCH_MAX_INSTANCES;
static_assert(kBatchMaxInstances * DDM_MAX_D <= 65535, "index grid");
constexpr uint32_t kBatchStatusCapacity = 1u;
constexpr uint32_t kBatchStatusInput = 2u;

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void b_reset_kernel(uint32_t* __restrict__ w, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) w[i] = 0;
}

// validate, keys, payload for every instance (flat over sum d n elements)
__global__ __launch_bounds__(256) void b_keys_kernel(const BInst* __restrict__ I, uint32_t count,
                                                     uint64_t total) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  uint32_t lo = 0, hi = count;  // last instance with ebase <= e
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (I[mid].ebase <= e) lo = mid;
    else hi = mid;
  }
  const BInst& b = I[lo];
  const uint64_t r = e - b.ebase;
  const uint32_t k = (uint32_t)(r / b.n);
  const uint32_t i = (uint32_t)(r - (uint64_t)k * b.n);
  const float a = b.s_lo[r], c = b.s_hi[r];
  if (!valid_extent(a, c)) atomicOr(b.flag, 1);
  b.klo[r] = f2key(a);
  if (b.khi) b.khi[r] = f2key(c);
  b.idb[(size_t)k * (b.n + 1) + 1 + i] = i;
}

__global__ void b_index_kernel(const TreeJob* __restrict__ jobs) {
  tree_index_item(jobs[blockIdx.y], blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(kTreeThreads) void b_tree_low_kernel(const TreeJob* __restrict__ jobs,
                                                                  const uint2* __restrict__ map) {
  const uint2 w = map[blockIdx.x];
  tree_low_chunk(jobs[w.x], w.y);
}

__global__ __launch_bounds__(kTreeThreads) void b_tree_high_kernel(const TreeJob* __restrict__ jobs,
                                                                   const uint2* __restrict__ map,
                                                                   uint32_t S) {
  const uint2 w = map[blockIdx.x];
  tree_high_chunk(jobs[w.x], w.y, S);
}

// Probe dimension, bucket and rank of every update; one workgroup belongs to
// one instance (map entry: instance, block within it).  d = 1: exact BITS
// count (also the final count); d > 1: quantile estimate of the candidate
// range as in the single-instance matcher.
__global__ __launch_bounds__(kProbeThreads) void b_probe_kernel(const BInst* __restrict__ I,
                                                                const uint2* __restrict__ map,
                                                                uint8_t* __restrict__ kstar,
                                                                uint32_t* __restrict__ bucket,
                                                                uint32_t* __restrict__ rank,
                                                                uint32_t* __restrict__ bhist,
                                                                uint32_t* __restrict__ cnt) {
  __shared__ uint32_t sq[DDM_MAX_D][kQuantPad];
  const uint2 w = map[blockIdx.x];
  const BInst& b = I[w.x];
  const uint32_t d = b.d;
  if (d > 1)
    for (uint32_t k = 0; k < d; ++k) {
      // a dimension's loads are issued before its LDS stores (in flight together)
      constexpr uint32_t Q = kQuant / kProbeThreads;
      uint32_t v[Q];
#pragma unroll
      for (uint32_t r = 0; r < Q; ++r) v[r] = b.T.quant[k][r * kProbeThreads + threadIdx.x];
#pragma unroll
      for (uint32_t r = 0; r < Q; ++r) sq[k][qslot(r * kProbeThreads + threadIdx.x)] = v[r];
    }
  __syncthreads();
  const uint32_t j = w.y * kProbeThreads + threadIdx.x;
  const bool act = j < b.m;
  bool bad = false;
  if (act) {
    const uint32_t gj = b.qbase + j;
    uint32_t bk = 0, sub = 0;
    if (d == 1) {
      const float a = b.u_lo[j], c = b.u_hi[j];
      bad = !valid_extent(a, c);
      const uint32_t* keys[2] = {b.T.skey_lo[0], b.T.skey_hi[0]};
      const uint32_t* idx[2] = {b.T.sidx_lo[0], b.T.sidx_hi[0]};
      const uint32_t x[2] = {f2key(c), f2key(a)};
      const bool up[2] = {true, false};
      uint32_t res[2];
      count_2l<2>(keys, idx, x, up, b.n, b.T.ns, res);
      cnt[gj] = bad ? 0u : res[0] - res[1];
      sub = (uint32_t)(((uint64_t)(bad ? 0u : res[0]) * b.nb) / ((uint64_t)b.n + 1));
    } else {
      uint32_t best = 0xffffffffu, bqa = 0, bx = 0;
      for (uint32_t k = 0; k < d; ++k) {
        const float a = b.u_lo[(size_t)k * b.m + j], c = b.u_hi[(size_t)k * b.m + j];
        bad = bad || !valid_extent(a, c);
        const uint32_t xh = f2key(c);
        const uint32_t qa = quant_count(sq[k], xh, true);
        const uint32_t qb =
            quant_count(sq[k], f2key(nextafterf(a - b.T.maxlen[k], -INFINITY)), false);
        const uint32_t est = qa - min(qa, qb);
        if (est < best) {
          best = est;
          bk = k;
          bqa = qa;
          bx = xh;
        }
      }
      float fine = 0.f;
      if (bqa >= kQuant) {
        fine = (float)kQuant - 0.5f;
      } else if (bqa > 0) {
        const uint32_t kl = sq[bk][qslot(bqa - 1)], ku = sq[bk][qslot(bqa)];
        const float fr = ku > kl ? (float)(bx - kl) / (float)(ku - kl) : 0.f;
        fine = (float)(bqa - 1) + fminf(fr, 0.999f);
      }
      if (bad) {
        bk = 0;
        fine = 0.f;
      }
      sub = (uint32_t)(fine * (float)b.nb / (float)kQuant);
    }
    sub = min(sub, b.nb - 1u);
    kstar[gj] = (uint8_t)bk;
    const uint32_t bu = b.bbase + bk * b.nb + sub;
    bucket[gj] = bu;
    rank[gj] = atomicAdd(&bhist[bu], 1u);
  }
  if (ballot(bad) != 0 && lane_id() == 0) atomicOr(b.flag, 2);
}

__global__ __launch_bounds__(256) void b_scatter_kernel(const uint32_t* __restrict__ bucket,
                                                        const uint32_t* __restrict__ rank,
                                                        uint32_t M, const uint64_t* __restrict__ boff,
                                                        uint32_t* __restrict__ perm) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < M) perm[(uint32_t)boff[bucket[j]] + rank[j]] = j;
}

// groups (instance, probe dimension): start, size, and the exclusive prefix
// of their tiles for the count pass (d > 1 only) and the fill pass
__global__ __launch_bounds__(1024) void b_groups_kernel(const BInst* __restrict__ I, uint32_t count,
                                                        const uint64_t* __restrict__ boff,
                                                        uint32_t* __restrict__ gstart,
                                                        uint32_t* __restrict__ gcount,
                                                        uint32_t* __restrict__ tpc,
                                                        uint32_t* __restrict__ tpf,
                                                        uint32_t* __restrict__ snext,
                                                        uint32_t sfirst, uint32_t sslice) {
  __shared__ uint32_t wsum[2][1024 / kWave];
  __shared__ uint32_t carry[2];
  const uint32_t G = count * DDM_MAX_D;
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  // the count traversal's stash: next free chunk of each slice, overflow
  if (snext && tid <= kStashSlices) snext[tid] = tid < kStashSlices ? sfirst + tid * sslice : 0u;
  if (tid == 0) carry[0] = carry[1] = 0;
  __syncthreads();
  for (uint32_t base = 0; base < G; base += 1024) {
    const uint32_t g = base + tid;
    uint32_t tc = 0, tf = 0;
    if (g < G) {
      const uint32_t i = g / DDM_MAX_D, k = g % DDM_MAX_D;
      const BInst& b = I[i];
      uint32_t st = 0, sz = 0;
      if (k < b.d) {
        const uint32_t b0 = b.bbase + k * b.nb;
        st = (uint32_t)boff[b0];
        sz = (uint32_t)(boff[b0 + b.nb] - boff[b0]);
      }
      gstart[g] = st;
      gcount[g] = sz;
      tf = (sz + b.qpt - 1) / b.qpt;
      tc = b.d > 1 ? tf : 0u;
    }
    uint32_t ic = tc, jf = tf;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t a = __shfl_up(ic, o, kWave), c = __shfl_up(jf, o, kWave);
      if (lane >= (uint32_t)o) {
        ic += a;
        jf += c;
      }
    }
    if (lane == kWave - 1) {
      wsum[0][wave] = ic;
      wsum[1][wave] = jf;
    }
    __syncthreads();
    uint32_t bc = carry[0], bf = carry[1], totc = 0, totf = 0;
    for (uint32_t q = 0; q < 1024 / kWave; ++q) {
      if (q < wave) {
        bc += wsum[0][q];
        bf += wsum[1][q];
      }
      totc += wsum[0][q];
      totf += wsum[1][q];
    }
    if (g < G) {
      tpc[g] = bc + ic - tc;
      tpf[g] = bf + jf - tf;
    }
    __syncthreads();
    if (tid == 0) {
      carry[0] += totc;
      carry[1] += totf;
    }
    __syncthreads();
  }
  if (tid == 0) {
    tpc[G] = carry[0];
    tpf[G] = carry[1];
  }
}

// tile -> group (instance, probe dimension): one thread per possible tile,
// binary search of the groups' first tiles
__global__ __launch_bounds__(256) void b_tilemap_kernel(uint32_t G, const uint32_t* __restrict__ tp,
                                                        uint32_t* __restrict__ tmap,
                                                        uint32_t tiles_max) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tiles_max || t >= tp[G]) return;
  uint32_t lo = 0, hi = G;  // last g with tp[g] <= t
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tp[mid] <= t) lo = mid;
    else hi = mid;
  }
  tmap[t] = lo;
}

// Traversal over the tiles of every group.  persistent == 0: one wavefront
// per tile (the grid covers the largest possible number of tiles, waves
// beyond the actual number return); otherwise a fixed grid whose
// wavefronts take tiles from the ticket until they are exhausted.
template <bool FILL, bool STASH = false>
__global__ __launch_bounds__(kTileWaves * kWave) void b_traverse_kernel(
    const BInst* __restrict__ I, uint32_t G, const uint32_t* __restrict__ tp,
    const uint32_t* __restrict__ tmap, const uint32_t* __restrict__ gstart,
    const uint32_t* __restrict__ gcount, const uint32_t* __restrict__ perm,
    uint32_t* __restrict__ ticket, uint32_t persistent, const uint32_t* __restrict__ status,
    SegOut O, const uint32_t* __restrict__ stash_done) {
  __shared__ float s_cand[kTileWaves][2 * DDM_MAX_D * kRing];
  __shared__ uint32_t s_cid[kTileWaves][kRing];
  __shared__ float4 s_q[kTileWaves][kWave * 2];
  const uint32_t wave = threadIdx.x / kWave;
  const uint32_t lane = lane_id();
  if (FILL && uniform_u32(*status) != 0) return;
  // the stash holds the pairs of every instance with d > 1
  const bool skip_multi = FILL && stash_done && uniform_u32(*stash_done) != 0;
  const uint32_t total = uniform_u32(tp[G]);
  uint32_t next = blockIdx.x * kTileWaves + wave;
  while (true) {
    uint32_t item = next;
    if (persistent) {
      if (lane == 0) item = atomicAdd(ticket, 1u);
      item = uniform_u32(__shfl(item, 0, kWave));
    }
    if (item >= total) break;
    next = total;  // without a ticket a wavefront takes one tile
    const uint32_t g = uniform_u32(tmap[item]);
    const uint32_t inst = g / DDM_MAX_D, k = g % DDM_MAX_D;
    const BInst& b = I[inst];
    const uint32_t qpt = uniform_u32(b.qpt);
    const uint32_t lt = item - uniform_u32(tp[g]);
    const uint32_t gs = uniform_u32(gcount[g]);
    const uint32_t qbeg = uniform_u32(gstart[g]) + lt * qpt;
    const uint32_t nq = min(qpt, gs - lt * qpt);
    const uint32_t dd = uniform_u32(b.d);
    if (skip_multi && dd > 1) continue;
    switch (dd) {
      case 1:
        tile_body<1, FILL, STASH>(b.T, b.u_lo, b.u_hi, b.m, perm, b.qbase, k, qbeg, nq, O,
                                  s_cand[wave], s_cid[wave], s_q[wave], lane, item);
        break;
      case 2:
        tile_body<2, FILL, STASH>(b.T, b.u_lo, b.u_hi, b.m, perm, b.qbase, k, qbeg, nq, O,
                                  s_cand[wave], s_cid[wave], s_q[wave], lane, item);
        break;
      case 3:
        tile_body<3, FILL, STASH>(b.T, b.u_lo, b.u_hi, b.m, perm, b.qbase, k, qbeg, nq, O,
                                  s_cand[wave], s_cid[wave], s_q[wave], lane, item);
        break;
      default:
        tile_body<4, FILL, STASH>(b.T, b.u_lo, b.u_hi, b.m, perm, b.qbase, k, qbeg, nq, O,
                                  s_cand[wave], s_cid[wave], s_q[wave], lane, item);
        break;
    }
    wave_sync();
  }
}

// capacity and input check (one thread): status and total for the host
// With a stash (snext non-null), *stash_done = 1 if the check passed and
// the stash holds every hit of the count traversal (then the stash scatter
// places the pairs of the instances with d > 1 and the fill skips them).
__global__ void b_status_kernel(const BInst* __restrict__ I, uint32_t count,
                                const uint64_t* __restrict__ off, uint32_t M, uint64_t capacity,
                                uint32_t* __restrict__ status, uint64_t* __restrict__ words,
                                const uint32_t* __restrict__ snext,
                                uint32_t* __restrict__ stash_done) {
  if (threadIdx.x != 0) return;
  const uint64_t total = off[M];
  uint32_t st = total > capacity ? kBatchStatusCapacity : 0u;
  for (uint32_t i = 0; i < count; ++i)
    if (*I[i].flag) st |= kBatchStatusInput;
  *status = st;
  if (snext) *stash_done = (st == 0 && snext[kStashSlices] == 0) ? 1u : 0u;
  words[0] = total;
  words[1] = st;
}

// stashed hits to out[off[gj] + rank]: first the static chunks of the count
// traversal's tiles, then, slice by slice, the counted chunks in use (their
// tile is recorded per chunk); a chunk's tile gives its group and instance,
// which turn the instance-local update index of the key into the global one
__global__ __launch_bounds__(256) void b_stash_scatter_kernel(
    const BInst* __restrict__ I, uint32_t G, uint32_t M, const uint32_t* __restrict__ tpc,
    const uint32_t* __restrict__ tmapc, const uint64_t* __restrict__ skey,
    const uint32_t* __restrict__ srank, const uint32_t* __restrict__ sused,
    const uint32_t* __restrict__ sowner, const uint32_t* __restrict__ snext, uint32_t sfirst,
    uint32_t sslice, const uint32_t* __restrict__ stash_done, const uint64_t* __restrict__ off,
    uint64_t* __restrict__ out) {
  if (uniform_u32(*stash_done) == 0) return;
  const uint64_t nthr = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t g0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  auto place = [&](uint64_t e, uint32_t tile) {
    const uint32_t c = (uint32_t)(e / kStashChunk);
    if ((uint32_t)(e % kStashChunk) >= sused[c]) return;
    const uint64_t key = skey[e];
    const uint32_t inst = tmapc[tile] / DDM_MAX_D;
    const uint32_t gj = I[inst].qbase + (uint32_t)(key >> 32);
    if (gj >= M) return;
    const uint64_t dst = off[gj] + srank[e];
    if (dst < off[gj + 1]) out[dst] = key;
  };
  const uint32_t tiles = tpc[G];
  const uint64_t nst = (uint64_t)tiles * kStashStatic * kStashChunk;
  for (uint64_t e = g0; e < nst; e += nthr)
    place(e, (uint32_t)(e / ((uint64_t)kStashStatic * kStashChunk)));
  for (uint32_t sl = 0; sl < kStashSlices; ++sl) {
    const uint64_t c0 = (uint64_t)sfirst + (uint64_t)sl * sslice;
    const uint64_t c1 = min<uint64_t>(snext[sl], c0 + sslice);
    const uint64_t ne = (c1 - c0) * kStashChunk;
    for (uint64_t i = g0; i < ne; i += nthr) {
      const uint64_t e = c0 * kStashChunk + i;
      place(e, sowner[e / kStashChunk]);
    }
  }
}

// after a failed check every segment is emptied, so that the segment sort
// touches no output
__global__ __launch_bounds__(256) void b_clear_kernel(const uint32_t* __restrict__ status,
                                                     uint64_t* __restrict__ off, uint32_t M) {
  if (uniform_u32(*status) == 0) return;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j <= M; j += gridDim.x * blockDim.x)
    off[j] = 0;
}

// per-instance output ranges (before a failed check empties them, the
// check kernel has already recorded the total)
__global__ void b_ranges_kernel(const BInst* __restrict__ I, uint32_t count,
                                const uint64_t* __restrict__ off, uint64_t* __restrict__ ranges) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) ranges[i] = off[I[i].qbase];
  if (i == 0 && count > 0) ranges[count] = off[I[count - 1].qbase + I[count - 1].m];
}

}  // namespace ddm

using namespace ddm;

struct ddm_batch {
  int device = 0;
  uint32_t count = 0;
  uint32_t M = 0;         // total updates
  uint32_t B = 0;         // total buckets
  uint32_t G = 0;         // groups = count * DDM_MAX_D
  uint32_t nmax = 0;      // largest n
  uint64_t elems = 0;     // sum of d n
  uint64_t capacity = 0;
  uint64_t* out = nullptr;
  ddm_batch_opts opts{};
  uint32_t grid = 0;      // persistent traversal workgroups
  char* mem = nullptr;    // one device block for everything
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipStream_t last = nullptr;
  uint64_t* host_words = nullptr;  // pinned: total, status, ranges[count+1]
  // device pointers into mem
  BInst* inst = nullptr;
  TreeJob* jobs = nullptr;
  uint32_t ntrees = 0, index_items = 0;
  uint2* lowmap = nullptr;
  uint32_t nlow = 0;
  std::vector<std::pair<uint2*, uint32_t>> highmaps;  // per pass S = 11, 22, ...
  uint2* probemap = nullptr;
  uint32_t nprobe = 0;
  SortArr* sarr = nullptr;
  uint32_t narr = 0, ntiles = 0;
  uint32_t* tile_map = nullptr;
  uint32_t* hist = nullptr;
  uint8_t* kstar = nullptr;
  uint32_t *bucket = nullptr, *rank = nullptr, *perm = nullptr, *cnt = nullptr;
  uint32_t* bhist = nullptr;
  uint64_t* boff = nullptr;
  uint64_t* off = nullptr;
  uint64_t* scan_tmp_b = nullptr;
  uint64_t* scan_tmp_q = nullptr;
  uint32_t *gstart = nullptr, *gcount = nullptr, *tpc = nullptr, *tpf = nullptr;
  uint32_t* lists = nullptr;
  uint32_t* tickets = nullptr;  // [2]; lists counters follow the lists
  uint32_t* tmapc = nullptr;    // tile -> group, count and fill traversals
  uint32_t* tmapf = nullptr;
  uint32_t tiles_max = 0;       // bound of the tiles of either traversal
  uint32_t* status = nullptr;
  uint64_t* words = nullptr;   // total, status, ranges[count+1]
  uint32_t* zero_base = nullptr;  // contiguous words cleared per run
  uint32_t nzero = 0;
  uint32_t* list_counters = nullptr;  // two words in the cleared block
  bool counted = false;               // ddm_batch_count ran, ddm_batch_fill may follow
  // the count traversal's stash of hits (capacity > 0, some instance d > 1)
  bool stash = false;
  uint64_t* skey = nullptr;
  uint32_t *srank = nullptr, *sused = nullptr, *sowner = nullptr, *snext = nullptr;
  uint32_t* stash_done = nullptr;
  uint32_t sfirst = 0, sslice = 0, smax = 0;
};

namespace ddm {
ddm_status ensure_segsort_attr();

// count half: trees, probe, order, count traversal, offsets, ranges
static ddm_status batch_count_half(ddm_batch* b, hipStream_t s) {
  // clear counters, histograms, flags and length bounds
  b_reset_kernel<<<(b->nzero + 255) / 256, 256, 0, s>>>(b->zero_base, b->nzero);
  DDM_LAUNCHED("b_reset_kernel");
  b_keys_kernel<<<(unsigned)((b->elems + 255) / 256), 256, 0, s>>>(b->inst, b->count, b->elems);
  DDM_LAUNCHED("b_keys_kernel");
  ddm_status r = radix_sort_batch(b->sarr, b->narr, b->tile_map, b->ntiles, b->hist, 0, 4, s);
  if (r != DDM_OK) return r;
  b_index_kernel<<<dim3((b->index_items + 255) / 256, b->ntrees), 256, 0, s>>>(b->jobs);
  DDM_LAUNCHED("b_index_kernel");
  b_tree_low_kernel<<<b->nlow, kTreeThreads, 0, s>>>(b->jobs, b->lowmap);
  DDM_LAUNCHED("b_tree_low_kernel");
  uint32_t S = kChunkLog;
  for (auto& hm : b->highmaps) {
    b_tree_high_kernel<<<hm.second, kTreeThreads, 0, s>>>(b->jobs, hm.first, S);
    DDM_LAUNCHED("b_tree_high_kernel");
    S += kChunkLog;
  }
  b_probe_kernel<<<b->nprobe, kProbeThreads, 0, s>>>(b->inst, b->probemap, b->kstar, b->bucket,
                                                     b->rank, b->bhist, b->cnt);
  DDM_LAUNCHED("b_probe_kernel");
  r = scan_u32_u64(b->bhist, b->boff, b->B, b->scan_tmp_b, s);
  if (r != DDM_OK) return r;
  b_scatter_kernel<<<(b->M + 255) / 256, 256, 0, s>>>(b->bucket, b->rank, b->M, b->boff, b->perm);
  DDM_LAUNCHED("b_scatter_kernel");
  b_groups_kernel<<<1, 1024, 0, s>>>(b->inst, b->count, b->boff, b->gstart, b->gcount, b->tpc,
                                     b->tpf, b->stash ? b->snext : nullptr, b->sfirst,
                                     b->sslice);
  DDM_LAUNCHED("b_groups_kernel");
  b_tilemap_kernel<<<(b->tiles_max + 255) / 256, 256, 0, s>>>(b->G, b->tpc, b->tmapc,
                                                               b->tiles_max);
  DDM_LAUNCHED("b_tilemap_kernel");
  b_tilemap_kernel<<<(b->tiles_max + 255) / 256, 256, 0, s>>>(b->G, b->tpf, b->tmapf,
                                                               b->tiles_max);
  DDM_LAUNCHED("b_tilemap_kernel");
  {
    ProfScope ps("batch_traverse_count", s);
    SegOut O{};
    O.cnt = b->cnt;
    if (b->stash) {
      O.skey = b->skey;
      O.srank = b->srank;
      O.sused = b->sused;
      O.sowner = b->sowner;
      O.snext = b->snext;
      O.sfirst = b->sfirst;
      O.sslice = b->sslice;
      b_traverse_kernel<false, true><<<b->grid, kTileWaves * kWave, 0, s>>>(
          b->inst, b->G, b->tpc, b->tmapc, b->gstart, b->gcount, b->perm, b->tickets,
          b->opts.waves_per_cu, b->status, O, nullptr);
    } else {
      b_traverse_kernel<false><<<b->grid, kTileWaves * kWave, 0, s>>>(
          b->inst, b->G, b->tpc, b->tmapc, b->gstart, b->gcount, b->perm, b->tickets,
          b->opts.waves_per_cu, b->status, O, nullptr);
    }
    DDM_LAUNCHED("b_traverse_kernel");
  }
  r = scan_u32_u64(b->cnt, b->off, b->M, b->scan_tmp_q, s);
  if (r != DDM_OK) return r;
  b_ranges_kernel<<<(b->count + 1 + 255) / 256, 256, 0, s>>>(b->inst, b->count, b->off,
                                                             b->words + 2);
  DDM_LAUNCHED("b_ranges_kernel");
  return DDM_OK;
}

// fill half: capacity and validity check, fill traversal, segment sort into
// b->out (b->capacity keys)
static ddm_status batch_fill_half(ddm_batch* b, hipStream_t s) {
  b_status_kernel<<<1, 64, 0, s>>>(b->inst, b->count, b->off, b->M, b->capacity, b->status,
                                   b->words, b->stash ? b->snext : nullptr, b->stash_done);
  DDM_LAUNCHED("b_status_kernel");
  b_clear_kernel<<<256, 256, 0, s>>>(b->status, b->off, b->M);
  DDM_LAUNCHED("b_clear_kernel");
  if (b->stash) {
    ProfScope ps("batch_stash_scatter", s);
    b_stash_scatter_kernel<<<2048, 256, 0, s>>>(b->inst, b->G, b->M, b->tpc, b->tmapc, b->skey,
                                                b->srank, b->sused, b->sowner, b->snext,
                                                b->sfirst, b->sslice, b->stash_done, b->off,
                                                b->out);
    DDM_LAUNCHED("b_stash_scatter_kernel");
  }
  {
    ProfScope ps("batch_traverse_fill", s);
    SegOut O{};
    O.base = b->off;
    O.out = b->out;
    b_traverse_kernel<true><<<b->grid, kTileWaves * kWave, 0, s>>>(
        b->inst, b->G, b->tpf, b->tmapf, b->gstart, b->gcount, b->perm, b->tickets + 1,
        b->opts.waves_per_cu, b->status, O, b->stash ? b->stash_done : nullptr);
    DDM_LAUNCHED("b_traverse_kernel");
  }
  return sort_segments_inplace(b->off, b->M, b->out, b->nmax, b->lists, b->list_counters, s);
}

static ddm_status batch_enqueue(ddm_batch* b, hipStream_t s) {
  ddm_status r = batch_count_half(b, s);
  if (r != DDM_OK) return r;
  return batch_fill_half(b, s);
}

}  // namespace ddm

static size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

extern "C" ddm_status ddm_batch_create(const ddm_batch_instance* inst, uint32_t count,
                                       uint64_t* out_pairs, uint64_t capacity,
                                       const ddm_batch_opts* opts, ddm_batch** out_batch) {
  set_detail("");
  if (!out_batch || (count && !inst)) {
    set_detail("ddm_batch_create: NULL argument");
    return DDM_E_INVALID_ARG;
  }
  *out_batch = nullptr;
  if (count == 0 || count > kBatchMaxInstances) {
    set_detail("ddm_batch_create: count must be in [1, DDM_BATCH_MAX_INSTANCES]");
    return DDM_E_INVALID_ARG;
  }
  if (capacity && !out_pairs) {
    set_detail("ddm_batch_create: NULL output with nonzero capacity");
    return DDM_E_INVALID_ARG;
  }
  ddm_batch_opts o{};
  if (opts) o = *opts;
  for (int i = 0; i < 5; ++i)
    if (o.reserved[i]) {
      set_detail("ddm_batch_opts: reserved fields must be zero");
      return DDM_E_INVALID_ARG;
    }
  if (o.qpt == 0) o.qpt = 64;
  if (o.qpt != 64 && o.qpt != 32 && o.qpt != 16) {
    set_detail("ddm_batch_opts: qpt must be 16, 32 or 64");
    return DDM_E_INVALID_ARG;
  }
  if (o.waves_per_cu > 64) {
    set_detail("ddm_batch_opts: waves_per_cu must be at most 64");
    return DDM_E_INVALID_ARG;
  }
  uint64_t M = 0, elems = 0, Btot = 0;
  uint32_t nmax = 0, ntrees = 0, narr = 0, ntiles = 0, nlow = 0, nprobe = 0, items = kQuant;
  uint32_t maxH = 0;
  uint64_t tiles_max = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const ddm_batch_instance& q = inst[i];
    if (q.d < 1 || q.d > DDM_MAX_D || q.n == 0 || q.m == 0 || !q.sub_lo || !q.sub_hi ||
        !q.upd_lo || !q.upd_hi || q.n >= (1u << 20) ||
        (q.qpt != 0 && q.qpt != 16 && q.qpt != 32 && q.qpt != 64)) {
      set_detail("ddm_batch_create: every instance needs 1 <= d <= DDM_MAX_D, "
                 "0 < n < 2^20, m > 0, coordinate pointers and qpt in {0, 16, 32, 64}");
      return DDM_E_INVALID_ARG;
    }
    uint32_t H = 0;
    while (((1ull << H) - 1) < q.n) ++H;
    maxH = std::max(maxH, H);
    M += q.m;
    elems += (uint64_t)q.d * q.n;
    nmax = std::max(nmax, q.n);
    Btot += (uint64_t)q.d * std::max<uint32_t>(1, (q.m + 7) / 8);
    ntrees += q.d;
    const uint32_t tiles = (q.n + kSortTile - 1) / kSortTile;
    narr += q.d + (q.d == 1 ? 1 : 0);
    ntiles += tiles * (q.d + (q.d == 1 ? 1 : 0));
    const uint32_t P = (uint32_t)((1ull << H) - 1);
    nlow += q.d * ((P + 1 + kChunk - 1) / kChunk);
    nprobe += (q.m + kProbeThreads - 1) / kProbeThreads;
    items = std::max(items, (q.n + 63) / 64);
    const uint32_t qq = q.qpt ? q.qpt : o.qpt;
    tiles_max += (q.m + qq - 1) / qq + q.d;  // at most one partial tile per group
  }
  if (M >= (1ull << 31) || Btot >= (1ull << 31)) {
    set_detail("ddm_batch_create: too many updates");
    return DDM_E_INVALID_ARG;
  }
  ddm_batch* b = new (std::nothrow) ddm_batch();
  if (!b) return DDM_E_NOMEM;
  b->count = count;
  b->M = (uint32_t)M;
  b->B = (uint32_t)Btot;
  b->G = count * DDM_MAX_D;
  b->nmax = nmax;
  b->elems = elems;
  b->capacity = capacity;
  b->out = out_pairs;
  b->opts = o;
  b->ntrees = ntrees;
  b->narr = narr;
  b->ntiles = ntiles;
  b->nlow = nlow;
  b->nprobe = nprobe;
  b->index_items = items;
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipGetDevice", __FILE__, __LINE__);
  }
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
  b->tiles_max = (uint32_t)std::min<uint64_t>(tiles_max, 0xffffffffull);
  b->grid = o.waves_per_cu
                ? std::max<uint32_t>(1, (uint32_t)cus * o.waves_per_cu / kTileWaves)
                : std::max<uint32_t>(1, (b->tiles_max + kTileWaves - 1) / kTileWaves);

  // ---- host-side layout ----
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t at = cur;
    cur += al256(bytes);
    return at;
  };
  std::vector<BInst> hin(count);
  std::vector<TreeJob> hjobs;
  std::vector<uint2> hlow, hprobe;
  std::vector<std::vector<uint2>> hhigh;
  std::vector<SortArr> hs;
  std::vector<uint32_t> htile;
  // offsets of per-instance storage (relative to mem), patched to pointers
  struct InstOff {
    size_t rec[DDM_MAX_D], mx[DDM_MAX_D], bm[DDM_MAX_D], sidx_lo[DDM_MAX_D], quant[DDM_MAX_D];
    size_t id, klo, khi, sidx_hi, maxlen, flag, klo_tmp, khi_tmp, val_tmp;
    uint32_t H, P, C, ns;
  };
  std::vector<InstOff> io(count);
  const size_t o_inst = take(sizeof(BInst) * count);
  uint64_t qbase = 0, bbase = 0, ebase = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const ddm_batch_instance& q = inst[i];
    InstOff& f = io[i];
    uint32_t H = 0;
    while (((1ull << H) - 1) < q.n) ++H;
    f.H = H;
    f.P = (uint32_t)((1ull << H) - 1);
    f.C = std::max<uint32_t>(1u, (uint32_t)(((uint64_t)f.P + 1) >> kBlockLog));
    f.ns = (q.n + 63) / 64;
    for (uint32_t k = 0; k < q.d; ++k) {
      f.rec[k] = take(sizeof(float) * (size_t)(q.n + 1) * 2 * q.d);
      f.mx[k] = take(sizeof(float) * ((size_t)f.P + 1));
      f.bm[k] = take(sizeof(float) * f.C);
      f.sidx_lo[k] = take(sizeof(uint32_t) * f.ns);
      f.quant[k] = take(sizeof(uint32_t) * kQuant);
    }
    f.id = take(sizeof(uint32_t) * (size_t)(q.n + 1) * q.d);
    f.klo = take(sizeof(uint32_t) * (size_t)q.n * q.d);
    f.khi = q.d == 1 ? take(sizeof(uint32_t) * q.n) : 0;
    f.sidx_hi = q.d == 1 ? take(sizeof(uint32_t) * f.ns) : 0;
    f.klo_tmp = take(sizeof(uint32_t) * (size_t)q.n * q.d);
    f.val_tmp = take(sizeof(uint32_t) * (size_t)q.n * q.d);
    f.khi_tmp = q.d == 1 ? take(sizeof(uint32_t) * q.n) : 0;
    BInst& bi = hin[i];
    bi.s_lo = q.sub_lo;
    bi.s_hi = q.sub_hi;
    bi.u_lo = q.upd_lo;
    bi.u_hi = q.upd_hi;
    bi.n = q.n;
    bi.m = q.m;
    bi.d = q.d;
    bi.qbase = (uint32_t)qbase;
    bi.bbase = (uint32_t)bbase;
    bi.nb = std::max<uint32_t>(1, (q.m + 7) / 8);
    bi.qpt = q.qpt ? q.qpt : o.qpt;
    bi.ebase = ebase;
    qbase += q.m;
    bbase += (uint64_t)q.d * bi.nb;
    ebase += (uint64_t)q.d * q.n;
  }
  // words cleared at every run: flags + length bounds (2 + DDM_MAX_D per
  // instance), bucket histogram, tickets, segment-list counters
  const size_t zero_words = (size_t)count * (2 + DDM_MAX_D) + Btot + 2 + 2;
  const size_t o_zero = take(sizeof(uint32_t) * zero_words);
  const size_t o_jobs = take(sizeof(TreeJob) * ntrees);
  const size_t o_low = take(sizeof(uint2) * nlow);
  // high passes
  std::vector<size_t> o_high;
  for (uint32_t S = kChunkLog; S < maxH; S += kChunkLog) {
    std::vector<uint2> v;
    uint32_t t = 0;
    for (uint32_t i = 0; i < count; ++i)
      for (uint32_t k = 0; k < inst[i].d; ++k, ++t)
        if (S < io[i].H) {
          const uint32_t q_end = (io[i].P >> S) + 1;
          for (uint32_t c = 0; c < (q_end + kChunk - 1) / kChunk; ++c) v.push_back(make_uint2(t, c));
        }
    o_high.push_back(take(sizeof(uint2) * std::max<size_t>(1, v.size())));
    hhigh.push_back(v);
  }
  const size_t o_probe = take(sizeof(uint2) * nprobe);
  const size_t o_sarr = take(sizeof(SortArr) * narr);
  const size_t o_tile = take(sizeof(uint32_t) * ntiles);
  const size_t o_hist = take(sizeof(uint32_t) * 256 * (size_t)ntiles);
  const size_t o_kstar = take(M);
  const size_t o_bucket = take(sizeof(uint32_t) * M);
  const size_t o_rank = take(sizeof(uint32_t) * M);
  const size_t o_perm = take(sizeof(uint32_t) * M);
  const size_t o_cnt = take(sizeof(uint32_t) * M);
  const size_t o_boff = take(sizeof(uint64_t) * (Btot + 1));
  const size_t o_off = take(sizeof(uint64_t) * (M + 1));
  const size_t o_stb = take(sizeof(uint64_t) * scan_tmp_words((uint32_t)Btot));
  const size_t o_stq = take(sizeof(uint64_t) * scan_tmp_words((uint32_t)M));
  const size_t o_groups = take(sizeof(uint32_t) * (4 * (size_t)b->G + 2));
  const size_t o_tmapc = take(sizeof(uint32_t) * tiles_max);
  const size_t o_tmapf = take(sizeof(uint32_t) * tiles_max);
  const size_t o_lists = take(sizeof(uint32_t) * 2 * M);
  const size_t o_status = take(sizeof(uint32_t) * 4);
  const size_t o_words = take(sizeof(uint64_t) * (count + 3));
  // the stash: static chunks of every possible count tile, then slices for
  // the capacity (or 4 hits per update) plus a partly used chunk per tile
  bool any_multi = false;
  for (uint32_t i = 0; i < count; ++i) any_multi = any_multi || inst[i].d > 1;
  b->stash = any_multi && capacity > 0 && capacity <= kStashMaxEntries &&
             capacity <= kStashMaxPerUpdate * M;
  size_t o_skey = 0, o_srank = 0, o_sused = 0, o_sowner = 0, o_snext = 0;
  if (b->stash) {
    const uint64_t dyn = std::min<uint64_t>(std::max<uint64_t>(capacity, 4ull * M),
                                            kStashMaxEntries);
    const uint64_t cdyn =
        (dyn + kStashChunk - 1) / kStashChunk + (uint64_t)b->tiles_max * kStashGrab + 1024;
    const uint64_t sfirst = (uint64_t)b->tiles_max * kStashStatic;
    const uint64_t sslice = (cdyn + kStashSlices - 1) / kStashSlices;
    const uint64_t smax = sfirst + sslice * kStashSlices;
    if (smax >= (1ull << 32) / kStashChunk) {
      b->stash = false;
    } else {
      b->sfirst = (uint32_t)sfirst;
      b->sslice = (uint32_t)sslice;
      b->smax = (uint32_t)smax;
      o_skey = take(sizeof(uint64_t) * smax * kStashChunk);
      o_srank = take(sizeof(uint32_t) * smax * kStashChunk);
      o_sused = take(sizeof(uint32_t) * smax);
      o_sowner = take(sizeof(uint32_t) * smax);
      o_snext = take(sizeof(uint32_t) * (kStashSlices + 2));
    }
  }
  const size_t total = cur;

  b->mem = dev_alloc(total, nullptr);
  if (!b->mem) {
    delete b;
    set_detail("ddm_batch_create: device allocation failed");
    return DDM_E_NOMEM;
  }
  char* base = b->mem;
  auto P32 = [&](size_t off) { return (uint32_t*)(base + off); };
  auto PF = [&](size_t off) { return (float*)(base + off); };
  // zero block layout: [flags count][maxlen count*DDM_MAX_D][bhist Btot][tickets 2][list counters 2]
  uint32_t* zb = P32(o_zero);
  b->zero_base = zb;
  b->nzero = (uint32_t)zero_words;
  uint32_t* zflags = zb;
  uint32_t* zmaxlen = zb + count * 2;
  b->bhist = zmaxlen + (size_t)count * DDM_MAX_D;
  b->tickets = b->bhist + Btot;
  b->list_counters = b->tickets + 2;

  uint32_t t = 0, a = 0, tile0 = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const ddm_batch_instance& q = inst[i];
    InstOff& f = io[i];
    BInst& bi = hin[i];
    bi.flag = (int32_t*)(zflags + 2 * i);
    bi.klo = P32(f.klo);
    bi.khi = q.d == 1 ? P32(f.khi) : nullptr;
    bi.idb = P32(f.id);
    TreeDev& T = bi.T;
    for (uint32_t k = 0; k < q.d; ++k) {
      T.rec[k] = PF(f.rec[k]);
      T.maxhi[k] = PF(f.mx[k]);
      T.id[k] = P32(f.id) + (size_t)k * (q.n + 1);
      T.skey_lo[k] = P32(f.klo) + (size_t)k * q.n;
      T.skey_hi[k] = q.d == 1 ? P32(f.khi) : nullptr;
      T.bmax[k] = PF(f.bm[k]);
      T.sidx_lo[k] = P32(f.sidx_lo[k]);
      T.sidx_hi[k] = q.d == 1 ? P32(f.sidx_hi) : nullptr;
      T.quant[k] = P32(f.quant[k]);
    }
    T.maxlen = (const float*)(zmaxlen + (size_t)i * DDM_MAX_D);
    T.n = q.n;
    T.d = q.d;
    T.H = f.H;
    T.ns = f.ns;
    const uint32_t tiles = (q.n + kSortTile - 1) / kSortTile;
    for (uint32_t k = 0; k < q.d; ++k, ++t) {
      TreeJob j{};
      j.s_lo = q.sub_lo;
      j.s_hi = q.sub_hi;
      j.rec = PF(f.rec[k]);
      j.maxhi = PF(f.mx[k]);
      j.bmax = PF(f.bm[k]);
      j.id = T.id[k];
      j.skey_lo = T.skey_lo[k];
      j.skey_hi = T.skey_hi[k];
      j.sidx_lo = P32(f.sidx_lo[k]);
      j.sidx_hi = q.d == 1 ? P32(f.sidx_hi) : nullptr;
      j.quant = P32(f.quant[k]);
      j.maxlen_bits = zmaxlen + (size_t)i * DDM_MAX_D + k;
      j.n = q.n;
      j.d = q.d;
      j.k = k;
      j.P = f.P;
      j.C = f.C;
      j.H = f.H;
      j.ns = f.ns;
      hjobs.push_back(j);
      for (uint32_t c = 0; c < (f.P + 1 + kChunk - 1) / kChunk; ++c) hlow.push_back(make_uint2(t, c));
      SortArr sa{};
      sa.k[0] = P32(f.klo) + (size_t)k * q.n;
      sa.k[1] = P32(f.klo_tmp) + (size_t)k * q.n;
      sa.v[0] = P32(f.id) + (size_t)k * (q.n + 1) + 1;
      sa.v[1] = P32(f.val_tmp) + (size_t)k * q.n;
      sa.n = q.n;
      sa.tile0 = tile0;
      hs.push_back(sa);
      for (uint32_t x = 0; x < tiles; ++x) htile.push_back(a);
      tile0 += tiles;
      ++a;
    }
    if (q.d == 1) {
      SortArr sh{};
      sh.k[0] = P32(f.khi);
      sh.k[1] = P32(f.khi_tmp);
      sh.n = q.n;
      sh.tile0 = tile0;
      hs.push_back(sh);
      for (uint32_t x = 0; x < tiles; ++x) htile.push_back(a);
      tile0 += tiles;
      ++a;
    }
    for (uint32_t x = 0; x < (q.m + kProbeThreads - 1) / kProbeThreads; ++x)
      hprobe.push_back(make_uint2(i, x));
  }
  b->inst = (BInst*)(base + o_inst);
  b->jobs = (TreeJob*)(base + o_jobs);
  b->lowmap = (uint2*)(base + o_low);
  for (size_t x = 0; x < hhigh.size(); ++x)
    b->highmaps.push_back({(uint2*)(base + o_high[x]), (uint32_t)hhigh[x].size()});
  b->probemap = (uint2*)(base + o_probe);
  b->sarr = (SortArr*)(base + o_sarr);
  b->tile_map = P32(o_tile);
  b->hist = P32(o_hist);
  b->kstar = (uint8_t*)(base + o_kstar);
  b->bucket = P32(o_bucket);
  b->rank = P32(o_rank);
  b->perm = P32(o_perm);
  b->cnt = P32(o_cnt);
  b->boff = (uint64_t*)(base + o_boff);
  b->off = (uint64_t*)(base + o_off);
  b->scan_tmp_b = (uint64_t*)(base + o_stb);
  b->scan_tmp_q = (uint64_t*)(base + o_stq);
  uint32_t* gr = P32(o_groups);
  b->gstart = gr;
  b->gcount = gr + b->G;
  b->tpc = gr + 2 * (size_t)b->G;
  b->tpf = gr + 3 * (size_t)b->G + 1;
  b->lists = P32(o_lists);
  b->tmapc = P32(o_tmapc);
  b->tmapf = P32(o_tmapf);
  b->status = P32(o_status);
  b->words = (uint64_t*)(base + o_words);
  if (b->stash) {
    b->skey = (uint64_t*)(base + o_skey);
    b->srank = P32(o_srank);
    b->sused = P32(o_sused);
    b->sowner = P32(o_sowner);
    b->snext = P32(o_snext);
    b->stash_done = b->snext + kStashSlices + 1;
  }

  // ---- upload the static tables ----
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  e = up(b->inst, hin.data(), sizeof(BInst) * count);
  if (e == hipSuccess) e = up(b->jobs, hjobs.data(), sizeof(TreeJob) * hjobs.size());
  if (e == hipSuccess) e = up(b->lowmap, hlow.data(), sizeof(uint2) * hlow.size());
  for (size_t x = 0; x < hhigh.size() && e == hipSuccess; ++x)
    e = up(b->highmaps[x].first, hhigh[x].data(), sizeof(uint2) * hhigh[x].size());
  if (e == hipSuccess) e = up(b->probemap, hprobe.data(), sizeof(uint2) * hprobe.size());
  if (e == hipSuccess) e = up(b->sarr, hs.data(), sizeof(SortArr) * hs.size());
  if (e == hipSuccess) e = up(b->tile_map, htile.data(), sizeof(uint32_t) * htile.size());
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&b->host_words, sizeof(uint64_t) * (count + 3), hipHostMallocDefault);
  if (e == hipSuccess && o.use_graph) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess && o.use_graph) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess && o.use_graph) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e != hipSuccess) {
    ddm_status r = hip_fail(e, "ddm_batch_create", __FILE__, __LINE__);
    ddm_batch_free(b);
    return r;
  }
  ddm_status r = ensure_segsort_attr();
  if (r != DDM_OK) {
    ddm_batch_free(b);
    return r;
  }
  *out_batch = b;
  return DDM_OK;
}

extern "C" ddm_status ddm_batch_run(ddm_batch* b, void* stream) {
  set_detail("");
  if (!b) return DDM_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  b->last = s;
  if (!b->opts.use_graph) return batch_enqueue(b, s);
  if (!b->exec) {
    DDM_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    ddm_status r = batch_enqueue(b, b->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (r != DDM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
    b->graph = g;
    DDM_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  }
  // order the replay after the caller's stream and the caller's stream after it
  DDM_HIP(hipEventRecord(b->ev_in, s));
  DDM_HIP(hipStreamWaitEvent(b->cap, b->ev_in, 0));
  DDM_HIP(hipGraphLaunch(b->exec, b->cap));
  DDM_HIP(hipEventRecord(b->ev_out, b->cap));
  DDM_HIP(hipStreamWaitEvent(s, b->ev_out, 0));
  return DDM_OK;
}

extern "C" ddm_status ddm_batch_result(ddm_batch* b, uint64_t* total, uint64_t* ranges) {
  set_detail("");
  if (!b) return DDM_E_INVALID_ARG;
  hipStream_t s = b->last;
  DDM_HIP(hipMemcpyAsync(b->host_words, b->words, sizeof(uint64_t) * (b->count + 3),
                         hipMemcpyDeviceToHost, s));
  DDM_HIP(hipStreamSynchronize(s));
  if (total) *total = b->host_words[0];
  const uint64_t st = b->host_words[1];
  if (ranges)
    for (uint32_t i = 0; i <= b->count; ++i) ranges[i] = b->host_words[2 + i];
  if (st & kBatchStatusInput) {
    set_detail("a batch instance has NaN/inf coordinates or lo > hi");
    return DDM_E_INVALID_INPUT;
  }
  if (st & kBatchStatusCapacity) {
    set_detail("batch result larger than capacity");
    return DDM_E_CAPACITY;
  }
  return DDM_OK;
}

extern "C" ddm_status ddm_batch_count(ddm_batch* b, void* stream, uint64_t* total,
                                      uint64_t* ranges) {
  set_detail("");
  if (!b || !total) return DDM_E_INVALID_ARG;
  if (b->opts.use_graph) {
    set_detail("ddm_batch_count: only for batches created without a graph");
    return DDM_E_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  b->last = s;
  ddm_status r = batch_count_half(b, s);
  if (r != DDM_OK) return r;
  // validity only: the capacity is given to ddm_batch_fill
  b_status_kernel<<<1, 64, 0, s>>>(b->inst, b->count, b->off, b->M, ~0ull, b->status, b->words,
                                   nullptr, nullptr);
  DDM_LAUNCHED("b_status_kernel");
  DDM_HIP(hipMemcpyAsync(b->host_words, b->words, sizeof(uint64_t) * (b->count + 3),
                         hipMemcpyDeviceToHost, s));
  DDM_HIP(hipStreamSynchronize(s));
  *total = b->host_words[0];
  if (ranges)
    for (uint32_t i = 0; i <= b->count; ++i) ranges[i] = b->host_words[2 + i];
  b->counted = true;
  if (b->host_words[1] & kBatchStatusInput) {
    set_detail("a batch instance has NaN/inf coordinates or lo > hi");
    return DDM_E_INVALID_INPUT;
  }
  return DDM_OK;
}

extern "C" ddm_status ddm_batch_fill(ddm_batch* b, uint64_t* out_pairs, uint64_t capacity,
                                     void* stream) {
  set_detail("");
  if (!b || (capacity && !out_pairs)) return DDM_E_INVALID_ARG;
  if (!b->counted) {
    set_detail("ddm_batch_fill: ddm_batch_count must run first");
    return DDM_E_INVALID_ARG;
  }
  if (b->host_words[0] > capacity) {
    set_detail("batch result larger than capacity");
    return DDM_E_CAPACITY;
  }
  hipStream_t s = (hipStream_t)stream;
  b->last = s;
  b->out = out_pairs;
  b->capacity = capacity;
  b->counted = false;
  return batch_fill_half(b, s);
}

extern "C" void ddm_batch_free(ddm_batch* b) {
  if (!b) return;
  if (b->last) (void)hipStreamSynchronize(b->last);
  if (b->cap) (void)hipStreamSynchronize(b->cap);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->host_words) (void)hipHostFree(b->host_words);
  if (b->mem) dev_free(b->mem, nullptr);
  delete b;
}
