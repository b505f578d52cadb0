// Matching on the device: Algorithm 5 (IntTree-Matching) with Algorithm 4
// (Interval-Query) for every update in parallel, Sec. IV "Parallelizing ITM",
// and the d-dimensional combine of Sec. III-A.
//
// Sequence for m updates against a tree set of d dimensions:
//   1. probe: d = 1 (bits1_kernel): the exact count of every update from
//      two binary searches on sorted lower and upper bounds (the BITS
//      identity recalled in Sec. II), already the final count.  d > 1
//      (probe_kernel): the probe dimension k* with the fewest candidate
//      positions, estimated from quantiles of the sorted lower bounds held
//      in LDS, bounds of those positions, and the update's bucket (k* and
//      its place in tree k*, or a cell of tree positions and the other
//      dimensions) with its rank inside the bucket.
//   2. updates placed in bucket order (a counting sort), cut into tiles of
//      up to 64 updates of one bucket.
//   3. count traversal (d > 1): one wavefront per tile scans the tile's
//      candidate positions of tree k* and tests every candidate in all d
//      dimensions (membership in every per-dimension overlap set is decided
//      by that dimension's own predicate, so the intersection of Sec. III-A
//      is formed without listing the per-dimension sets); the hits are kept
//      when they fit.  The lane form walks Algorithm 4 per update instead.
//   4. exclusive scan of the counts -> segment offsets, total K.
//   5. the kept hits placed, or a fill traversal (the same scan) writing
//      each hit into the update's own segment (each query owns its column
//      of M, so lanes never conflict).
//   6. per-segment sort by subscription id.
// The learned single pass replaces 3-5 by one traversal that writes into
// slots sized by a predictor while counting exactly.
#include "ddm_internal.h"
#include "traverse.h"

#include <algorithm>
#include <mutex>
#include <new>

namespace ddm {

TreeDev tree_dev(const ddm_tree* t);
FeatDev tree_feat(const ddm_tree* t);
ddm_status tree_ensure_features(const ddm_tree* t, hipStream_t s);
const float* predictor_params(const ddm_predictor* p);
float predictor_delta(const ddm_predictor* p);
int predictor_device(const ddm_predictor* p);
const int32_t* tree_flag(const ddm_tree* t);
uint32_t tree_n(const ddm_tree* t);
uint32_t tree_d(const ddm_tree* t);
int tree_device(const ddm_tree* t);

// --------------------------------------------------------------------------
// 1. Probe dimension and update order.
//
// d = 1 (bits1_kernel): the BITS identity recalled in Sec. II gives the exact
// number of closed segments meeting q: c = #{lo <= q.hi} - #{hi < q.lo}
// (lo <= hi holds for every subscription), which is already the final count.
//
// d > 1 (probe_kernel): the probe dimension k* minimises the number of tree
// positions that can hold a candidate, i.e. positions p with
// t <= lo_p <= q.hi where t <= q.lo - maxlen (rounded down): a segment that
// meets q has hi >= q.lo and lo >= hi - maxlen >= t.  The count is estimated
// from kQuant quantiles of the sorted lower bounds held in LDS; any choice of
// k* gives the same pairs, only the work differs.
//
// Both kernels bucket the update by (k*, position of q.hi in tree k*) and
// take its rank inside the bucket from the histogram atomic, so the order is
// a counting sort without a second pass of atomics.
// --------------------------------------------------------------------------
constexpr uint32_t kBucketsPerDim = 8192;
constexpr uint32_t kBuckets = kBucketsPerDim * DDM_MAX_D;
// The rank of an update in its bucket comes from a device-scope atomic on
// the bucket's counter; counters 128 bytes apart (one per cache line), so
// that the atomics of different buckets do not queue on one line (at
// 10^6 boxes all updates fall into the 4096 cells of their probe dimension,
// and with packed counters about a thousand atomics would share each line).
constexpr uint32_t kCntPad = 32;

// d > 1: the first half of a dimension's buckets are ranges of the position
// in tree k*; an update whose candidate range is longer than kCellRange
// positions goes instead to the second half: cells of B0 position ranges
// times B1 ranges (equal numbers of lower bounds, from the quantiles) of
// each other dimension, B0 * B1^(d-1) = kLineBins, so that the updates of a
// tile are close in every dimension and the tile's enclosing box filters
// most candidates before they are tested one by one.  Only very short
// ranges, where scanning dominates, keep the 1-D order.  The shape follows
// the update's estimated range: a tile scans its cell's width plus one
// update's range, so B0 is the power of two nearest to the number of
// ranges of that length in the tree (B1 = 2^e, B0 = kLineBins / 2^(e(d-1))).
// Measured (match, one MI355X): 10^6 boxes d = 2 alpha = 1 0.40 -> 0.30 ms,
// d = 3 0.50 -> 0.25 ms, alpha = 10 1.22 -> 1.00 ms, against a threshold of
// 4096 and fixed shapes.
constexpr uint32_t kLineBins = kBucketsPerDim / 2;
constexpr uint32_t kCellRange = 256;
constexpr float kCellBias = 0.0f;  // log2 of (B0 * range / positions) aimed at

// log2 B1 for an update whose candidate range holds about `best` of the
// kQuant quantile steps (B0 then about kQuant / best), at least 2 cells per
// dimension and at least 16 position ranges
template <int D>
__device__ __forceinline__ uint32_t cell_log2(uint32_t best) {
  const float x = (log2f((float)best) - kCellBias) / (float)(D - 1);
  const int e = (int)floorf(x + 0.5f);
  return (uint32_t)max(1, min(e, 8 / (D - 1)));
}
// the shape of a probe dimension no sampled update takes with cells
__host__ __device__ constexpr uint32_t kCellLog2Default(int D) { return D == 2 ? 3 : D == 3 ? 2 : 1; }

__global__ __launch_bounds__(256) void bits1_kernel(TreeDev T, const float* __restrict__ ulo,
                                                    const float* __restrict__ uhi, uint32_t m,
                                                    uint32_t* __restrict__ cmin,
                                                    uint8_t* __restrict__ kstar,
                                                    uint32_t* __restrict__ bucket,
                                                    uint32_t* __restrict__ rank,
                                                    uint32_t* __restrict__ bhist,
                                                    int32_t* __restrict__ flag) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = j < m;
  bool bad = false;
  if (act) {
    const float a = ulo[j], b = uhi[j];
    bad = !valid_extent(a, b);
    const uint32_t* keys[2] = {T.skey_lo[0], T.skey_hi[0]};
    const uint32_t* idx[2] = {T.sidx_lo[0], T.sidx_hi[0]};
    const uint32_t x[2] = {f2key(b), f2key(a)};
    const bool up[2] = {true, false};
    uint32_t res[2];
    count_2l<2>(keys, idx, x, up, T.n, T.ns, res);
    const uint32_t c = bad ? 0u : res[0] - res[1];
    const uint32_t ph = bad ? 0u : res[0];
    cmin[j] = c;
    kstar[j] = 0;
    const uint32_t bu = min((uint32_t)(((uint64_t)ph * kBucketsPerDim) / ((uint64_t)T.n + 1)),
                            kBucketsPerDim - 1u);
    bucket[j] = bu;
    rank[j] = atomicAdd(&bhist[bu * kCntPad], 1u);
  }
  if (ballot(bad) != 0 && lane_id() == 0) atomicOr(flag, 2);
}

// the probe estimate of update j: the dimension k* with the fewest
// candidate positions (best, in quantile steps), #quantiles <= q.hi there
// (bqa) and its key (bx), the box centre, and whether the extent is invalid
template <int D>
struct ProbeEst {
  uint32_t best, bk, bqa, bqb, bx;
  float mid[D];
  bool bad;
};

// the update's extents (ua, ub: dimension k of update j), loaded before the
// quantiles are (their loads overlap)
template <int D>
struct UpdExt {
  float a[D], b[D];
};
template <int D>
__device__ __forceinline__ UpdExt<D> load_ext(const float* __restrict__ ulo,
                                              const float* __restrict__ uhi, uint32_t m,
                                              uint32_t j) {
  UpdExt<D> e;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    e.a[k] = ulo[(size_t)k * m + j];
    e.b[k] = uhi[(size_t)k * m + j];
  }
  return e;
}

// the kQuant quantiles of every dimension into LDS (sq[k][qslot(i)]), by
// THREADS threads: every load is issued before the first LDS store, so that
// they are in flight together
template <int D, uint32_t THREADS>
__device__ __forceinline__ void load_quant_lds(const TreeDev& T, uint32_t (*sq)[kQuantPad]) {
  static_assert(kQuant % THREADS == 0, "whole rounds");
  constexpr uint32_t Q = kQuant / THREADS;
  uint32_t v[D][Q];
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (uint32_t r = 0; r < Q; ++r) v[k][r] = T.quant[k][r * THREADS + threadIdx.x];
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (uint32_t r = 0; r < Q; ++r) sq[k][qslot(r * THREADS + threadIdx.x)] = v[k][r];
}

template <int D>
__device__ __forceinline__ ProbeEst<D> probe_estimate(const TreeDev& T,
                                                      const uint32_t (*sq)[kQuantPad],
                                                      const UpdExt<D>& e) {
  ProbeEst<D> P;
  P.best = 0xffffffffu;
  P.bk = 0;
  P.bqa = 0;
  P.bqb = 0;
  P.bx = 0;
  P.bad = false;
  uint32_t xh[D], xl[D], qa[D], qb[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float a = e.a[k], b = e.b[k];
    P.bad = P.bad || !valid_extent(a, b);
    P.mid[k] = 0.5f * a + 0.5f * b;
    xh[k] = f2key(b);
    xl[k] = f2key(nextafterf(a - T.maxlen[k], -INFINITY));
    qa[k] = 0;
    qb[k] = 0;
  }
  // the 2D quantile searches (#quantiles <= xh, #quantiles < xl per
  // dimension) advance in lockstep, so their LDS reads overlap
#pragma unroll
  for (uint32_t step = kQuant; step > 0; step >>= 1) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const uint32_t ca = qa[k] + step, cb = qb[k] + step;
      const uint32_t va = ca <= kQuant ? sq[k][qslot(ca - 1)] : 0xffffffffu;
      const uint32_t vb = cb <= kQuant ? sq[k][qslot(cb - 1)] : 0xffffffffu;
      if (ca <= kQuant && va <= xh[k]) qa[k] = ca;
      if (cb <= kQuant && vb < xl[k]) qb[k] = cb;
    }
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const uint32_t est = qa[k] - min(qa[k], qb[k]);
    if (est < P.best) {
      P.best = est;
      P.bk = (uint32_t)k;
      P.bqa = qa[k];
      P.bqb = qb[k];
      P.bx = xh[k];
    }
  }
  return P;
}

template <int D>
__device__ __forceinline__ bool cell_mode(uint32_t best, uint32_t n) {
  return (uint64_t)best * n > (uint64_t)kCellRange * kQuant;
}

// The cell shape of each probe dimension (run by one workgroup of at least
// kShapeSamples threads): the most common cell_log2 over up to
// kShapeSamples updates spread evenly over the set, among those that would
// take that dimension with cells.
// One shape per dimension keeps the cells of different updates from sharing
// buckets while meaning different boxes (a tile that mixed them would scan
// the union of far-apart ranges).
constexpr uint32_t kShapeSamples = 256;

template <int D, uint32_t THREADS>
__device__ __forceinline__ void sample_cell_shape(const TreeDev& T, const float* __restrict__ ulo,
                                                  const float* __restrict__ uhi, uint32_t m,
                                                  uint32_t* __restrict__ shape) {
  static_assert(THREADS >= kShapeSamples, "one sample per thread");
  __shared__ uint32_t sq[D][kQuantPad];
  __shared__ uint32_t hist[D][16];
  const uint32_t S = min(m, kShapeSamples);
  UpdExt<D> e{};
  if (threadIdx.x < S) e = load_ext<D>(ulo, uhi, m, (uint32_t)(((uint64_t)threadIdx.x * m) / S));
  for (uint32_t i = threadIdx.x; i < D * 16; i += THREADS) hist[i / 16][i % 16] = 0;
  load_quant_lds<D, THREADS>(T, sq);
  __syncthreads();
  if (threadIdx.x < kShapeSamples) {
    // (k*, shape) of this lane's sample, or none; counted per wavefront
    // (one LDS add per distinct value, as the samples mostly agree)
    uint32_t key = ~0u;
    if (threadIdx.x < S) {
      const ProbeEst<D> P = probe_estimate<D>(T, sq, e);
      if (!P.bad && cell_mode<D>(P.best, T.n)) key = P.bk * 16u + cell_log2<D>(P.best);
    }
    uint64_t left = ballot(key != ~0u);
    while (left) {
      const uint32_t lead = (uint32_t)__builtin_ctzll(left);
      const uint32_t lk = (uint32_t)__shfl((int)key, (int)lead, kWave);
      const uint64_t same = ballot(key == lk) & left;
      if (lane_id() == lead) atomicAdd(&hist[lk / 16u][lk % 16u], (uint32_t)__popcll(same));
      left &= ~same;
    }
  }
  __syncthreads();
  if (threadIdx.x < D) {
    const uint32_t k = threadIdx.x;
    uint32_t e = kCellLog2Default(D), c = 0;
    for (uint32_t x = 1; x < 16; ++x)
      if (hist[k][x] > c) {
        c = hist[k][x];
        e = x;
      }
    shape[k] = e;
  }
}

constexpr uint32_t kProbeThreads = 1024;
template <int D>
__global__ __launch_bounds__(kProbeThreads) void probe_kernel(TreeDev T, const float* __restrict__ ulo,
                                                     const float* __restrict__ uhi, uint32_t m,
                                                     const uint32_t* __restrict__ shape,
                                                     uint8_t* __restrict__ kstar,
                                                     uint32_t* __restrict__ bucket,
                                                     uint32_t* __restrict__ rank,
                                                     uint32_t* __restrict__ bhist,
                                                     int32_t* __restrict__ flag,
                                                     uint2* __restrict__ pb) {
  __shared__ uint32_t sq[D][kQuantPad];
  const uint32_t j = blockIdx.x * kProbeThreads + threadIdx.x;
  const bool act = j < m;
  UpdExt<D> e{};
  if (act) e = load_ext<D>(ulo, uhi, m, j);
  load_quant_lds<D, kProbeThreads>(T, sq);
  __syncthreads();
  bool bad = false;
  if (act) {
    const ProbeEst<D> P = probe_estimate<D>(T, sq, e);
    bad = P.bad;
    uint32_t bk = P.bk;
    const uint32_t best = P.best, bqa = P.bqa, bx = P.bx;
    // position of q.hi in tree k*, interpolated between its two quantiles
    float fine;
    if (bqa == 0) {
      fine = 0.f;
    } else if (bqa >= kQuant) {
      fine = (float)kQuant - 0.5f;
    } else {
      uint32_t kl = 0, ku = 0;
#pragma unroll
      for (int k = 0; k < D; ++k)
        if ((uint32_t)k == bk) {
          kl = sq[k][qslot(bqa - 1)];
          ku = sq[k][qslot(bqa)];
        }
      const float fr = ku > kl ? (float)(bx - kl) / (float)(ku - kl) : 0.f;
      fine = (float)(bqa - 1) + fminf(fr, 0.999f);
    }
    if (bad) {
      bk = 0;
      fine = 0.f;
    }
    kstar[j] = (uint8_t)bk;
    // bounds of the candidate positions in tree k* from the quantiles
    // quant[i] = skey_lo[floor(i n / kQuant)]: bqb quantiles lie below
    // t = q.lo - maxlen, so at least floor((bqb - 1) n / kQuant) + 1 keys do;
    // bqa quantiles are <= q.hi and quantile bqa is not, so at most
    // floor(bqa n / kQuant) keys are (positions are 1-based)
    {
      const uint32_t qb = P.bqb, qa = bqa;
      const uint32_t lo = qb ? (uint32_t)(((uint64_t)(qb - 1) * T.n) / kQuant) + 1u : 0u;
      const uint32_t hi = qa < kQuant ? (uint32_t)(((uint64_t)qa * T.n) / kQuant) : T.n;
      pb[j] = bad ? make_uint2(1u, 0u) : make_uint2(lo + 1u, hi);
    }
    uint32_t sub;
    if (!bad && cell_mode<D>(best, T.n)) {
      const uint32_t e = shape[bk];
      const uint32_t B1 = 1u << e, B0 = kLineBins >> ((D - 1) * e);
      sub = min((uint32_t)(fine * (float)B0 / (float)kQuant), B0 - 1u);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        if ((uint32_t)k == bk) continue;
        const uint32_t qp = quant_count(sq[k], f2key(P.mid[k]), true);
        sub = sub * B1 + min(qp * B1 / (kQuant + 1u), B1 - 1u);
      }
      sub += kLineBins;
    } else {
      sub = min((uint32_t)(fine * (float)kLineBins / (float)kQuant), kLineBins - 1u);
    }
    const uint32_t bu = bk * kBucketsPerDim + sub;
    bucket[j] = bu;
    rank[j] = atomicAdd(&bhist[bu * kCntPad], 1u);
  }
  if (ballot(bad) != 0 && lane_id() == 0) atomicOr(flag, 2);
}

// exclusive scan of the bucket counts (one workgroup, through LDS); the
// number of updates of each probe dimension falls out of group boundaries.
// With tprefix non-null, also the exclusive prefix of the buckets' tiles of
// at most 64 updates (tprefix[kBuckets] = all tiles).  Only the d *
// kBucketsPerDim buckets of the probe dimensions in use are scanned (PER =
// d * 8 per thread); bhist and tprefix are written up to that bound
// inclusive, so that the last bucket has an end.
// the padded bucket counters gathered into consecutive words (many
// workgroups, so that the single-workgroup scan below reads dense memory)
__global__ __launch_bounds__(256) void bucket_gather_kernel(const uint32_t* __restrict__ bcnt,
                                                            uint32_t nb,
                                                            uint32_t* __restrict__ dense) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) dense[i] = bcnt[(size_t)i * kCntPad];
}

template <uint32_t PER>
__global__ __launch_bounds__(1024) void bucket_scan_kernel(uint32_t* __restrict__ bhist,
                                                           uint32_t m,
                                                           uint32_t* __restrict__ gstart_out,
                                                           uint32_t* __restrict__ gcount,
                                                           uint32_t* __restrict__ tprefix) {
  // thread tid owns buckets tid*PER .. tid*PER+PER-1, kept in registers; the
  // LDS copy is padded (one word per PER, PER + 1 odd) so that these reads
  // do not conflict, and global reads and writes go through it in
  // coalesced order
  constexpr uint32_t NB = PER * 1024;
  static_assert(NB <= kBuckets && NB % kBucketsPerDim == 0, "whole probe dimensions");
  __shared__ uint32_t sb[NB + 1024];
  __shared__ uint32_t wsum[1024 / kWave];
  __shared__ uint32_t tws[1024 / kWave];
  __shared__ uint32_t gstart[DDM_MAX_D + 1];
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  if (tid <= DDM_MAX_D) gstart[tid] = m;  // dimensions beyond d hold no update
  for (uint32_t i = tid; i < NB; i += 1024) sb[i + i / PER] = bhist[i];
  __syncthreads();
  uint32_t c[PER];
  uint32_t sum = 0, tsum = 0;
#pragma unroll
  for (uint32_t i = 0; i < PER; ++i) {
    c[i] = sb[tid * (PER + 1) + i];
    sum += c[i];
    tsum += (c[i] + 63u) / 64u;
  }
  uint32_t inc = sum, tinc = tsum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t2 = __shfl_up(inc, o, kWave);
    const uint32_t t3 = __shfl_up(tinc, o, kWave);
    if (lane >= (uint32_t)o) {
      inc += t2;
      tinc += t3;
    }
  }
  if (lane == kWave - 1) {
    wsum[wave] = inc;
    tws[wave] = tinc;
  }
  __syncthreads();
  uint32_t before = 0, tbefore = 0, ttotal = 0;
  for (uint32_t w = 0; w < 1024 / kWave; ++w) {
    if (w < wave) {
      before += wsum[w];
      tbefore += tws[w];
    }
    ttotal += tws[w];
  }
  if (tprefix) {
    uint32_t trun = tbefore + tinc - tsum;
#pragma unroll
    for (uint32_t i = 0; i < PER; ++i) {
      sb[tid * (PER + 1) + i] = trun;
      trun += (c[i] + 63u) / 64u;
    }
    __syncthreads();
    for (uint32_t i = tid; i < NB; i += 1024) tprefix[i] = sb[i + i / PER];
    if (tid == 0) {
      tprefix[NB] = ttotal;
      tprefix[kBuckets] = ttotal;
    }
    __syncthreads();
  }
  uint32_t run = before + inc - sum;
#pragma unroll
  for (uint32_t i = 0; i < PER; ++i) {
    const uint32_t x = tid * PER + i;  // a probe dimension starts at x % kBucketsPerDim == 0
    if (x % kBucketsPerDim == 0) gstart[x / kBucketsPerDim] = run;
    sb[tid * (PER + 1) + i] = run;
    run += c[i];
  }
  __syncthreads();
  for (uint32_t i = tid; i < NB; i += 1024) bhist[i] = sb[i + i / PER];
  if (tid == 0 && NB < kBuckets) bhist[NB] = m;
  if (tid < DDM_MAX_D) {
    gcount[tid] = gstart[tid + 1] - gstart[tid];
    gstart_out[tid] = gstart[tid];
  }
}

// updates in bucket order; with tmap non-null also tile -> bucket for the
// nb buckets (thread j does update j and bucket j)
__global__ __launch_bounds__(256) void bucket_scatter_kernel(const uint32_t* __restrict__ bucket,
                                                             const uint32_t* __restrict__ rank,
                                                             uint32_t m,
                                                             const uint32_t* __restrict__ bhist,
                                                             uint32_t* __restrict__ perm,
                                                             const uint32_t* __restrict__ tprefix,
                                                             uint32_t* __restrict__ tmap,
                                                             uint32_t nb) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) perm[bhist[bucket[j]] + rank[j]] = j;
  if (tmap && j < nb)
    for (uint32_t t = tprefix[j]; t < tprefix[j + 1]; ++t) tmap[t] = j;
}

// --------------------------------------------------------------------------
// Tiles balanced by work (the learned single pass: predicted hits; the
// plain fill: the exact counts).  Within each bucket the updates are cut
// into tiles at every 64th update (as for the count) and also wherever the
// hits accumulated since the bucket's start cross a multiple of H (below),
// so that a wavefront never takes a tile of much more output than H: dense
// regions get several small tiles, which run on separate wavefronts,
// instead of one long one.
// --------------------------------------------------------------------------
// H = twice an average full tile's work / kCutDiv, but at least
// kCutMinHits: with 8, an average tile of 64 updates of the hotspot
// workload (3600 hits per update) is cut in about four (a flush's
// per-update work then spreads over more wavefronts; each piece scans its
// candidate range again).  Measured on that workload's learned fill:
// kCutDiv 1 11.1 ms, 4 8.7, 16 7.9, 64 10.3, 256 13.2; later, on the whole
// learned step: 6 14.93 ms, 8 14.85, 11 14.91, 16 15.14, 32 15.87.  Tiles
// of a few thousand hits gain nothing from the cut (uniform sets at 200
// hits per update: fill 0.51 ms uncut, 1.04 ms cut in eight), hence the
// floor.
#ifndef DDM_CUT_DIV
#define DDM_CUT_DIV 8
#endif
constexpr uint32_t kCutDiv = DDM_CUT_DIV;
constexpr uint64_t kCutMinHits = 32768;
__global__ __launch_bounds__(256) void work_in_order_kernel(const uint32_t* __restrict__ perm,
                                                            const uint32_t* __restrict__ cap,
                                                            uint32_t m,
                                                            uint32_t* __restrict__ w) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < m) w[p] = cap[perm[p]];
}

// flag[p] = 1 where a tile starts; cw: exclusive scan of w (cw[m] = total)
__global__ __launch_bounds__(256) void tile_cut_kernel(const uint32_t* __restrict__ perm,
                                                       const uint32_t* __restrict__ bucket,
                                                       const uint32_t* __restrict__ boff,
                                                       const uint64_t* __restrict__ cw,
                                                       uint32_t m, uint32_t* __restrict__ flag) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const uint64_t H = max((2ull * 64ull * cw[m]) / ((uint64_t)m * kCutDiv), kCutMinHits);
  const uint32_t s = boff[bucket[perm[p]]];
  bool cut = p == s || ((p - s) & 63u) == 0;
  if (!cut) cut = (cw[p] - cw[s]) / H != (cw[p - 1] - cw[s]) / H;
  flag[p] = cut ? 1u : 0u;
}

// tile t starts at the t-th flagged position; tstart[ntiles] = m
__global__ __launch_bounds__(256) void tile_list_kernel(const uint32_t* __restrict__ perm,
                                                        const uint32_t* __restrict__ bucket,
                                                        const uint32_t* __restrict__ flag,
                                                        const uint64_t* __restrict__ tidx,
                                                        uint32_t m, uint32_t* __restrict__ tstart,
                                                        uint32_t* __restrict__ tbuck) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < m && flag[p]) {
    const uint32_t t = (uint32_t)tidx[p];
    tstart[t] = p;
    tbuck[t] = bucket[perm[p]];
  }
  if (p == 0) tstart[(uint32_t)tidx[m]] = m;
}

// --------------------------------------------------------------------------
// 3/5a. one lane per update: Algorithm 4 without a stack.
//
// On the implicit in-order tree the recursion of Algorithm 4 becomes a walk
// over positions in increasing order with two states:
//   ENTER x  (call on subtree x of height h, span [a, x + 2^h - 1]):
//            a > n (all padding)            -> stop (so is everything after);
//            minlower = lo[a] > q.upper     -> stop (every later lower bound
//                                              is at least as large);
//            maxupper[x] < q.lower          -> skip the subtree, VISIT x + 2^h;
//            else descend to the left child, or VISIT x at a leaf.
//   VISIT x  (left subtree of x done): x > n or lo[x] > q.upper -> stop;
//            test x (Algorithm 1, closed, all dimensions); then ENTER the
//            right child, or VISIT x + 1 at a leaf.
// Positions after the end of a subtree are exactly the next in-order node
// whose left subtree is complete, so no stack is needed.  The nodes tested
// are those Algorithm 4 tests, in the same (in-order) order, except that the
// walk stops at the first lower bound beyond q.upper instead of returning
// through ancestors that would all fail the same test.
// --------------------------------------------------------------------------
template <int D, bool FILL>
__global__ __launch_bounds__(1024) void lane_kernel(TreeDev T, const float* __restrict__ ulo,
                                                   const float* __restrict__ uhi, uint32_t m,
                                                   UpdSet US, const uint8_t* __restrict__ kstar,
                                                   SegOut O) {
  constexpr int R = 2 * D;
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t pi;
  if (!upd_index(US, t, D, &pi)) return;
  const uint32_t j = US.perm[pi];
  const uint32_t k = kstar[j];
  float ql[D], qh[D];
  load_query<D>(ulo, uhi, m, j, k, ql, qh);
  const float* __restrict__ rec = T.rec[k];
  const float* __restrict__ mx = T.maxhi[k];
  const uint32_t* __restrict__ ids = T.id[k];
  const uint32_t n = T.n;
  uint32_t x = 1u << (T.H - 1);
  bool enter = true;
  uint32_t c = 0;
  uint64_t base = 0, segend = 0;
  if (FILL) seg_bounds(O, j, &base, &segend);
  const uint64_t lim = segend - base;  // writable slots (write guard)
  uint64_t* __restrict__ out = O.out;
  const uint64_t jhi = (uint64_t)j << 32;
  while (true) {
    if (enter) {
      const uint32_t h = (uint32_t)__builtin_ctz(x);
      const uint32_t a = x - (1u << h) + 1u;
      if (a > n) break;
      if (rec[(size_t)a * R] > qh[0]) break;
      if (mx[x] < ql[0]) {
        x += 1u << h;
        enter = false;
      } else if (h == 0) {
        enter = false;
      } else {
        x -= 1u << (h - 1);
      }
    } else {
      if (x > n) break;
      float v[R];
      load_rec<D>(rec + (size_t)x * R, v);
      if (v[0] > qh[0]) break;
      if (overlaps<D>(v, ql, qh)) {
        if (FILL && c < lim) {
          if (O.ids) O.ids[base + c] = ids[x];
          else out[base + c] = jhi | ids[x];
        }
        ++c;
      }
      const uint32_t h = (uint32_t)__builtin_ctz(x);
      if (h == 0) {
        x += 1u;
      } else {
        x += 1u << (h - 1);
        enter = true;
      }
    }
  }
  if (!FILL || O.cnt) O.cnt[j] = c;
}

// --------------------------------------------------------------------------
// 3/5b. tile traversal for one instance (body in traverse.h)
// --------------------------------------------------------------------------
template <int D, bool FILL>
__global__ __launch_bounds__(kTileWaves * kWave) void tile_kernel(
    TreeDev T, const float* __restrict__ ulo, const float* __restrict__ uhi, uint32_t m,
    UpdSet US, SegOut O) {
  constexpr int R = 2 * D;
  constexpr int RV = (R + 3) / 4;
  __shared__ float s_cand[kTileWaves][R][kRing];
  __shared__ uint32_t s_cid[kTileWaves][kRing];
  __shared__ float4 s_q[kTileWaves][kWave][RV];
  const uint32_t wave = threadIdx.x / kWave;
  const uint32_t lane = lane_id();
  const uint32_t tile = blockIdx.x * kTileWaves + wave;

  // locate the tile inside its probe-dimension group
  uint32_t qbeg = 0, tacc = 0, nq = 0, k = 0;
  bool found = false;
  const uint32_t qpt = US.qpt;
#pragma unroll
  for (int g = 0; g < D; ++g) {
    const uint32_t gs = uniform_u32(US.gcount[g]);
    const uint32_t nt = (gs + qpt - 1) / qpt;
    if (!found) {
      if (tile < tacc + nt) {
        found = true;
        k = (uint32_t)g;
        const uint32_t lt = tile - tacc;
        qbeg = uniform_u32(US.gstart[g]) + lt * qpt;
        nq = min(qpt, gs - lt * qpt);
      } else {
        tacc += nt;
      }
    }
  }
  if (!found) return;
  k = uniform_u32(k);
  nq = uniform_u32(nq);
  qbeg = uniform_u32(qbeg);

  tile_body<D, FILL>(T, ulo, uhi, m, US.perm, 0, k, qbeg, nq, O, &s_cand[wave][0][0],
                     &s_cid[wave][0], &s_q[wave][0][0], lane, 0u, US.pb);
}

// --------------------------------------------------------------------------
// 6. per-segment sort by subscription id
// --------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void bitonic_regs(uint64_t (&v)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ jj;
        if (l > i) {
          const bool up = (i & k) == 0;
          const uint64_t a = v[i], b = v[l];
          const bool sw = up ? (a > b) : (a < b);
          v[i] = sw ? b : a;
          v[l] = sw ? a : b;
        }
      }
    }
  }
}

// Where segment j's unsorted keys are.  In the single-pass form the updates
// that fitted their slots still sit in the slot arena; every other segment
// is in place in the output.  The sorts below read a segment from its source
// and write it sorted to its final position, so moving slots into place
// costs no extra pass.
// bucket-aligned tiles, one wavefront each (the grid covers the largest
// possible number of tiles; the waves beyond the actual number return).
// The traversal is latency-bound, so the register budget of the fill and of
// the d = 1 forms is set for eight wavefronts per SIMD; the count kernels
// for d >= 2 (with the transposed flush beside the direct one) for seven,
// where they spill nothing (at eight they kept 12 registers per lane in
// scratch and ran 4% slower).
#ifndef DDM_TILE_COUNT_WAVES
#define DDM_TILE_COUNT_WAVES 7
#endif
constexpr uint32_t kXcds = 8;     // accelerator dies (each with its own L2) of the device
constexpr uint32_t kXcdRun = 32;  // consecutive workgroups of tiles given to one die

// The count pass (d >= 2) runs the transposed flush beside the untransposed
// one; with both, seven wavefronts per SIMD leave it room without spilling.
template <int D, bool FILL>
constexpr int tile_waves_per_eu() {
  return (!FILL && D >= 2) ? DDM_TILE_COUNT_WAVES : 8;
}

template <int D, bool FILL, bool STASH = false>
__global__ __launch_bounds__(kTileWaves * kWave)
__attribute__((amdgpu_waves_per_eu(tile_waves_per_eu<D, FILL>())))
void tile_bucket_kernel(
    TreeDev T, const float* __restrict__ ulo, const float* __restrict__ uhi, uint32_t m,
    UpdSet US, SegOut O) {
  constexpr int R = 2 * D;
  constexpr int RV = (R + 3) / 4;
  // the count pass (d >= 2) takes the transposed flush
  constexpr bool XP = !FILL && D >= 2;
  constexpr int XW = XP ? kWave : 1;
  __shared__ float s_cand[kTileWaves][R * kRing];
  __shared__ uint32_t s_cid[kTileWaves][kRing];
  __shared__ float4 s_q[kTileWaves][kWave * RV];
  __shared__ float s_lo1[kTileWaves][XW];
  __shared__ uint32_t s_xcnt[kTileWaves][XW];
  __shared__ uint32_t s_xj[kTileWaves][XW];
  const uint32_t wave = threadIdx.x / kWave;
  const uint32_t lane = lane_id();
  const bool list = US.tstart != nullptr;
  const uint32_t total = list ? uniform_u32((uint32_t)*US.ntiles)
                              : uniform_u32(US.tprefix[kBuckets]);
  {
    // Workgroups go to the XCDs in turn (workgroup i to XCD i mod kXcds).
    // Neighbouring tiles (the cells of one probe range) scan the same part
    // of the tree, so within each window of kXcds * kXcdRun workgroups the
    // ones on XCD x take kXcdRun consecutive groups of tiles, whose scans
    // then share that XCD's L2; the workgroups past the last whole window
    // keep their order.  Any one-to-one map is correct; this one only
    // changes which L2 serves a tile (measured at 10^6 boxes: d = 2, alpha
    // = 1 -1%, d = 3 -8%, d = 4 -25%, d = 2, alpha = 10 +7%).
    const uint32_t nblk = (total + kTileWaves - 1) / kTileWaves;
    uint32_t blk = blockIdx.x;
    if (blk >= nblk) return;
    constexpr uint32_t W = kXcds * kXcdRun;
    if (blk < nblk / W * W) blk = blk / W * W + blk % kXcds * kXcdRun + blk % W / kXcds;
    const uint32_t item = blk * kTileWaves + wave;
    if (item >= total) return;
    uint32_t b, qbeg, nq;
    if (list) {
      b = uniform_u32(US.tbuck[item]);
      qbeg = uniform_u32(US.tstart[item]);
      nq = uniform_u32(US.tstart[item + 1]) - qbeg;
    } else {
      b = uniform_u32(US.tmap[item]);
      const uint32_t lt = item - uniform_u32(US.tprefix[b]);
      const uint32_t start = uniform_u32(US.boff[b]);
      const uint32_t end = b + 1 < kBuckets ? uniform_u32(US.boff[b + 1]) : US.total;
      qbeg = start + lt * 64u;
      nq = min(64u, end - qbeg);
    }
    tile_body<D, FILL, STASH, XP>(T, ulo, uhi, m, US.perm, 0u, b / kBucketsPerDim, qbeg, nq, O,
                                  s_cand[wave], s_cid[wave], s_q[wave], lane, item, US.pb,
                                  XpLds{s_lo1[wave], s_xcnt[wave], s_xj[wave]});
  }
}

// Where the segment sort finds each segment's unsorted hits: in place in
// out as keys, or as 4-byte subscription ids (the keys then formed with the
// update's index as the high word) in the single pass's slots (the updates
// whose hits fitted) or, from the plain fill, at the segment's own places.
struct SegSrc {
  const uint32_t* slots = nullptr;  // single pass: ids in the slots
  SegOut so{};                      // slot bounds (base = slot offsets, cap, limit)
  const uint32_t* cnt = nullptr;    // hits per update
  const uint32_t* ids = nullptr;    // plain fill: ids at the segments' places
};

// segment j (output offset b): its ids, or else its keys (in place in out)
struct SegAt {
  const uint32_t* ids;
  const uint64_t* keys;
};
__device__ __forceinline__ SegAt seg_at(const SegSrc& S, uint32_t j, const uint64_t* out,
                                        uint64_t b) {
  if (S.ids) return SegAt{S.ids + b, nullptr};
  if (S.slots) {
    uint64_t sb, se;
    seg_bounds(S.so, j, &sb, &se);
    if ((uint64_t)S.cnt[j] <= se - sb) return SegAt{S.slots + sb, nullptr};
  }
  return SegAt{nullptr, out + b};
}

template <int N>
__device__ __forceinline__ void sort_small_segment(const uint64_t* __restrict__ src,
                                                   uint64_t* __restrict__ dst, uint32_t len) {
  uint64_t v[N];
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = ((uint32_t)i < len) ? src[i] : ~0ull;
  bitonic_regs<N>(v);
#pragma unroll
  for (int i = 0; i < N; ++i)
    if ((uint32_t)i < len) dst[i] = v[i];
}

constexpr uint32_t kSegMid = 2048;  // longest segment sorted in LDS by bitonic

// the same, from 4-byte ids, keys formed with the update's high word
template <int N>
__device__ __forceinline__ void sort_small_ids(const uint32_t* __restrict__ src, uint64_t jhi,
                                               uint64_t* __restrict__ dst, uint32_t len) {
  uint64_t v[N];
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = ((uint32_t)i < len) ? (jhi | src[i]) : ~0ull;
  bitonic_regs<N>(v);
#pragma unroll
  for (int i = 0; i < N; ++i)
    if ((uint32_t)i < len) dst[i] = v[i];
}

// IDS: segments may be 4-byte ids (S.ids or S.slots); else all are keys
template <bool IDS>
__global__ __launch_bounds__(256) void segsort_small_kernel(const uint64_t* __restrict__ off,
                                                            uint32_t m, uint64_t* __restrict__ out,
                                                            SegSrc S,
                                                            uint32_t* __restrict__ lists,
                                                            uint32_t* __restrict__ list_count) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const uint64_t b = off[j];
  const uint64_t len64 = off[j + 1] - b;
  if (len64 == 0) return;
  const uint32_t len = len64 > 0xffffffffull ? 0xffffffffu : (uint32_t)len64;
  const SegAt a = IDS ? seg_at(S, j, out, b) : SegAt{nullptr, out + b};
  if (IDS && a.ids && len <= 32) {
    const uint32_t* ip = a.ids;
    const uint64_t jhi = (uint64_t)j << 32;
    if (len == 1) out[b] = jhi | ip[0];
    else if (len <= 4) sort_small_ids<4>(ip, jhi, out + b, len);
    else if (len <= 8) sort_small_ids<8>(ip, jhi, out + b, len);
    else if (len <= 16) sort_small_ids<16>(ip, jhi, out + b, len);
    else sort_small_ids<32>(ip, jhi, out + b, len);
    return;
  }
  const uint64_t* src = a.keys;  // in place
  if (len == 1) return;
  if (len <= 4) {
    sort_small_segment<4>(src, out + b, len);
  } else if (len <= 8) {
    sort_small_segment<8>(src, out + b, len);
  } else if (len <= 16) {
    sort_small_segment<16>(src, out + b, len);
  } else if (len <= 32) {
    sort_small_segment<32>(src, out + b, len);
  } else if (len <= kSegMid) {
    lists[atomicAdd(&list_count[0], 1u)] = j;
  } else {
    lists[m + atomicAdd(&list_count[1], 1u)] = j;
  }
}

// One wavefront per listed segment (33..2048 keys).  The segment's ids are
// staged through LDS (coalesced global reads and writes) into registers in
// blocked order (element i = lane * V + r), V = P2/64 per lane (P2 = the
// segment length rounded up to a power of two, at least 64), and sorted by
// a bitonic network.  From V = 4 on it is written with every comparator
// ascending: to merge sorted blocks of k/2 into blocks of k, element i is
// first compared with i ^ (k - 1) (the mirror image in its block of k),
// then with i ^ j for j = k/4 .. 1; a comparator is a min and a max.
// Partners less than V apart stay inside a lane's registers, the others
// are in the lane whose index differs in the partner's bits (the mirror
// pairs register r with register V - 1 - r there).  With V <= 2 nearly
// every stage crosses lanes, and the classic form (comparators of both
// directions, partner i ^ j for j = k/2 .. 1) is faster there: measured on
// the 256-instance batch, segment sort 0.83 ms classic, 0.88 all-ascending,
// 0.79 with the split; 16-hotspot workload 9.7 -> 9.1 ms.
template <int V, typename SRC>
__device__ __forceinline__ void wave_bitonic_segment(const SRC* __restrict__ src,
                                                     uint64_t* __restrict__ dst, uint32_t len,
                                                     uint64_t jhi, uint32_t* __restrict__ sh,
                                                     uint32_t lane) {
  constexpr uint32_t P2 = 64u * V;
  for (uint32_t i = lane; i < P2; i += kWave) sh[i] = (i < len) ? (uint32_t)src[i] : 0xffffffffu;
  wave_sync();
  uint32_t v[V];
#pragma unroll
  for (int r = 0; r < V; ++r) v[r] = sh[lane * V + r];
  if constexpr (V <= 2) {
    // classic form: the lower index keeps the smaller key when the block
    // of k it lies in sorts up
#pragma unroll
    for (uint32_t k = 2; k <= P2; k <<= 1) {
#pragma unroll
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        if (j >= (uint32_t)V) {
          // partner: lane ^ (j / V), same register
          const uint32_t lx = j / V;
          const bool lower = (lane & lx) == 0;
#pragma unroll
          for (int r = 0; r < V; ++r) {
            const uint32_t o = (uint32_t)__shfl_xor((int)v[r], (int)lx, kWave);
            const bool up = ((lane * V + r) & k) == 0;
            // the lower index keeps the smaller key when sorting up
            v[r] = (lower == up) ? min(v[r], o) : max(v[r], o);
          }
        } else {
#pragma unroll
          for (int r = 0; r < V; ++r) {
            if (((uint32_t)r & j) != 0) continue;
            const int q = r + (int)j;
            const bool up = ((lane * V + r) & k) == 0;
            const uint32_t a = v[r], b = v[q];
            const bool sw = up ? (a > b) : (a < b);
            v[r] = sw ? b : a;
            v[q] = sw ? a : b;
          }
        }
      }
    }
  } else {
#pragma unroll
    for (uint32_t k = 2; k <= P2; k <<= 1) {
      if (k <= (uint32_t)V) {
        // the mirror inside the lane: r and r ^ (k - 1)
#pragma unroll
        for (int r = 0; r < V; ++r) {
          const int q = r ^ (int)(k - 1);
          if (q <= r) continue;
          const uint32_t a = v[r], b = v[q];
          v[r] = min(a, b);
          v[q] = max(a, b);
        }
      } else {
        // the mirror across lanes: lane ^ (k/V - 1), register V - 1 - r; the
        // lane in the lower half of the block keeps the smaller key
        const int lm = (int)(k / V - 1);
        const bool lower = (lane & (k / (2 * V))) == 0;
#pragma unroll
        for (int r = 0; r < (V + 1) / 2; ++r) {
          const int q = V - 1 - r;
          const uint32_t t1 = (uint32_t)__shfl_xor((int)v[q], lm, kWave);
          const uint32_t t2 = (uint32_t)__shfl_xor((int)v[r], lm, kWave);
          v[r] = lower ? min(v[r], t1) : max(v[r], t1);
          if (q != r) v[q] = lower ? min(v[q], t2) : max(v[q], t2);
        }
      }
#pragma unroll
      for (uint32_t j = k >> 2; j > 0; j >>= 1) {
        if (j >= (uint32_t)V) {
          // partner: lane ^ (j / V), same register
          const uint32_t lx = j / V;
          const bool lower = (lane & lx) == 0;
#pragma unroll
          for (int r = 0; r < V; ++r) {
            const uint32_t o = (uint32_t)__shfl_xor((int)v[r], (int)lx, kWave);
            v[r] = lower ? min(v[r], o) : max(v[r], o);
          }
        } else {
#pragma unroll
          for (int r = 0; r < V; ++r) {
            if (((uint32_t)r & j) != 0) continue;
            const int q = r + (int)j;
            const uint32_t a = v[r], b = v[q];
            v[r] = min(a, b);
            v[q] = max(a, b);
          }
        }
      }
    }
  }
  wave_sync();
#pragma unroll
  for (int r = 0; r < V; ++r) sh[lane * V + r] = v[r];
  wave_sync();
  for (uint32_t i = lane; i < len; i += kWave) dst[i] = jhi | sh[i];
  wave_sync();
}

constexpr int kSegWaves = 4;  // wavefronts per workgroup of the mid sort

// the register width for a segment of len (33..2048) keys
template <typename SRC>
__device__ __forceinline__ void sort_wave_segment(const SRC* __restrict__ src,
                                                  uint64_t* __restrict__ dst, uint32_t len,
                                                  uint64_t jhi, uint32_t* __restrict__ sh,
                                                  uint32_t lane) {
  if (len <= 64) wave_bitonic_segment<1>(src, dst, len, jhi, sh, lane);
  else if (len <= 128) wave_bitonic_segment<2>(src, dst, len, jhi, sh, lane);
  else if (len <= 256) wave_bitonic_segment<4>(src, dst, len, jhi, sh, lane);
  else if (len <= 512) wave_bitonic_segment<8>(src, dst, len, jhi, sh, lane);
  else if (len <= 1024) wave_bitonic_segment<16>(src, dst, len, jhi, sh, lane);
  else wave_bitonic_segment<32>(src, dst, len, jhi, sh, lane);
}

template <bool IDS>
__global__ __launch_bounds__(kSegWaves * kWave) void segsort_mid_kernel(
    const uint64_t* __restrict__ off, uint64_t* __restrict__ out, SegSrc S,
    const uint32_t* __restrict__ lists, const uint32_t* __restrict__ list_count) {
  __shared__ uint32_t shw[kSegWaves][kSegMid];
  const uint32_t wave = threadIdx.x / kWave;
  const uint32_t lane = lane_id();
  uint32_t* sh = shw[wave];
  const uint32_t cntl = uniform_u32(list_count[0]);
  const uint32_t nw = gridDim.x * kSegWaves;
  for (uint32_t li = blockIdx.x * kSegWaves + wave; li < cntl; li += nw) {
    const uint32_t j = uniform_u32(lists[li]);
    const uint64_t b = off[j];
    const uint32_t len = uniform_u32((uint32_t)(off[j + 1] - b));
    uint64_t* dst = out + b;
    const SegAt a = IDS ? seg_at(S, j, out, b) : SegAt{nullptr, out + b};
    if (IDS && a.ids) {
      sort_wave_segment(a.ids, dst, len, (uint64_t)j << 32, sh, lane);
    } else {
      // every key of the segment carries the same update id in its high word
      const uint64_t jhi = readlane_u64(a.keys[0], 0) & 0xffffffff00000000ull;
      sort_wave_segment(a.keys, dst, len, jhi, sh, lane);
    }
  }
}

// One workgroup per listed segment of MAXLEN/2 + 1 .. MAXLEN keys (MAXLEN =
// 4096, 8192, 16384; one launch per size class, so that the smaller classes
// need less LDS and more workgroups share a compute unit and overlap their
// loads): a counting sort over MAXLEN buckets of consecutive ids
// (id >> shift, about one id per bucket at the largest size of the class),
// in LDS.  Each thread loads its (at most 16) keys once into registers; the
// ids are counted, the counts scanned (thread t owns buckets 16t .. 16t+15),
// the ids placed by bucket, and then each thread insertion-sorts its own run
// of the placed ids, which spans its 16 buckets and is already ordered
// between buckets (so it takes about as many steps as the run is long).
// The sorted segment is written once.  A segment whose ids crowd into few
// buckets (a thread's run longer than kRunCap) is left to the bitmap kernel
// below; every segment handled here is marked done in its list entry.
constexpr uint32_t kBucketSegMax = 16384;
constexpr uint32_t kPerThread = 16;  // keys per thread, buckets per thread
constexpr uint32_t kRunCap = 128;
constexpr uint32_t kListDone = 0x80000000u;

template <uint32_t MAXLEN>
__global__ __launch_bounds__(MAXLEN / kPerThread) void segsort_bucket_kernel(
    const uint64_t* __restrict__ off, uint32_t m, uint64_t* __restrict__ out, SegSrc S,
    uint32_t* __restrict__ lists, const uint32_t* __restrict__ list_count, uint32_t shift) {
  constexpr uint32_t NT = MAXLEN / kPerThread;  // threads
  constexpr uint32_t NB = MAXLEN;                // buckets
  __shared__ uint32_t sorted[MAXLEN];
  __shared__ uint32_t cnt[NB];
  __shared__ uint32_t wsum[NT / kWave];
  __shared__ uint32_t maxrun;
  const uint32_t cntl = list_count[1];
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  for (uint32_t li = blockIdx.x; li < cntl; li += gridDim.x) {
    const uint32_t j = lists[m + li];
    if (j & kListDone) continue;
    const uint64_t b = off[j];
    const uint64_t len64 = off[j + 1] - b;
    if (len64 > MAXLEN || len64 <= MAXLEN / 2) continue;
    const uint32_t len = (uint32_t)len64;
    const SegAt a = seg_at(S, j, out, b);
    const uint64_t jhi = a.ids ? (uint64_t)j << 32 : a.keys[0] & 0xffffffff00000000ull;
    // this thread's keys: positions tid + r * NT (all loads in flight while
    // the counters are cleared)
    uint32_t ids[kPerThread];
#pragma unroll
    for (uint32_t r = 0; r < kPerThread; ++r) {
      const uint32_t i = tid + r * NT;
      ids[r] = i < len ? (a.ids ? a.ids[i] : (uint32_t)a.keys[i]) : 0u;
    }
#pragma unroll
    for (uint32_t q = 0; q < kPerThread; ++q) cnt[q * NT + tid] = 0;
    if (tid == 0) maxrun = 0;
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < kPerThread; ++r)
      if (tid + r * NT < len) atomicAdd(&cnt[min(ids[r] >> shift, NB - 1u)], 1u);
    __syncthreads();
    // exclusive scan: this thread's 16 buckets, then across threads
    uint32_t c[kPerThread];
    uint32_t run = 0;
#pragma unroll
    for (uint32_t q = 0; q < kPerThread; ++q) {
      c[q] = cnt[tid * kPerThread + q];
      run += c[q];
    }
    uint32_t inc = run;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t2 = __shfl_up(inc, o, kWave);
      if (lane >= (uint32_t)o) inc += t2;
    }
    if (lane == kWave - 1) wsum[wave] = inc;
    atomicMax(&maxrun, run);
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t q = 0; q < wave; ++q) before += wsum[q];
    const uint32_t my0 = before + inc - run;  // first slot of this thread's run
    {
      uint32_t at = my0;
#pragma unroll
      for (uint32_t q = 0; q < kPerThread; ++q) {
        cnt[tid * kPerThread + q] = at;
        at += c[q];
      }
    }
    __syncthreads();
    const bool skip = maxrun > kRunCap;
    __syncthreads();  // every thread has read maxrun before the next segment resets it
    if (skip) continue;
#pragma unroll
    for (uint32_t r = 0; r < kPerThread; ++r)
      if (tid + r * NT < len) sorted[atomicAdd(&cnt[min(ids[r] >> shift, NB - 1u)], 1u)] = ids[r];
    __syncthreads();
    for (uint32_t i = my0 + 1; i < my0 + run; ++i) {
      const uint32_t x = sorted[i];
      uint32_t k = i;
      while (k > my0 && sorted[k - 1] > x) {
        sorted[k] = sorted[k - 1];
        --k;
      }
      sorted[k] = x;
    }
    __syncthreads();
    for (uint32_t i = tid; i < len; i += NT) out[b + i] = jhi | sorted[i];
    if (tid == 0) lists[m + li] = j | kListDone;
    __syncthreads();
  }
}

// One workgroup per long segment: mark ids in an LDS bitmap (dynamic size:
// `words` 32-bit words covering a window of ids), then emit them in
// increasing order.  Ids span [0, n): with more than one window, in-place
// segments read their ids from `tmp`, a copy taken before any write.
constexpr int kBigThreads = 1024;
constexpr uint32_t kMaxBitWords = 1u << 15;  // 128 KiB of LDS, 2^20 ids per window

__global__ __launch_bounds__(kBigThreads) void segsort_big_kernel(
    const uint64_t* __restrict__ off, uint32_t m, uint64_t* __restrict__ out, SegSrc S,
    const uint32_t* __restrict__ lists, const uint32_t* __restrict__ list_count,
    const uint32_t* __restrict__ tmp, uint32_t n, uint32_t words) {
  extern __shared__ uint32_t bits[];
  __shared__ uint32_t wsum[kBigThreads / kWave];
  const uint32_t cntl = list_count[1];
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t wave = tid / kWave;
  const uint32_t span = words * 32;
  const uint32_t nwin = (n + span - 1) / span;
  for (uint32_t li = blockIdx.x; li < cntl; li += gridDim.x) {
    const uint32_t j = lists[m + li];
    if (j & kListDone) continue;  // sorted by the bucket kernel
    const uint64_t b = off[j];
    const uint64_t len = off[j + 1] - b;
    const SegAt a = seg_at(S, j, out, b);
    // every key of the segment carries the same update id in its high word
    const uint64_t jhi = a.ids ? (uint64_t)j << 32 : a.keys[0] & 0xffffffff00000000ull;
    __syncthreads();  // read before any in-place write of this segment
    uint64_t written = 0;
    for (uint32_t w = 0; w < nwin; ++w) {
      const uint32_t w0 = w * span;
      const uint32_t wwords = min(words, (n - w0 + 31) / 32);
      for (uint32_t i = tid; i < wwords; i += kBigThreads) bits[i] = 0;
      __syncthreads();
      for (uint64_t i = tid; i < len; i += kBigThreads) {
        const uint32_t id = a.ids ? a.ids[i] : (nwin > 1 ? tmp[b + i] : (uint32_t)a.keys[i]);
        if (id >= w0 && id - w0 < span) {
          const uint32_t r = id - w0;
          atomicOr(&bits[r >> 5], 1u << (r & 31));
        }
      }
      __syncthreads();
      // each thread owns a contiguous run of words
      const uint32_t per = (wwords + kBigThreads - 1) / kBigThreads;
      const uint32_t w_beg = min(wwords, tid * per), w_end = min(wwords, w_beg + per);
      uint32_t mine = 0;
      for (uint32_t q = w_beg; q < w_end; ++q) mine += __popc(bits[q]);
      uint32_t inc = mine;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t2 = __shfl_up(inc, o, kWave);
        if (lane >= (uint32_t)o) inc += t2;
      }
      if (lane == kWave - 1) wsum[wave] = inc;
      __syncthreads();
      uint32_t before = 0, total = 0;
      for (uint32_t q = 0; q < kBigThreads / kWave; ++q) {
        if (q < wave) before += wsum[q];
        total += wsum[q];
      }
      uint64_t pos = written + before + inc - mine;
      for (uint32_t q = w_beg; q < w_end; ++q) {
        uint32_t word = bits[q];
        while (word) {
          const uint32_t bit = (uint32_t)__builtin_ctz(word);
          word &= word - 1;
          out[b + pos++] = jhi | (w0 + q * 32 + bit);
        }
      }
      written += total;
      __syncthreads();
    }
  }
}

// One workgroup per listed segment (more than kSegMid keys) when every id
// is below 2^20.  The ids of one update are distinct, so each is marked in
// an LDS bitmap of ceil(n/32) words, and an id's place in the sorted
// segment is the number of marked ids below it: the marks of the uint4
// entries before its own (a scan of the entries' counts) plus those below
// it in its entry.  Entry r*kBmThreads + t is counted by thread t
// (conflict-free 16-byte LDS reads); the entries' exclusive counts within
// their wave's block are kept as 16-bit values, the blocks' starts come
// from a scan of the wave totals that every wave does itself.  A segment
// of at most kBmPre * kBmThreads keys has its ids in registers: each
// thread ranks its own, and once every id is ranked the bitmap's LDS
// becomes the staging array: each id is written at its place there (as
// id + 1, 0 meaning empty), the rest of the array is cleared, and
// consecutive threads write the staged keys out (coalesced) and clear what
// they read.  A longer segment is read back from the bitmap in order,
// chunk by chunk.  Wave scans use DPP row shifts and row broadcasts.
//
// Each workgroup takes every G-th listed segment, and its loads run ahead
// (vector loads through buffer resources, so that the LDS waits of the work
// in between force no wait for them): a segment's first kBmPre * kBmThreads
// ids are loaded once the segment two before it is written, so that they
// arrive while the one in between is sorted (two register buffers, used in
// turn); its offsets are loaded three segments ahead, its list entry four.
__device__ __forceinline__ uint32_t popc4(uint4 q) {
  return __popc(q.x) + __popc(q.y) + __popc(q.z) + __popc(q.w);
}

// inclusive sum of v over lanes 0..lane of the wavefront: row shifts by 1,
// 2, 4 and 8 (lanes before the row's start add 0) give each 16-lane row
// its own prefix; broadcasting lane 15 into row 1 and lane 47 into row 3,
// then lane 31 into rows 2 and 3, carries the row totals forward
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
  return v;
}

// largest v over the wavefront (the same row shifts and broadcasts, with
// max; lanes before a row's start contribute 0), read from the last lane
__device__ __forceinline__ uint32_t wave_max_dpp(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}

// word 3 of a raw buffer resource on gfx9 parts (32-bit data format)
constexpr int kBufferFlags = 0x00020000;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           kBufferFlags);
}
__device__ __forceinline__ uint64_t buf_u64(const uint64_t* p) {
  const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(buf_rsrc(p, 8), 0, 0, 0);
  return (uint64_t)v.x | ((uint64_t)v.y << 32);
}
__device__ __forceinline__ uint32_t buf_u32(const uint32_t* p) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(buf_rsrc(p, 4), 0, 0, 0);
}
__device__ __forceinline__ uint32_t uniform_v(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uniform_v64(uint64_t v) {
  return ((uint64_t)uniform_v((uint32_t)(v >> 32)) << 32) | uniform_v((uint32_t)v);
}

// a listed segment's offsets (off[j], and the low word of off[j + 1]: the
// length is below 2^32), and in the single-pass form its slot base, the low
// word of its end (base + capacity, or the next base without capacities)
// and its hit count, as loaded
struct BmMeta {
  uint64_t b, sb;
  uint32_t elo, selo, cnt, j;
};
// where a segment is written (out + b, len keys) and read from
struct BmSeg {
  uint64_t b;
  uint32_t len;
  const uint64_t* src;    // keys (in place), when isrc is null
  const uint32_t* isrc;   // 4-byte ids (slots or the fill's), if any
  uint32_t j;  // the update (the keys' high word when they are formed from ids)
};

#ifndef DDM_BM_THREADS
#define DDM_BM_THREADS 1024
#endif
#ifndef DDM_BM_WAVES
#define DDM_BM_WAVES 8
#endif
constexpr int kBmThreads = DDM_BM_THREADS;
constexpr uint32_t kBmPre = 8192 / kBmThreads;  // ids per thread loaded ahead, per segment
// staging words past the entry starts (a long segment's chunk is those and
// the entry starts' words: two barriers per chunk; at 2048 two workgroups
// still fit a compute unit's 160 KiB of LDS up to about 522,000 ids)
constexpr uint32_t kBmLong = 2048;
// most uint4 entries per thread: ids below 2^19 (narrow), below 2^20
constexpr uint32_t kBmRNarrow = (kMaxBitWords / 2) / 4 / kBmThreads;
constexpr uint32_t kBmRWide = kMaxBitWords / 4 / kBmThreads;

// LDS of the bitmap sort: the bitmap (uint4 entries), a 16-bit start per
// entry (padded to 8 bytes), then kBmLong + 4 more words; a long segment is
// staged over the entry starts and those words (the last one spare)
constexpr size_t bitmap_lds_bytes(uint32_t words) {
  return (size_t)((words + 3) / 4) * sizeof(uint4) +
         (size_t)(((words + 3) / 4 + 3) / 4) * 4 * sizeof(uint16_t) +
         (size_t)(kBmLong + 4) * sizeof(uint32_t);
}
static_assert(bitmap_lds_bytes(kMaxBitWords) +
                      (kBmRWide * (kBmThreads / kWave) + 1) * sizeof(uint32_t) <=
                  160 * 1024,
              "the widest bitmap sort fits one compute unit's LDS");

// MAXR: most uint4 entries per thread (kBmRNarrow or kBmRWide); SLOTS:
// segments may be read from the slots of the single-pass form
template <uint32_t MAXR, bool SLOTS>
__global__ __launch_bounds__(kBmThreads) __attribute__((amdgpu_waves_per_eu(DDM_BM_WAVES)))
void segsort_bitmap_kernel(const uint64_t* __restrict__ off, uint32_t m,
                           uint64_t* __restrict__ out, SegSrc S,
                           const uint32_t* __restrict__ lists,
                           const uint32_t* __restrict__ list_count, uint32_t words) {
  extern __shared__ uint4 bm4[];
  const uint32_t w4 = (words + 3) / 4;
  uint32_t* bits = reinterpret_cast<uint32_t*>(bm4);  // bitmap, then staging
  uint16_t* ep = reinterpret_cast<uint16_t*>(bm4 + w4);  // entry starts within blocks
  const uint32_t cap = w4 * 4;  // staging capacity (ids)
  constexpr uint32_t NW = kBmThreads / kWave;
  __shared__ uint32_t part[MAXR * NW];
  __shared__ uint32_t s_hi;
  const uint32_t cntl = list_count[1];
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const uint32_t R = min(MAXR, (w4 + kBmThreads - 1) / kBmThreads);
  const uint32_t G = gridDim.x;
  const uint32_t* l1 = lists + m;
  constexpr uint32_t PRE = kBmPre * kBmThreads;  // ids held in registers

  auto list_at = [&](uint32_t li) { return li < cntl ? buf_u32(l1 + li) : 0u; };
  auto meta_of = [&](uint32_t li, uint32_t jv) {
    BmMeta q{0, 0, 0, 0, 0, 0};
    if (li < cntl) {
      const uint32_t j = uniform_v(jv);
      q.j = j;
      q.b = buf_u64(off + j);
      q.elo = buf_u32(reinterpret_cast<const uint32_t*>(off + j + 1));
      if (SLOTS) {
        q.sb = buf_u64(S.so.base + j);
        q.selo = S.so.cap ? buf_u32(S.so.cap + j)
                          : buf_u32(reinterpret_cast<const uint32_t*>(S.so.base + j + 1));
        q.cnt = buf_u32(S.cnt + j);
      }
    }
    return q;
  };
  // a segment's keys are in its slot when every hit fits there, else in place
  auto seg_of = [&](uint32_t li, const BmMeta& q) {
    BmSeg g{0, 0, out, nullptr, 0};
    if (li >= cntl) return g;
    g.j = uniform_v(q.j);
    g.b = uniform_v64(q.b);
    g.len = uniform_v(q.elo) - (uint32_t)g.b;
    g.src = out + g.b;
    if (S.ids) g.isrc = S.ids + g.b;
    if (SLOTS) {
      // slot room: min(base + cap, limit) - base (cap form), else next base - base
      const uint64_t sb = uniform_v64(q.sb);
      uint64_t room;
      if (S.so.cap) {
        const uint64_t cp = uniform_v(q.selo);
        room = S.so.limit > sb ? min(cp, S.so.limit - sb) : 0ull;
      } else {
        room = (uint32_t)(uniform_v(q.selo) - (uint32_t)sb);
      }
      if ((uint64_t)uniform_v(q.cnt) <= room) g.isrc = S.slots + sb;
    }
    return g;
  };
  // kBmPre ids per thread from key index `first` on (key first + tid + r *
  // kBmThreads), through a buffer resource over the segment's len keys (len
  // <= n <= 2^20, so len * 8 fits).  The range check covers the lane's
  // offset register, not the scalar offset: a round wholly inside the
  // segment keeps its round offset scalar (one address register for all
  // such loads); a round the end falls in or lies beyond puts the whole
  // offset in the lane's register, so that a lane past the end loads 0 and
  // touches no memory.  Every round issues one load whatever the length, so
  // the wait counts before the ids are used do not depend on it (from the
  // fill's 4-byte ids when there are: contiguous words)
  auto load_ids = [&](const BmSeg& g, uint32_t first, uint32_t (&v)[kBmPre]) {
    const uint32_t w = g.isrc ? (uint32_t)sizeof(uint32_t) : (uint32_t)sizeof(uint64_t);
    const __amdgpu_buffer_rsrc_t rs =
        g.isrc ? buf_rsrc(g.isrc, g.len * w) : buf_rsrc(g.src, g.len * w);
#pragma unroll
    for (uint32_t r = 0; r < kBmPre; ++r) {
      const uint32_t k0 = first + r * kBmThreads;
      const bool whole = k0 + kBmThreads <= g.len;
      const uint32_t vo = whole ? tid * w : (k0 + tid) * w;
      const uint32_t so = whole ? k0 * w : 0u;
      v[r] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)vo, (int)so, 0);
    }
  };
  auto load_hi = [&](const BmSeg& g) {  // key 0's high word (the update)
    if (g.isrc) return g.j;
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(
        buf_rsrc(g.src, g.len * (uint32_t)sizeof(uint64_t)), 0, 4, 0);
  };
  // rounds wholly past the end are skipped (uniform); in the last one a
  // lane past the end ORs 0 (its loaded id is 0)
  auto mark = [&](const uint32_t (&v)[kBmPre], uint32_t first, uint32_t len) {
#pragma unroll
    for (uint32_t r = 0; r < kBmPre; ++r) {
      if (first + r * kBmThreads >= len) break;
      const uint32_t bit = first + tid + r * kBmThreads < len ? 1u << (v[r] & 31u) : 0u;
      atomicOr(&bits[v[r] >> 5], bit);
    }
  };

  BmMeta mt;    // offsets of the segment two ahead of the one being sorted
  uint32_t jn;  // list entry of the segment three ahead

  // one segment: ids holds its first ids (loaded two segments ago); on
  // return it holds those of the segment two on, g and hi are updated alike
  auto body = [&](uint32_t li, uint32_t (&ids)[kBmPre], uint32_t& hi, BmSeg& g) {
    const BmSeg cg = g;
    if (tid == 0) s_hi = hi;
    mark(ids, 0u, cg.len);
    for (uint32_t first = PRE; first < cg.len; first += PRE) {
      uint32_t more[kBmPre];
      load_ids(cg, first, more);
      mark(more, first, cg.len);
    }
    __syncthreads();  // every id of the segment is read and marked

    // the segment two on and the offsets of the one after it
    const BmSeg g2 = seg_of(li + 2 * G, mt);
    mt = meta_of(li + 3 * G, jn);
    jn = list_at(li + 4 * G);

    // marks per entry: the entry's start within its (block, wave) and the
    // wave totals
#pragma unroll 1
    for (uint32_t r = 0; r < R; ++r) {
      const uint32_t x = r * kBmThreads + tid;
      const uint32_t c = x < w4 ? popc4(bm4[x]) : 0u;
      const uint32_t inc = wave_scan_dpp(c);
      if (x < w4) ep[x] = (uint16_t)(inc - c);
      if (lane == kWave - 1) part[r * NW + wave] = inc;
    }
    __syncthreads();
    // every wave: exclusive prefix of the R * NW totals in (block, wave)
    // order (= entry order): one per lane when they fit a wavefront (then a
    // rank takes its group's start with one shuffle), else two per lane
    constexpr bool ONE = MAXR * NW <= kWave;
    uint32_t a0, a1, ex0;
    if constexpr (ONE) {
      a0 = lane < R * NW ? part[lane] : 0u;
      a1 = 0u;
      ex0 = wave_scan_dpp(a0) - a0;
    } else {
      const uint32_t e0 = 2 * lane, e1 = 2 * lane + 1;
      a0 = e0 < R * NW ? part[e0] : 0u;
      a1 = e1 < R * NW ? part[e1] : 0u;
      ex0 = wave_scan_dpp(a0 + a1) - a0 - a1;
    }
    // place of id among the segment's ids (its block's start from the lane
    // holding that block's prefix)
    auto rank = [&](uint32_t id) {
      const uint32_t e = id >> 7, blk = e >> 6;
      const uint4 q = bm4[e];
      // marks below bit b = id % 128 of the entry: in its 64-bit half below
      // b % 64, and the whole lower half when b >= 64
      const uint64_t lo = (uint64_t)q.x | ((uint64_t)q.y << 32);
      const uint64_t hi = (uint64_t)q.z | ((uint64_t)q.w << 32);
      const uint64_t mk = (1ull << (id & 63u)) - 1ull;
      const bool up = (id & 64u) != 0;
      const uint32_t below = (uint32_t)__popcll(lo & (up ? ~0ull : mk)) +
                             (uint32_t)__popcll(hi & (up ? mk : 0ull));
      if constexpr (ONE) {
        return (uint32_t)__shfl((int)ex0, (int)blk, kWave) + (uint32_t)ep[e] + below;
      } else {
        const uint32_t pl = blk >> 1;
        const uint32_t exl = (uint32_t)__shfl((int)ex0, (int)pl, kWave);
        const uint32_t a0l = (uint32_t)__shfl((int)a0, (int)pl, kWave);
        return ((blk & 1u) ? exl + a0l : exl) + (uint32_t)ep[e] + below;
      }
    };
    const uint64_t jhi = (uint64_t)s_hi << 32;
    uint64_t* dst = out + cg.b;
    if (cg.len > PRE) {
      // a segment longer than the register window: its ids are read back
      // from the bitmap in order (the keys in memory may already be
      // overwritten), chunk by chunk through a staging array over the entry
      // starts (only the ranks of the register window read them) and the
      // kBmLong words after them.  Per entry block, a wave whose positions
      // miss the chunk skips it; else the lanes take their set bits lowest
      // first, the k-th in step k of a loop as long as the wave's fullest
      // entry (a lane out of bits or of the chunk writes the spare slot)
      uint32_t* const lst = reinterpret_cast<uint32_t*>(ep);
      const uint32_t lcap = 2u * ((w4 + 3) / 4) + kBmLong;  // spare slot lst[lcap]
      for (uint32_t cbase = 0; cbase < cg.len; cbase += lcap) {
        const uint32_t cend = min(cbase + lcap, cg.len);
#pragma unroll 1
        for (uint32_t r = 0; r < R; ++r) {
          const uint32_t eidx = r * NW + wave;
          uint32_t wstart, wtot;
          if constexpr (ONE) {
            wstart = (uint32_t)__builtin_amdgcn_readlane((int)ex0, (int)eidx);
            wtot = (uint32_t)__builtin_amdgcn_readlane((int)a0, (int)eidx);
          } else {
            const uint32_t pl = eidx >> 1;
            const uint32_t exl = (uint32_t)__builtin_amdgcn_readlane((int)ex0, (int)pl);
            const uint32_t a0l = (uint32_t)__builtin_amdgcn_readlane((int)a0, (int)pl);
            const uint32_t a1l = (uint32_t)__builtin_amdgcn_readlane((int)a1, (int)pl);
            wstart = (eidx & 1u) ? exl + a0l : exl;
            wtot = (eidx & 1u) ? a1l : a0l;
          }
          if (wtot == 0 || wstart >= cend || wstart + wtot <= cbase) continue;
          const uint32_t x = r * kBmThreads + tid;
          const uint4 q = x < w4 ? bm4[x] : make_uint4(0u, 0u, 0u, 0u);
          const uint32_t c = popc4(q);
          const uint32_t p0 = wstart + wave_scan_dpp(c) - c;
          const uint32_t maxc = wave_max_dpp(c);
          uint64_t lo = (uint64_t)q.x | ((uint64_t)q.y << 32);
          uint64_t hi2 = (uint64_t)q.z | ((uint64_t)q.w << 32);
          for (uint32_t k = 0; k < maxc; ++k) {
            const bool in_lo = lo != 0;
            const uint64_t w = in_lo ? lo : hi2;
            const uint32_t bit = (uint32_t)__builtin_ctzll(w | (1ull << 63)) + (in_lo ? 0u : 64u);
            const uint64_t wc = w & (w - 1);
            lo = in_lo ? wc : lo;
            hi2 = in_lo ? hi2 : wc;
            const uint32_t p = p0 + k;
            const bool ok = k < c && p >= cbase && p < cend;
            lst[ok ? p - cbase : lcap] = x * 128u + bit;
          }
        }
        __syncthreads();
        for (uint32_t i = tid; i < cend - cbase; i += kBmThreads) dst[cbase + i] = jhi | lst[i];
        __syncthreads();  // staging free; at the end the bitmap is no longer read
      }
#pragma unroll 1
      for (uint32_t r = 0; r < R; ++r) {
        const uint32_t x = r * kBmThreads + tid;
        if (x < w4) bm4[x] = make_uint4(0u, 0u, 0u, 0u);
      }
      __syncthreads();  // bitmap clear
    } else {
      // (every lane of a wave ranks, valid id or not: rank reads other lanes)
      uint32_t pos[kBmPre];
#pragma unroll
      for (uint32_t r = 0; r < kBmPre; ++r) {
        pos[r] = ~0u;
        if (r * kBmThreads >= cg.len) continue;
        const uint32_t rk = rank(ids[r]);
        pos[r] = tid + r * kBmThreads < cg.len ? rk : ~0u;
      }
      __syncthreads();  // every id ranked: the bitmap is no longer read

      for (uint32_t cbase = 0; cbase < cg.len; cbase += cap) {
        const uint32_t cn = min(cap, cg.len - cbase);
        if (cbase == 0) {
          // clear the array past the staged positions (whole entries)
          const uint32_t x0 = (cn + 3) / 4;
#pragma unroll 1
          for (uint32_t r = 0; r < R; ++r) {
            const uint32_t x = r * kBmThreads + tid;
            if (x >= x0 && x < w4) bm4[x] = make_uint4(0u, 0u, 0u, 0u);
          }
        }
#pragma unroll
        for (uint32_t r = 0; r < kBmPre; ++r)
          if (pos[r] - cbase < cn) bits[pos[r] - cbase] = ids[r] + 1u;
        __syncthreads();
        for (uint32_t i = tid; i < cn; i += kBmThreads) {
          const uint32_t v = bits[i];
          if (v) dst[cbase + i] = jhi | (v - 1u);
          bits[i] = 0u;
        }
        // the words of the last staged entry past the staged positions
        if (tid < 4 && cn + tid < 4 * ((cn + 3) / 4)) bits[cn + tid] = 0u;
        __syncthreads();  // array clear; s_hi and part read
      }
    }
    // the ids of the segment two on load while the next one is sorted
    g = g2;
    load_ids(g, 0u, ids);
    hi = load_hi(g);
  };

  uint32_t li = blockIdx.x;
  if (li >= cntl) return;
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t x = r * kBmThreads + tid;
    if (x < w4) bm4[x] = make_uint4(0u, 0u, 0u, 0u);
  }
  __syncthreads();
  // prologue: the first two segments' ids, the third's offsets, the fourth's
  // list entry
  BmSeg g0 = seg_of(li, meta_of(li, list_at(li)));
  uint32_t ids0[kBmPre], hi0;
  load_ids(g0, 0u, ids0);
  hi0 = load_hi(g0);
  BmSeg g1 = seg_of(li + G, meta_of(li + G, list_at(li + G)));
  uint32_t ids1[kBmPre], hi1;
  load_ids(g1, 0u, ids1);
  hi1 = load_hi(g1);
  mt = meta_of(li + 2 * G, list_at(li + 2 * G));
  jn = list_at(li + 3 * G);
  for (;;) {
    body(li, ids0, hi0, g0);
    li += G;
    if (li >= cntl) break;
    body(li, ids1, hi1, g1);
    li += G;
    if (li >= cntl) break;
  }
}

__global__ void copy_ids_kernel(const uint64_t* __restrict__ in, uint32_t* __restrict__ outp,
                                uint64_t K) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) outp[i] = (uint32_t)in[i];
}

__global__ void zero_u32_kernel(uint32_t* __restrict__ p, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

__global__ void copy_counts_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ o,
                                   uint32_t m) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) o[i] = in[i];
}

// --------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------
struct MatchPlan {
  uint32_t traversal;
  uint32_t block;
};

static ddm_status parse_opts(const ddm_match_opts* o, MatchPlan* p) {
  p->traversal = DDM_TRAVERSE_TILE;
  p->block = 256;
  if (!o) return DDM_OK;
  for (int i = 0; i < 6; ++i)
    if (o->reserved[i]) {
      set_detail("ddm_match_opts: reserved fields must be zero");
      return DDM_E_INVALID_ARG;
    }
  if (o->traversal > DDM_TRAVERSE_TILE) {
    set_detail("ddm_match_opts: unknown traversal");
    return DDM_E_INVALID_ARG;
  }
  if (o->traversal != DDM_TRAVERSE_AUTO) p->traversal = o->traversal;
  if (o->block) {
    if (o->block != 64 && o->block != 128 && o->block != 256 && o->block != 512 &&
        o->block != 1024) {
      set_detail("ddm_match_opts: block must be 64..1024, a power of two");
      return DDM_E_INVALID_ARG;
    }
    p->block = o->block;
  }
  return DDM_OK;
}


template <int D, bool FILL>
static ddm_status launch_traverse(const MatchPlan& P, const TreeDev& T, const float* ulo,
                                  const float* uhi, uint32_t m, const UpdSet& US,
                                  const uint8_t* kstar, const SegOut& O, hipStream_t s) {
  if (US.total == 0) return DDM_OK;
  if (P.traversal == DDM_TRAVERSE_LANE) {
    ProfScope ps(FILL ? "traverse_lane_fill" : "traverse_lane_count", s);
    const uint32_t bs = P.block;
    lane_kernel<D, FILL><<<(US.total + bs - 1) / bs, bs, 0, s>>>(T, ulo, uhi, m, US, kstar, O);
    DDM_LAUNCHED("lane_kernel");
  } else {
    ProfScope ps(FILL ? (US.qpt == 1 ? "traverse_tile1_fill"
                                     : US.tstart ? "traverse_tile_fill_balanced"
                                                 : "traverse_tile_fill")
                      : (O.skey && US.tmap ? "traverse_tile_count_stash" : "traverse_tile_count"),
                 s);
    if (US.tmap || US.tstart) {
      // at most one partial tile per bucket; a tile list cut by predicted
      // work as well has at most one more tile per crossing of a multiple
      // of H (at most total / H = m * kCutDiv / 128), and never more tiles
      // than updates
      uint32_t tiles = (US.total + 63u) / 64u + std::min<uint32_t>(US.total, kBuckets);
      if (US.tstart)
        tiles = (uint32_t)std::min<uint64_t>(
            (uint64_t)tiles + ((uint64_t)US.total * kCutDiv + 127u) / 128u + 1u, US.total);
      const uint32_t grid = (tiles + kTileWaves - 1) / kTileWaves;
      if (!FILL && O.skey)
        tile_bucket_kernel<D, false, true><<<grid, kTileWaves * kWave, 0, s>>>(T, ulo, uhi, m,
                                                                              US, O);
      else
        tile_bucket_kernel<D, FILL><<<grid, kTileWaves * kWave, 0, s>>>(T, ulo, uhi, m, US, O);
      DDM_LAUNCHED("tile_bucket_kernel");
    } else {
      const uint32_t tiles = (US.total + US.qpt - 1) / US.qpt + D;
      tile_kernel<D, FILL><<<(tiles + kTileWaves - 1) / kTileWaves, kTileWaves * kWave, 0, s>>>(
          T, ulo, uhi, m, US, O);
      DDM_LAUNCHED("tile_kernel");
    }
  }
  return DDM_OK;
}

template <bool FILL>
static ddm_status traverse_any(uint32_t d, const MatchPlan& P, const TreeDev& T,
                               const float* ulo, const float* uhi, uint32_t m, const UpdSet& US,
                               const uint8_t* kstar, const SegOut& O, hipStream_t s) {
  switch (d) {
    case 1: return launch_traverse<1, FILL>(P, T, ulo, uhi, m, US, kstar, O, s);
    case 2: return launch_traverse<2, FILL>(P, T, ulo, uhi, m, US, kstar, O, s);
    case 3: return launch_traverse<3, FILL>(P, T, ulo, uhi, m, US, kstar, O, s);
    default: return launch_traverse<4, FILL>(P, T, ulo, uhi, m, US, kstar, O, s);
  }
}

// pinned host words for the single device->host read of a match
// (one small block per host thread, kept for the life of the process)
struct HostWords {
  uint64_t* p = nullptr;
};
static thread_local HostWords g_host;

static ddm_status host_words(uint64_t** out) {
  if (!g_host.p) {
    hipError_t e = hipHostMalloc((void**)&g_host.p, 64, hipHostMallocDefault);
    if (e != hipSuccess) {
      g_host.p = nullptr;
      (void)hipGetLastError();
      set_detail("pinned host allocation failed");
      return DDM_E_NOMEM;
    }
  }
  *out = g_host.p;
  return DDM_OK;
}

// Common front half: validation/BITS, update order, counts, scan, K readback.
struct MatchState {
  Scratch sc;
  uint32_t* cmin = nullptr;
  uint8_t* kstar = nullptr;
  uint32_t* rank = nullptr;
  uint32_t* bucket = nullptr;
  uint32_t* bhist = nullptr;
  uint32_t* bcnt = nullptr;  // bucket counters, kCntPad words apart
  uint32_t* perm = nullptr;
  uint32_t* gstart = nullptr;
  uint32_t* gcount = nullptr;
  uint32_t* shape = nullptr;  // cell shape (log2 B1) of each probe dimension
  uint32_t* pb = nullptr;     // per update: candidate position bounds (d > 1)
  bool pb_ok = false;
  bool balanced = false;  // the learned single pass runs the work-cut tile list
  int32_t* flag = nullptr;
  uint32_t* cnt = nullptr;
  uint64_t* off = nullptr;
  uint64_t K = 0;
  uint32_t m = 0;
  // single-pass (learned sizing) state
  bool learned = false;
  Scratch slots_sc;
  float* X = nullptr;
  uint32_t* cap = nullptr;
  uint64_t* soff = nullptr;
  uint32_t* slots = nullptr;  // the single pass's 4-byte ids
  uint64_t budget = 0;
  uint64_t slots_total = 0;
  uint32_t* perm_ovf = nullptr;
  uint32_t* govf = nullptr;
  // tiles cut by predicted work (learned): list, bucket of each, count
  uint32_t* wtile = nullptr;   // work in perm order, then cut flags
  uint64_t* cwork = nullptr;   // exclusive scan of the work, then of the flags
  uint32_t* tstart = nullptr;
  uint32_t* tbuck = nullptr;
  uint32_t novf = 0;
  // bucket-aligned tiles
  uint32_t* tprefix = nullptr;
  uint32_t* tmap = nullptr;
  uint32_t* maxcnt = nullptr;  // device: the largest count (longest segment)
  uint64_t maxseg = ~0ull;     // host copy after the count
  // stash of the count traversal (plain path, d > 1): usable when complete
  Scratch stash_sc;
  bool stash = false;
  uint64_t* skey = nullptr;
  uint32_t* srank = nullptr;
  uint32_t* sused = nullptr;
  uint32_t* snext = nullptr;
  uint32_t smax = 0;
  uint32_t sfirst = 0;
  uint32_t sslice = 0;
  uint32_t stiles = 0;     // tiles that ran
  uint32_t sused_max = 0;  // most counted chunks used in one slice
  bool stash_ok = false;
  // no allocation of any kind (the scratch is external, the read-back goes
  // to pageable host memory): the no-allocation entry point
  bool noalloc = false;
  explicit MatchState(hipStream_t s) : sc(s), slots_sc(s), stash_sc(s) {}
  UpdSet all() const {
    UpdSet U{perm, gstart, gcount, m, 64};
    U.boff = bhist;
    U.tprefix = tprefix;
    U.tmap = tmap;
    U.pb = pb_ok ? pb : nullptr;
    if (balanced) {
      U.tstart = tstart;
      U.tbuck = tbuck;
      U.ntiles = cwork + m;
    }
    return U;
  }
};

// zeroes the match's counters; with a stash (snext non-null) also sets the
// slices' next free chunks; for d > 1 (D > 1) the last workgroup also picks
// the cell shape of every probe dimension
template <int D>
__global__ __launch_bounds__(1024) void match_init_kernel(
    uint32_t* __restrict__ gcount, int32_t* __restrict__ flag, uint32_t* __restrict__ lists_count,
    uint32_t* __restrict__ bcnt, uint32_t* __restrict__ snext, uint32_t sfirst, uint32_t sslice,
    uint32_t* __restrict__ maxcnt, TreeDev T, const float* __restrict__ ulo,
    const float* __restrict__ uhi, uint32_t m, uint32_t* __restrict__ shape) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kBuckets) bcnt[(size_t)i * kCntPad] = 0;
  if (i < DDM_MAX_D) gcount[i] = 0;
  if (i == 0) {
    *flag = 0;
    *maxcnt = 0;
  }
  if (i < 2) lists_count[i] = 0;
  if (snext && i <= kStashSlices) snext[i] = i < kStashSlices ? sfirst + i * sslice : 0u;
  if constexpr (D > 1) {
    if (blockIdx.x == gridDim.x - 1) sample_cell_shape<D, 1024>(T, ulo, uhi, m, shape);
  }
}

// the words the host reads after the count: dst[0] = K, dst[1] = the tree's
// and the updates' flags; with a stash, dst[2] = (tiles << 32) | most
// counted chunks used in one slice, dst[3] = overflow; dst[4] = the largest
// count
__global__ void gather_flags_kernel(const int32_t* __restrict__ tflag,
                                    const int32_t* __restrict__ uflag,
                                    const uint64_t* __restrict__ off, uint32_t m,
                                    uint64_t* __restrict__ dst,
                                    const uint32_t* __restrict__ snext,
                                    const uint32_t* __restrict__ tprefix, uint32_t sfirst,
                                    uint32_t sslice, const uint32_t* __restrict__ maxcnt) {
  // one wavefront; the lanes share the slices
  const uint32_t lane = threadIdx.x;
  if (lane == 0) {
    dst[4] = *maxcnt;
    dst[0] = off[m];
    dst[1] = (uint64_t)(uint32_t)(*tflag) | ((uint64_t)(uint32_t)(*uflag) << 32);
  }
  if (snext) {
    uint32_t mx = 0;
    for (uint32_t s = lane; s < kStashSlices; s += kWave)
      mx = max(mx, min(snext[s] - (sfirst + s * sslice), sslice));
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, kWave));
    if (lane == 0) {
      dst[2] = ((uint64_t)tprefix[kBuckets] << 32) | mx;
      dst[3] = snext[kStashSlices];
    }
  }
}

template <int D>
static ddm_status launch_probe(const TreeDev& T, const float* ulo, const float* uhi, uint32_t m,
                               MatchState& st, hipStream_t s) {
  if (D == 1) {
    ProfScope ps("bits", s);
    bits1_kernel<<<(m + 255) / 256, 256, 0, s>>>(T, ulo, uhi, m, st.cmin, st.kstar, st.bucket,
                                                 st.rank, st.bcnt, st.flag);
    DDM_LAUNCHED("bits1_kernel");
  } else {
    ProfScope ps("probe", s);
    probe_kernel<D><<<(m + kProbeThreads - 1) / kProbeThreads, kProbeThreads, 0, s>>>(
        T, ulo, uhi, m, st.shape, st.kstar, st.bucket, st.rank, st.bcnt, st.flag,
        reinterpret_cast<uint2*>(st.pb));
    DDM_LAUNCHED("probe_kernel");
  }
  return DDM_OK;
}

// updates whose hits exceeded their slots, kept in their probe group
__global__ __launch_bounds__(256) void overflow_kernel(UpdSet US, uint32_t d, SegOut O,
                                                       const uint32_t* __restrict__ cnt,
                                                       uint32_t* __restrict__ perm_ovf,
                                                       uint32_t* __restrict__ govf) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t pi, g;
  if (!upd_index(US, t, d, &pi, &g)) return;
  const uint32_t j = US.perm[pi];
  uint64_t b, e;
  seg_bounds(O, j, &b, &e);
  if ((uint64_t)cnt[j] > e - b) perm_ovf[US.gstart[g] + atomicAdd(&govf[g], 1u)] = j;
}

__global__ void learned_init_kernel(uint32_t* __restrict__ govf) {
  if (threadIdx.x < DDM_MAX_D) govf[threadIdx.x] = 0;
}

__global__ void learned_words_kernel(const uint32_t* __restrict__ govf,
                                     const uint64_t* __restrict__ soff, uint32_t m,
                                     uint64_t* __restrict__ dst) {
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int g = 0; g < DDM_MAX_D; ++g) t += govf[g];
    dst[2] = t;
    dst[3] = soff[m];
  }
}

// stashed hits to their final places: out[off[j] + rank] (the same places
// the fill traversal gives them).  Thread e covers entry e of the static
// chunks of the `tiles` tiles that ran, then, slice by slice, the first
// `used` counted chunks of each slice.
__global__ void stash_scatter_kernel(const uint64_t* __restrict__ skey,
                                     const uint32_t* __restrict__ srank,
                                     const uint32_t* __restrict__ sused,
                                     const uint32_t* __restrict__ snext, uint32_t tiles,
                                     uint32_t sfirst, uint32_t sslice, uint32_t used,
                                     const uint64_t* __restrict__ off, uint32_t m,
                                     uint64_t* __restrict__ out) {
  const uint64_t e0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nstatic = (uint64_t)tiles * kStashStatic * kStashChunk;
  uint64_t e;
  if (e0 < nstatic) {
    e = e0;
  } else {
    if (used == 0) return;
    const uint64_t r = e0 - nstatic, per = (uint64_t)used * kStashChunk;
    const uint32_t sl = (uint32_t)(r / per);
    if (sl >= kStashSlices) return;
    const uint32_t c = sfirst + sl * sslice + (uint32_t)((r % per) / kStashChunk);
    if (c >= snext[sl]) return;
    e = (uint64_t)c * kStashChunk + r % kStashChunk;
  }
  const uint32_t c = (uint32_t)(e / kStashChunk);
  if ((uint32_t)(e % kStashChunk) >= sused[c]) return;
  const uint64_t key = skey[e];
  const uint32_t j = (uint32_t)(key >> 32);
  if (j >= m) return;
  const uint64_t dst = off[j] + srank[e];
  if (dst < off[j + 1]) out[dst] = key;
}

// stash entries: the hint (a caller's capacity) or 4 per update, plus one
// chunk per possible tile (a tile's last chunk is partly used; the bound is
// the launch's own: one tile per 64 updates plus one partial tile per
// bucket), plus 64Ki
static uint64_t stash_tiles(uint32_t m) {
  return (m + 63u) / 64u + std::min<uint64_t>(m, kBuckets);
}
// counted chunks per slice: room for the hint (or 4 hits per update) plus
// one partly used chunk per tile and 1024 more, over the slices
static uint32_t stash_slice(uint32_t m, uint64_t hint) {
  const uint64_t dyn = std::min<uint64_t>(std::max<uint64_t>(hint, 4ull * m), kStashMaxEntries);
  const uint64_t c = (dyn + kStashChunk - 1) / kStashChunk + stash_tiles(m) * kStashGrab + 1024;
  return (uint32_t)((c + kStashSlices - 1) / kStashSlices);
}

size_t match_stash_bytes(uint32_t m) {
  const uint64_t c = stash_tiles(m) * kStashStatic + (uint64_t)stash_slice(m, 0) * kStashSlices;
  return (size_t)(c * kStashChunk * 12 + c * 4 + 1024);
}

// The scratch layout of the match's front half: one reservation per piece
// (each rounded up to 256 bytes by Scratch), then the pieces taken in the
// same sizes.  The match, the no-allocation match and the host-only layout
// check (ddm_match_scratch_bytes) share these two functions, so that a
// piece taken without its reservation is caught on the host.
struct FrontPieces {
  uint64_t* stmp = nullptr;
  uint32_t* lists = nullptr;
  uint32_t* lists_count = nullptr;
  uint64_t* dwords = nullptr;
};

static size_t front_max_tiles(uint32_t m) { return ((size_t)m + 63) / 64 + kBuckets; }

static void front_reserve(Scratch& sc, uint32_t m, bool learned) {
  if (learned) {
    sc.reserve(sizeof(float) * (size_t)m * kFeatures);  // X
    sc.reserve(sizeof(uint32_t) * m);                   // cap
    sc.reserve(sizeof(uint64_t) * (m + 1));             // soff
    sc.reserve(sizeof(uint32_t) * m);                   // perm_ovf
    sc.reserve(sizeof(uint32_t) * DDM_MAX_D);           // govf
    sc.reserve(sizeof(uint32_t) * m);                   // work / cut flags
    sc.reserve(sizeof(uint64_t) * (m + 1));             // their scan
    sc.reserve(sizeof(uint32_t) * ((size_t)m + 1));     // tile starts
    sc.reserve(sizeof(uint32_t) * m);                   // tile buckets
  }
  sc.reserve(sizeof(uint32_t) * m);          // cmin
  sc.reserve(m);                             // kstar
  sc.reserve(sizeof(uint32_t) * m);          // rank
  sc.reserve(sizeof(uint32_t) * m);          // bucket
  sc.reserve(sizeof(uint32_t) * m);          // perm
  sc.reserve(sizeof(uint32_t) * kBuckets);   // bucket offsets
  sc.reserve(sizeof(uint32_t) * kBuckets * kCntPad);  // bucket counters
  sc.reserve(sizeof(uint32_t) * DDM_MAX_D);  // gstart
  sc.reserve(sizeof(uint32_t) * DDM_MAX_D);  // gcount
  sc.reserve(sizeof(uint32_t) * DDM_MAX_D);  // shape
  sc.reserve(sizeof(int32_t));               // flag
  sc.reserve(sizeof(uint32_t) * m);          // cnt
  sc.reserve(sizeof(uint64_t) * (m + 1));    // off
  sc.reserve(sizeof(uint64_t) * scan_tmp_words(m));
  sc.reserve(sizeof(uint32_t) * 2 * (size_t)m);  // segment lists
  sc.reserve(sizeof(uint32_t) * 2);              // segment list counts
  sc.reserve(sizeof(uint64_t) * 8);              // device words for readback
  sc.reserve(sizeof(uint32_t));                  // largest count
  sc.reserve(sizeof(uint32_t) * (kBuckets + 1));     // tile prefix
  sc.reserve(sizeof(uint32_t) * front_max_tiles(m));  // tile -> bucket
  sc.reserve(sizeof(uint32_t) * 2 * (size_t)m);       // candidate position bounds
}

static void front_take(Scratch& sc, MatchState& st, uint32_t m, bool learned, FrontPieces* fp) {
  st.cmin = sc.take<uint32_t>(m);
  st.kstar = sc.take<uint8_t>(m);
  st.rank = sc.take<uint32_t>(m);
  st.bucket = sc.take<uint32_t>(m);
  st.perm = sc.take<uint32_t>(m);
  st.bhist = sc.take<uint32_t>(kBuckets);
  st.bcnt = sc.take<uint32_t>((size_t)kBuckets * kCntPad);
  st.gstart = sc.take<uint32_t>(DDM_MAX_D);
  st.gcount = sc.take<uint32_t>(DDM_MAX_D);
  st.shape = sc.take<uint32_t>(DDM_MAX_D);
  st.m = m;
  st.flag = sc.take<int32_t>(1);
  st.cnt = sc.take<uint32_t>(m);
  st.off = sc.take<uint64_t>(m + 1);
  fp->stmp = sc.take<uint64_t>(scan_tmp_words(m));
  fp->lists = sc.take<uint32_t>(2 * (size_t)m);
  fp->lists_count = sc.take<uint32_t>(2);
  fp->dwords = sc.take<uint64_t>(8);
  st.maxcnt = sc.take<uint32_t>(1);
  st.tprefix = sc.take<uint32_t>(kBuckets + 1);
  st.tmap = sc.take<uint32_t>(front_max_tiles(m));
  st.pb = sc.take<uint32_t>(2 * (size_t)m);
  if (learned) {
    st.X = sc.take<float>((size_t)m * kFeatures);
    st.cap = sc.take<uint32_t>(m);
    st.soff = sc.take<uint64_t>(m + 1);
    st.perm_ovf = sc.take<uint32_t>(m);
    st.govf = sc.take<uint32_t>(DDM_MAX_D);
    st.wtile = sc.take<uint32_t>(m);
    st.cwork = sc.take<uint64_t>(m + 1);
    st.tstart = sc.take<uint32_t>((size_t)m + 1);
    st.tbuck = sc.take<uint32_t>(m);
  }
}

// the count traversal's stash: sizes (into st) and reservations, then takes
static void stash_reserve(Scratch& sc, MatchState& st, uint32_t m, uint64_t hint) {
  st.sfirst = (uint32_t)(stash_tiles(m) * kStashStatic);
  st.sslice = stash_slice(m, hint);
  st.smax = st.sfirst + st.sslice * kStashSlices;
  const uint64_t e = (uint64_t)st.smax * kStashChunk;
  sc.reserve(sizeof(uint64_t) * e);
  sc.reserve(sizeof(uint32_t) * e);
  sc.reserve(sizeof(uint32_t) * st.smax);
  sc.reserve(sizeof(uint32_t) * (kStashSlices + 1));
}

static void stash_take(Scratch& sc, MatchState& st) {
  const uint64_t e = (uint64_t)st.smax * kStashChunk;
  st.skey = sc.take<uint64_t>(e);
  st.srank = sc.take<uint32_t>(e);
  st.sused = sc.take<uint32_t>(st.smax);
  st.snext = sc.take<uint32_t>(kStashSlices + 1);
}

static ddm_status front_half(const ddm_tree* t, const float* ulo, const float* uhi, uint32_t m,
                             const MatchPlan& P, MatchState& st, uint32_t* counts_out,
                             uint32_t** lists, uint32_t** lists_count, hipStream_t s,
                             const ddm_predictor* pred = nullptr, uint64_t budget = 0,
                             bool want_stash = false, uint64_t stash_hint = 0,
                             const ArenaGrant* grant = nullptr) {
  const uint32_t d = tree_d(t);
  const TreeDev T = tree_dev(t);
  Scratch& sc = st.sc;
  // the single pass replaces the count traversal, which only exists for d > 1
  st.learned = pred != nullptr && d > 1;
  front_reserve(sc, m, st.learned);
  if (!sc.commit()) return DDM_E_NOMEM;
  FrontPieces fp;
  front_take(sc, st, m, st.learned, &fp);
  uint64_t* stmp = fp.stmp;
  *lists = fp.lists;
  *lists_count = fp.lists_count;
  uint64_t* dwords = fp.dwords;
  if (!sc.fits()) return scratch_overrun("front_half");
  st.pb_ok = d > 1;  // written by the probe kernel (d = 1 takes exact counts instead)
  if (st.learned) {
    learned_init_kernel<<<1, 64, 0, s>>>(st.govf);
    DDM_LAUNCHED("learned_init_kernel");
  }

  // the count traversal's stash (plain path, d > 1, tile traversal)
  st.stash = !st.learned && d > 1 && want_stash && !counts_out &&
             P.traversal == DDM_TRAVERSE_TILE;
  if (st.stash) {
    // the count traversal also keeps every hit, so that no fill traversal
    // is needed when they all fit; without the memory it only counts
    stash_reserve(st.stash_sc, st, m, stash_hint);
    if (!st.stash_sc.commit()) {
      set_detail("");
      st.stash = false;
    } else {
      stash_take(st.stash_sc, st);
      if (!st.stash_sc.fits()) return scratch_overrun("stash");
    }
  }
  {
    uint32_t* sn = st.stash ? st.snext : nullptr;
    const unsigned g = kBuckets / 1024;
#define DDM_INIT(DD)                                                                          \
  match_init_kernel<DD><<<g, 1024, 0, s>>>(st.gcount, st.flag, *lists_count, st.bcnt, sn,    \
                                          st.sfirst, st.sslice, st.maxcnt, T, ulo, uhi, m, \
                                          st.shape)
    switch (d) {
      case 1: DDM_INIT(1); break;
      case 2: DDM_INIT(2); break;
      case 3: DDM_INIT(3); break;
      default: DDM_INIT(4); break;
    }
#undef DDM_INIT
    DDM_LAUNCHED("match_init_kernel");
  }
  ddm_status r;
  switch (d) {
    case 1: r = launch_probe<1>(T, ulo, uhi, m, st, s); break;
    case 2: r = launch_probe<2>(T, ulo, uhi, m, st, s); break;
    case 3: r = launch_probe<3>(T, ulo, uhi, m, st, s); break;
    default: r = launch_probe<4>(T, ulo, uhi, m, st, s); break;
  }
  if (r != DDM_OK) return r;
  {
    ProfScope ps("order", s);
    uint32_t* tp = P.traversal == DDM_TRAVERSE_TILE ? st.tprefix : nullptr;
    // the counts of the d probe dimensions' buckets, dense, into bhist (the
    // scan turns them into offsets in place)
    const uint32_t nbd = d * kBucketsPerDim;
    bucket_gather_kernel<<<(nbd + 255) / 256, 256, 0, s>>>(st.bcnt, nbd, st.bhist);
    DDM_LAUNCHED("bucket_gather_kernel");
    switch (d) {
      case 1: bucket_scan_kernel<8><<<1, 1024, 0, s>>>(st.bhist, m, st.gstart, st.gcount, tp); break;
      case 2: bucket_scan_kernel<16><<<1, 1024, 0, s>>>(st.bhist, m, st.gstart, st.gcount, tp); break;
      case 3: bucket_scan_kernel<24><<<1, 1024, 0, s>>>(st.bhist, m, st.gstart, st.gcount, tp); break;
      default: bucket_scan_kernel<32><<<1, 1024, 0, s>>>(st.bhist, m, st.gstart, st.gcount, tp); break;
    }
    DDM_LAUNCHED("bucket_scan_kernel");
    const bool tiles = P.traversal == DDM_TRAVERSE_TILE;
    const uint32_t nb = tiles ? d * kBucketsPerDim : 0u;
    bucket_scatter_kernel<<<(std::max(m, nb) + 255) / 256, 256, 0, s>>>(
        st.bucket, st.rank, m, st.bhist, st.perm, st.tprefix, tiles ? st.tmap : nullptr, nb);
    DDM_LAUNCHED("bucket_scatter_kernel");
  }
  // per-update counts
  const uint32_t* counts = st.cmin;
  SegOut SO{};
  if (st.learned) {
    // predicted capacities -> slot offsets; one traversal writes hits into
    // the slots and counts every hit exactly
    r = tree_ensure_features(t, s);
    if (r != DDM_OK) return r;
    r = launch_features(tree_feat(t), d, ulo, uhi, m, st.X, s);
    if (r != DDM_OK) return r;
    r = launch_mlp_forward(predictor_params(pred), st.X, m, 1, predictor_delta(pred), 1u << 30,
                           nullptr, st.cap, s);
    if (r != DDM_OK) return r;
    r = scan_u32_u64(st.cap, st.soff, m, stmp, s);
    if (r != DDM_OK) return r;
    if (P.traversal == DDM_TRAVERSE_TILE) {
      ProfScope ps("balance", s);
      const unsigned g = (m + 255) / 256;
      work_in_order_kernel<<<g, 256, 0, s>>>(st.perm, st.cap, m, st.wtile);
      DDM_LAUNCHED("work_in_order_kernel");
      r = scan_u32_u64(st.wtile, st.cwork, m, stmp, s);
      if (r != DDM_OK) return r;
      tile_cut_kernel<<<g, 256, 0, s>>>(st.perm, st.bucket, st.bhist, st.cwork, m, st.wtile);
      DDM_LAUNCHED("tile_cut_kernel");
      r = scan_u32_u64(st.wtile, st.cwork, m, stmp, s);
      if (r != DDM_OK) return r;
      tile_list_kernel<<<g, 256, 0, s>>>(st.perm, st.bucket, st.wtile, st.cwork, m, st.tstart,
                                         st.tbuck);
      DDM_LAUNCHED("tile_list_kernel");
      st.balanced = true;
    }
    {
      // arena sized to the predicted total, or to the caller's budget if
      // that is smaller (one extra stream synchronization); updates whose
      // slots fall beyond the arena overflow and are filled exactly later
      uint64_t* hw0 = nullptr;
      r = host_words(&hw0);
      if (r != DDM_OK) return r;
      DDM_HIP(hipMemcpyAsync(hw0 + 4, st.soff + m, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      DDM_HIP(hipStreamSynchronize(s));
      budget = budget == 0 ? hw0[4] : std::min<uint64_t>(budget, hw0[4]);
      // a caller that accounts device memory grants the arena before it is
      // allocated (it may wait there, or grant less)
      if (grant) {
        const uint64_t g = (*grant)(budget);
        if (g == kArenaRefused) {
          set_detail("slot arena not granted");
          return DDM_E_NOMEM;
        }
        budget = std::min<uint64_t>(budget, g);
      }
    }
    st.budget = budget;
    st.slots_sc.reserve(sizeof(uint32_t) * (budget ? budget : 1));
    if (!st.slots_sc.commit()) return DDM_E_NOMEM;
    st.slots = st.slots_sc.take<uint32_t>(budget ? budget : 1);
    if (!st.slots_sc.fits()) return scratch_overrun("slot arena");
    SO.base = st.soff;
    SO.cap = st.cap;
    SO.limit = budget;
    SO.cnt = st.cnt;
    SO.out = nullptr;
    SO.ids = st.slots;  // the hits' subscription ids, 4 bytes each
    r = traverse_any<true>(d, P, T, ulo, uhi, m, st.all(), st.kstar, SO, s);
    if (r != DDM_OK) return r;
    counts = st.cnt;
  } else if (d > 1) {
    SegOut O{};
    O.cnt = st.cnt;
    if (st.stash) {
      O.skey = st.skey;
      O.srank = st.srank;
      O.sused = st.sused;
      O.snext = st.snext;
      O.sfirst = st.sfirst;
      O.sslice = st.sslice;
    }
    r = traverse_any<false>(d, P, T, ulo, uhi, m, st.all(), st.kstar, O, s);
    if (r != DDM_OK) return r;
    counts = st.cnt;
  }
  if (counts_out) {
    copy_counts_kernel<<<(m + 255) / 256, 256, 0, s>>>(counts, counts_out, m);
    DDM_LAUNCHED("copy_counts_kernel");
  }
  r = scan_u32_u64(counts, st.off, m, stmp, s, st.maxcnt);
  if (r != DDM_OK) return r;
  gather_flags_kernel<<<1, 64, 0, s>>>(tree_flag(t), st.flag, st.off, m, dwords,
                                       st.stash ? st.snext : nullptr, st.tprefix, st.sfirst,
                                       st.sslice, st.maxcnt);
  DDM_LAUNCHED("gather_flags_kernel");
  if (st.learned) {
    overflow_kernel<<<(m + 255) / 256, 256, 0, s>>>(st.all(), d, SO, st.cnt, st.perm_ovf,
                                                    st.govf);
    DDM_LAUNCHED("overflow_kernel");
    learned_words_kernel<<<1, 64, 0, s>>>(st.govf, st.soff, m, dwords);
    DDM_LAUNCHED("learned_words_kernel");
  }
  uint64_t hw_local[8] = {};
  uint64_t* hw = hw_local;
  if (!st.noalloc) {
    r = host_words(&hw);
    if (r != DDM_OK) return r;
  }
  DDM_HIP(hipMemcpyAsync(hw, dwords, 5 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  DDM_HIP(hipStreamSynchronize(s));
  const uint64_t flags = hw[1];
  st.K = hw[0];
  st.maxseg = hw[4];
  if (st.learned) {
    st.novf = (uint32_t)hw[2];
    st.slots_total = hw[3];
  }
  if (st.stash) {
    st.stash_ok = hw[3] == 0;
    st.stiles = (uint32_t)(hw[2] >> 32);
    st.sused_max = (uint32_t)hw[2];
  }
  if (flags & (uint64_t)(uint32_t)kFlagSortTimeout) {
    set_detail("tree build: a radix sort look-back wait gave up");
    return DDM_E_DEVICE;
  }
  if (flags & 0xffffffffull) {
    set_detail("subscription coordinates: NaN/inf or lo > hi");
    return DDM_E_INVALID_INPUT;
  }
  if (flags >> 32) {
    set_detail("update coordinates: NaN/inf or lo > hi");
    return DDM_E_INVALID_INPUT;
  }
  return DDM_OK;
}

static ddm_status check_common(const ddm_tree* t, const float* ulo, const float* uhi,
                               uint32_t m) {
  if (!t) {
    set_detail("tree is NULL");
    return DDM_E_INVALID_ARG;
  }
  if (m > 0 && (!ulo || !uhi)) {
    set_detail("NULL update coordinate pointer");
    return DDM_E_INVALID_ARG;
  }
  if (m >= 0x80000000u) {
    set_detail("m must be below 2^31");
    return DDM_E_INVALID_ARG;
  }
  int cur = -1;
  DDM_HIP(hipGetDevice(&cur));
  if (cur != tree_device(t)) {
    set_detail("the current device is not the tree's device");
    return DDM_E_INVALID_ARG;
  }
  return DDM_OK;
}

ddm_status sort_segments(const uint64_t* off, uint32_t m, uint64_t* out, uint64_t K, uint32_t n,
                         uint32_t* lists, uint32_t* lists_count, hipStream_t s, const SegSrc& S,
                         uint64_t max_len = ~0ull, Scratch* tmp_sc = nullptr);

// the bitmap kernels' LDS exceeds the default dynamic LDS limit
ddm_status ensure_segsort_attr() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] {
    err = hipFuncSetAttribute((const void*)segsort_big_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(kMaxBitWords * sizeof(uint32_t)));
    const void* fns[4] = {(const void*)segsort_bitmap_kernel<kBmRNarrow, false>,
                          (const void*)segsort_bitmap_kernel<kBmRNarrow, true>,
                          (const void*)segsort_bitmap_kernel<kBmRWide, false>,
                          (const void*)segsort_bitmap_kernel<kBmRWide, true>};
    for (int i = 0; i < 4 && err == hipSuccess; ++i)
      err = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bitmap_lds_bytes(i < 2 ? kMaxBitWords / 2 : kMaxBitWords));
  });
  if (err != hipSuccess) return hip_fail(err, "hipFuncSetAttribute", __FILE__, __LINE__);
  return DDM_OK;
}

ddm_status sort_segments_inplace(const uint64_t* off, uint32_t m, uint64_t* out, uint32_t n,
                                 uint32_t* lists, uint32_t* lists_count, hipStream_t s) {
  // ids of at most 2^20: one bitmap window, no id copy (K is not needed)
  if (n > kMaxBitWords * 32) {
    set_detail("segment sort without host sizing needs n <= 2^20");
    return DDM_E_INVALID_ARG;
  }
  return sort_segments(off, m, out, 0, n, lists, lists_count, s, SegSrc{});
}

ddm_status sort_segments_keys(const uint64_t* off, uint32_t m, uint64_t* out, uint64_t K,
                              uint32_t n, uint32_t* lists, uint32_t* lists_count, hipStream_t s) {
  return sort_segments(off, m, out, K, n, lists, lists_count, s, SegSrc{});
}

// max_len: the longest segment if known; size classes that cannot occur
// are not launched.  tmp_sc: where the id copy of the bitmap sort comes from
// (an external scratch in the no-allocation match), else allocated here.
ddm_status sort_segments(const uint64_t* off, uint32_t m, uint64_t* out, uint64_t K, uint32_t n,
                         uint32_t* lists, uint32_t* lists_count, hipStream_t s,
                         const SegSrc& S, uint64_t max_len, Scratch* tmp_sc) {
  ProfScope ps("segsort", s);
  if (S.ids || S.slots)
    segsort_small_kernel<true><<<(m + 255) / 256, 256, 0, s>>>(off, m, out, S, lists, lists_count);
  else
    segsort_small_kernel<false><<<(m + 255) / 256, 256, 0, s>>>(off, m, out, S, lists,
                                                                lists_count);
  DDM_LAUNCHED("segsort_small_kernel");
  if (max_len <= 32) return DDM_OK;  // every segment sorted in registers
  if (S.ids || S.slots)
    segsort_mid_kernel<true><<<4096, kSegWaves * kWave, 0, s>>>(off, out, S, lists, lists_count);
  else
    segsort_mid_kernel<false><<<4096, kSegWaves * kWave, 0, s>>>(off, out, S, lists, lists_count);
  DDM_LAUNCHED("segsort_mid_kernel");
  if (max_len <= kSegMid) return DDM_OK;
  ddm_status r = ensure_segsort_attr();
  if (r != DDM_OK) return r;
  if (n <= kMaxBitWords * 32) {
    // one bitmap window: every listed segment by the bitmap kernel, one
    // resident workgroup per slot of the chip (each takes every G-th segment)
    const uint32_t words = std::max<uint32_t>(1u, (n + 31) / 32);
    const size_t lds = bitmap_lds_bytes(words);
    int dev = 0, cus = 0, per = 0;
    DDM_HIP(hipGetDevice(&dev));
    DDM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const bool narrow = n <= kMaxBitWords * 16, slots = S.slots != nullptr;
    const void* fn = narrow ? (slots ? (const void*)segsort_bitmap_kernel<kBmRNarrow, true>
                                     : (const void*)segsort_bitmap_kernel<kBmRNarrow, false>)
                            : (slots ? (const void*)segsort_bitmap_kernel<kBmRWide, true>
                                     : (const void*)segsort_bitmap_kernel<kBmRWide, false>);
    DDM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kBmThreads, lds));
    const uint32_t grid = (uint32_t)std::max(1, cus * std::max(1, per));
    if (narrow && slots)
      segsort_bitmap_kernel<kBmRNarrow, true><<<grid, kBmThreads, lds, s>>>(off, m, out, S, lists,
                                                                   lists_count, words);
    else if (narrow)
      segsort_bitmap_kernel<kBmRNarrow, false><<<grid, kBmThreads, lds, s>>>(off, m, out, S, lists,
                                                                    lists_count, words);
    else if (slots)
      segsort_bitmap_kernel<kBmRWide, true><<<grid, kBmThreads, lds, s>>>(off, m, out, S, lists,
                                                                   lists_count, words);
    else
      segsort_bitmap_kernel<kBmRWide, false><<<grid, kBmThreads, lds, s>>>(off, m, out, S, lists,
                                                                    lists_count, words);
    DDM_LAUNCHED("segsort_bitmap_kernel");
    return DDM_OK;
  }
  const uint32_t words = std::min<uint32_t>(kMaxBitWords, (n + 31) / 32);
  uint32_t* tmp = nullptr;
  Scratch local(s);
  Scratch& sc = tmp_sc ? *tmp_sc : local;
  if (n > words * 32) {
    // ids of in-place segments are read window by window from a copy
    sc.reserve(sizeof(uint32_t) * K);
    if (!sc.commit()) return DDM_E_NOMEM;
    tmp = sc.take<uint32_t>(K);
    if (!sc.fits()) return scratch_overrun("segment sort");
    copy_ids_kernel<<<(unsigned)((K + 255) / 256), 256, 0, s>>>(out, tmp, K);
    DDM_LAUNCHED("copy_ids_kernel");
  }
  {
    // buckets of 2^shift consecutive ids, as many as the class's largest
    // segment has keys (fewer when n is smaller)
    uint32_t bits = 0;
    while (bits < 32 && (1ull << bits) < n) ++bits;
    const uint32_t s12 = bits > 12 ? bits - 12 : 0, s13 = bits > 13 ? bits - 13 : 0,
                   s14 = bits > 14 ? bits - 14 : 0;
    segsort_bucket_kernel<4096><<<2048, 4096 / kPerThread, 0, s>>>(off, m, out, S, lists,
                                                                   lists_count, s12);
    DDM_LAUNCHED("segsort_bucket_kernel<4096>");
    if (max_len > 4096) {
      segsort_bucket_kernel<8192><<<1024, 8192 / kPerThread, 0, s>>>(off, m, out, S, lists,
                                                                     lists_count, s13);
      DDM_LAUNCHED("segsort_bucket_kernel<8192>");
    }
    if (max_len > 8192) {
      segsort_bucket_kernel<16384><<<512, 16384 / kPerThread, 0, s>>>(off, m, out, S, lists,
                                                                      lists_count, s14);
      DDM_LAUNCHED("segsort_bucket_kernel<16384>");
    }
  }
  segsort_big_kernel<<<512, kBigThreads, words * sizeof(uint32_t), s>>>(off, m, out, S, lists,
                                                                        lists_count, tmp, n, words);
  DDM_LAUNCHED("segsort_big_kernel");
  return DDM_OK;
}

}  // namespace ddm

using namespace ddm;

struct ddm_pending {
  ddm::MatchState st;
  ddm::MatchPlan plan;
  const ddm_tree* t;
  const float* ulo;
  const float* uhi;
  uint32_t m;
  uint32_t* lists = nullptr;
  uint32_t* lists_count = nullptr;
  hipStream_t s;
  explicit ddm_pending(hipStream_t st_) : st(st_), s(st_) {}
};

static ddm_status match_begin(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                              uint32_t m, uint64_t* out_count, void* stream,
                              const ddm_match_opts* opts, ddm_pending** out_pending,
                              bool want_stash, uint64_t stash_hint);

extern "C" ddm_status ddm_match_begin(const ddm_tree* t, const float* upd_lo,
                                      const float* upd_hi, uint32_t m, uint64_t* out_count,
                                      void* stream, const ddm_match_opts* opts,
                                      ddm_pending** out_pending) {
  return match_begin(t, upd_lo, upd_hi, m, out_count, stream, opts, out_pending, true, 0);
}

static ddm_status match_begin(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                              uint32_t m, uint64_t* out_count, void* stream,
                              const ddm_match_opts* opts, ddm_pending** out_pending,
                              bool want_stash, uint64_t stash_hint) {
  set_detail("");
  if (!out_count || !out_pending) {
    set_detail("out_count / out_pending is NULL");
    return DDM_E_INVALID_ARG;
  }
  *out_count = 0;
  *out_pending = nullptr;
  ddm_status r = check_common(t, upd_lo, upd_hi, m);
  if (r != DDM_OK) return r;
  MatchPlan P;
  r = parse_opts(opts, &P);
  if (r != DDM_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  if (m == 0 || tree_n(t) == 0) {
    if (tree_n(t) != 0) return ddm_tree_check(t);
    return DDM_OK;
  }
  ddm_pending* pd = new (std::nothrow) ddm_pending(s);
  if (!pd) return DDM_E_NOMEM;
  pd->plan = P;
  pd->t = t;
  pd->ulo = upd_lo;
  pd->uhi = upd_hi;
  pd->m = m;
  r = front_half(t, upd_lo, upd_hi, m, P, pd->st, nullptr, &pd->lists, &pd->lists_count, s,
                 nullptr, 0, want_stash, stash_hint);
  if (r != DDM_OK) {
    delete pd;
    return r;
  }
  *out_count = pd->st.K;
  *out_pending = pd;
  return DDM_OK;
}

static ddm_status learned_begin(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                                uint32_t m, const ddm_predictor* pred, uint64_t slot_budget,
                                uint64_t* out_count, void* stream, const ddm_match_opts* opts,
                                ddm_pending** out_pending, const ArenaGrant* grant) {
  set_detail("");
  if (!out_count || !out_pending || !pred) {
    set_detail("out_count / out_pending / predictor is NULL");
    return DDM_E_INVALID_ARG;
  }
  *out_count = 0;
  *out_pending = nullptr;
  ddm_status r = check_common(t, upd_lo, upd_hi, m);
  if (r != DDM_OK) return r;
  if (tree_d(t) > 3) {
    set_detail("learned sizing supports d <= 3");
    return DDM_E_INVALID_ARG;
  }
  if (predictor_device(pred) != tree_device(t)) {
    set_detail("predictor and tree live on different devices");
    return DDM_E_INVALID_ARG;
  }
  MatchPlan P;
  r = parse_opts(opts, &P);
  if (r != DDM_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  if (m == 0 || tree_n(t) == 0) {
    if (tree_n(t) != 0) return ddm_tree_check(t);
    return DDM_OK;
  }
  ddm_pending* pd = new (std::nothrow) ddm_pending(s);
  if (!pd) return DDM_E_NOMEM;
  pd->plan = P;
  pd->t = t;
  pd->ulo = upd_lo;
  pd->uhi = upd_hi;
  pd->m = m;
  r = front_half(t, upd_lo, upd_hi, m, P, pd->st, nullptr, &pd->lists, &pd->lists_count, s, pred,
                 slot_budget, false, 0, grant);
  if (r != DDM_OK) {
    delete pd;
    return r;
  }
  *out_count = pd->st.K;
  *out_pending = pd;
  return DDM_OK;
}

extern "C" ddm_status ddm_match_learned_begin(const ddm_tree* t, const float* upd_lo,
                                              const float* upd_hi, uint32_t m,
                                              const ddm_predictor* pred, uint64_t slot_budget,
                                              uint64_t* out_count, void* stream,
                                              const ddm_match_opts* opts,
                                              ddm_pending** out_pending) {
  return learned_begin(t, upd_lo, upd_hi, m, pred, slot_budget, out_count, stream, opts,
                       out_pending, nullptr);
}

namespace ddm {
ddm_status match_learned_begin_granted(const ddm_tree* t, const float* upd_lo,
                                       const float* upd_hi, uint32_t m,
                                       const ddm_predictor* pred, uint64_t* out_count,
                                       hipStream_t s, const ddm_match_opts* opts,
                                       ddm_pending** out_pending, const ArenaGrant& grant) {
  return learned_begin(t, upd_lo, upd_hi, m, pred, 0, out_count, s, opts, out_pending, &grant);
}
}  // namespace ddm

extern "C" ddm_status ddm_pending_info(const ddm_pending* pd, uint64_t* slots, uint64_t* budget,
                                       uint32_t* overflowed) {
  if (!pd) return DDM_E_INVALID_ARG;
  if (slots) *slots = pd->st.slots_total;
  if (budget) *budget = pd->st.budget;
  if (overflowed) *overflowed = pd->st.novf;
  return DDM_OK;
}

extern "C" ddm_status ddm_features(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                                   uint32_t m, float* X, void* stream) {
  set_detail("");
  ddm_status r = check_common(t, upd_lo, upd_hi, m);
  if (r != DDM_OK) return r;
  if (m > 0 && !X) return DDM_E_INVALID_ARG;
  if (tree_d(t) > 3) {
    set_detail("features are defined for d <= 3");
    return DDM_E_INVALID_ARG;
  }
  if (tree_n(t) == 0) {
    set_detail("features need a non-empty subscription set");
    return DDM_E_INVALID_ARG;
  }
  r = tree_ensure_features(t, (hipStream_t)stream);
  if (r != DDM_OK) return r;
  return launch_features(tree_feat(t), tree_d(t), upd_lo, upd_hi, m, X, (hipStream_t)stream);
}

// The fill of the plain two-pass form on tiles balanced by the exact
// counts (the cut of the learned single pass): the arrays are reserved in
// bsc first (with whatever else the caller reserves), then taken and
// filled; U gets the tile list.  bsc must outlive the fill.
static void balance_reserve(uint32_t m, Scratch& bsc) {
  bsc.reserve(sizeof(uint32_t) * m);                  // work, then cut flags
  bsc.reserve(sizeof(uint64_t) * ((size_t)m + 1));    // their scans
  bsc.reserve(sizeof(uint32_t) * ((size_t)m + 1));    // tile starts
  bsc.reserve(sizeof(uint32_t) * m);                  // tile buckets
  bsc.reserve(sizeof(uint64_t) * scan_tmp_words(m));  // scan scratch
}

static ddm_status balance_fill_tiles(const MatchState& st, uint32_t m, Scratch& bsc, UpdSet* U,
                                     hipStream_t s) {
  uint32_t* w = bsc.take<uint32_t>(m);
  uint64_t* cw = bsc.take<uint64_t>((size_t)m + 1);
  uint32_t* ts = bsc.take<uint32_t>((size_t)m + 1);
  uint32_t* tb = bsc.take<uint32_t>(m);
  uint64_t* tmp = bsc.take<uint64_t>(scan_tmp_words(m));
  if (!bsc.fits()) return scratch_overrun("fill tile balance");
  ProfScope ps("balance", s);
  const unsigned g = (m + 255) / 256;
  work_in_order_kernel<<<g, 256, 0, s>>>(st.perm, st.cnt, m, w);
  DDM_LAUNCHED("work_in_order_kernel");
  ddm_status r = scan_u32_u64(w, cw, m, tmp, s);
  if (r != DDM_OK) return r;
  tile_cut_kernel<<<g, 256, 0, s>>>(st.perm, st.bucket, st.bhist, cw, m, w);
  DDM_LAUNCHED("tile_cut_kernel");
  r = scan_u32_u64(w, cw, m, tmp, s);
  if (r != DDM_OK) return r;
  tile_list_kernel<<<g, 256, 0, s>>>(st.perm, st.bucket, w, cw, m, ts, tb);
  DDM_LAUNCHED("tile_list_kernel");
  U->tstart = ts;
  U->tbuck = tb;
  U->ntiles = cw + m;
  return DDM_OK;
}

extern "C" ddm_status ddm_match_finish(ddm_pending* pd, uint64_t* out_pairs, uint64_t capacity) {
  set_detail("");
  if (!pd) return DDM_OK;  // empty match: nothing to do
  ddm_status r = DDM_OK;
  if (pd->st.K > capacity) {
    set_detail("result larger than capacity");
    r = DDM_E_CAPACITY;
  } else if (pd->st.K > 0 && !out_pairs) {
    set_detail("out_pairs is NULL");
    r = DDM_E_INVALID_ARG;
  } else if (pd->st.K > 0) {
    const TreeDev T = tree_dev(pd->t);
    MatchState& st = pd->st;
    SegOut O{};
    O.base = st.off;
    O.out = out_pairs;
    Scratch fsc(pd->s);        // the fill's ids and tile lists (until the sort has run)
    uint32_t* fids = nullptr;  // the fill's 4-byte ids, if it writes them
    if (st.learned) {
      // segments that fitted their slots are moved into place by the
      // segment sort; overflowed ones are filled in place here
      if (st.novf > 0) {
        // overflowed updates are few and scattered, and each has many
        // hits: one wavefront per update scans its candidate range
        UpdSet OV{st.perm_ovf, st.gstart, st.govf, st.novf, 1};
        OV.pb = st.all().pb;
        MatchPlan TP = pd->plan;
        TP.traversal = DDM_TRAVERSE_TILE;
        r = traverse_any<true>(tree_d(pd->t), TP, T, pd->ulo, pd->uhi, pd->m, OV, st.kstar, O,
                               pd->s);
      }
    } else if (st.stash_ok) {
      ProfScope ps("stash_scatter", pd->s);
      const uint64_t n = ((uint64_t)st.stiles * kStashStatic +
                          (uint64_t)st.sused_max * kStashSlices) * kStashChunk;
      if (n > 0) {
        stash_scatter_kernel<<<(unsigned)((n + 255) / 256), 256, 0, pd->s>>>(
            st.skey, st.srank, st.sused, st.snext, st.stiles, st.sfirst, st.sslice,
            st.sused_max, st.off, pd->m, out_pairs);
        const hipError_t le = hipGetLastError();
        if (le != hipSuccess) r = hip_fail(le, "stash_scatter_kernel", __FILE__, __LINE__);
      }
    } else {
      // Not in the no-allocation form: (1) the fill writes 4-byte ids,
      // which the segment sort expands into keys (half the bytes written by
      // the fill and read by the sort), when the sort can read ids (every
      // id below 2^20); (2) tiles cut by the exact counts, when a tile of 64
      // of the longest segments could exceed the cut's H.
      UpdSet U = st.all();
      const uint64_t H = std::max<uint64_t>(
          (2ull * 64ull * st.K) / ((uint64_t)pd->m * kCutDiv), kCutMinHits);
      const bool use_ids = !st.noalloc && tree_n(pd->t) <= kMaxBitWords * 32;
      const bool bal = !st.noalloc && pd->plan.traversal == DDM_TRAVERSE_TILE && U.tmap &&
                       (st.maxseg == ~0ull || 64ull * st.maxseg > H);
      if (use_ids) fsc.reserve(sizeof(uint32_t) * st.K);
      if (bal) balance_reserve(pd->m, fsc);
      if ((use_ids || bal) && !fsc.commit()) r = DDM_E_NOMEM;
      if (r == DDM_OK && use_ids) {
        fids = fsc.take<uint32_t>(st.K);
        if (!fsc.fits()) r = scratch_overrun("fill ids");
      }
      if (r == DDM_OK && bal) r = balance_fill_tiles(st, pd->m, fsc, &U, pd->s);
      O.ids = fids;
      if (r == DDM_OK)
        r = traverse_any<true>(tree_d(pd->t), pd->plan, T, pd->ulo, pd->uhi, pd->m, U, st.kstar,
                               O, pd->s);
    }
    if (r == DDM_OK) {
      SegSrc S{};
      S.ids = fids;
      if (st.learned) {
        S.slots = st.slots;
        S.so.base = st.soff;
        S.so.cap = st.cap;
        S.so.limit = st.budget;
        S.cnt = st.cnt;
      }
      r = sort_segments(st.off, pd->m, out_pairs, st.K, tree_n(pd->t), pd->lists,
                        pd->lists_count, pd->s, S, st.maxseg);
    }
  }
  delete pd;
  return r;
}

extern "C" void ddm_match_abort(ddm_pending* pd) { delete pd; }

extern "C" ddm_status ddm_match_ex(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                                   uint32_t m, uint64_t* out_pairs, uint64_t capacity,
                                   uint64_t* out_count, void* stream,
                                   const ddm_match_opts* opts) {
  ddm_pending* pd = nullptr;
  // the capacity sizes the count traversal's stash (none for a size query,
  // for capacities beyond what a stash may hold, or for dense results)
  ddm_status r = match_begin(t, upd_lo, upd_hi, m, out_count, stream, opts, &pd,
                             capacity > 0 && capacity <= kStashMaxEntries &&
                                 capacity <= kStashMaxPerUpdate * m,
                             capacity);
  if (r != DDM_OK) return r;
  if (*out_count > capacity) {
    ddm_match_abort(pd);
    set_detail("result larger than capacity");
    return DDM_E_CAPACITY;
  }
  return ddm_match_finish(pd, out_pairs, capacity);
}

extern "C" ddm_status ddm_match(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                                uint32_t m, uint64_t* out_pairs, uint64_t capacity,
                                uint64_t* out_count, void* stream) {
  return ddm_match_ex(t, upd_lo, upd_hi, m, out_pairs, capacity, out_count, stream, nullptr);
}

extern "C" ddm_status ddm_count(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                                uint32_t m, uint32_t* counts, uint64_t* out_total, void* stream,
                                const ddm_match_opts* opts) {
  set_detail("");
  if (out_total) *out_total = 0;
  ddm_status r = check_common(t, upd_lo, upd_hi, m);
  if (r != DDM_OK) return r;
  if (m > 0 && !counts) {
    set_detail("counts is NULL");
    return DDM_E_INVALID_ARG;
  }
  MatchPlan P;
  r = parse_opts(opts, &P);
  if (r != DDM_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  if (m == 0) return tree_n(t) ? ddm_tree_check(t) : DDM_OK;
  if (tree_n(t) == 0) {
    zero_u32_kernel<<<(m + 255) / 256, 256, 0, s>>>(counts, m);
    DDM_LAUNCHED("zero_u32_kernel");
    return DDM_OK;
  }
  MatchState st(s);
  uint32_t *lists = nullptr, *lists_count = nullptr;
  r = front_half(t, upd_lo, upd_hi, m, P, st, counts, &lists, &lists_count, s);
  if (r != DDM_OK) return r;
  if (out_total) *out_total = st.K;
  return DDM_OK;
}

// --------------------------------------------------------------------------
// Scratch sizes of the match, computed on the host by the same layout
// functions the match uses (a dry run: no memory, no GPU).
// --------------------------------------------------------------------------
extern "C" ddm_status ddm_match_scratch_bytes(uint32_t m, uint32_t d, uint32_t form,
                                              uint64_t hint, uint64_t* bytes) {
  set_detail("");
  if (!bytes || d < 1 || d > DDM_MAX_D || form > DDM_SCRATCH_LEARNED || m >= 0x80000000u) {
    set_detail("ddm_match_scratch_bytes: bad argument");
    return DDM_E_INVALID_ARG;
  }
  *bytes = 0;
  if (m == 0) return DDM_OK;
  MatchState st(nullptr);
  const bool learned = form == DDM_SCRATCH_LEARNED && d > 1;
  Scratch& sc = st.sc;
  sc.dry_run();
  front_reserve(sc, m, learned);
  if (!sc.commit()) return DDM_E_NOMEM;
  FrontPieces fp;
  front_take(sc, st, m, learned, &fp);
  if (!sc.fits()) return scratch_overrun("front_half");
  uint64_t total = sc.want_;
  if (form == DDM_SCRATCH_STASH && d > 1) {
    Scratch& ss = st.stash_sc;
    ss.dry_run();
    stash_reserve(ss, st, m, hint);
    if (!ss.commit()) return DDM_E_NOMEM;
    stash_take(ss, st);
    if (!ss.fits()) return scratch_overrun("stash");
    total += ss.want_;
  }
  *bytes = total;
  return DDM_OK;
}

namespace ddm {

// --------------------------------------------------------------------------
// The plain match (count -> scan -> fill, no stash) with every piece of
// scratch carved from caller-provided device memory [base, base + cap) and
// the count read back into pageable host memory: no allocation of any kind.
// Errors: DDM_E_INVALID_ARG when the layout for m updates does not fit in
// cap bytes, or when the id copy of the bitmap sort (more than 2^20
// subscriptions and a segment beyond kSegMid pairs: 4 bytes per pair) does
// not fit in what is left, both before anything is written; otherwise as
// ddm_match.
// --------------------------------------------------------------------------
ddm_status match_external_scratch(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                                  uint32_t m, uint64_t* out_pairs, uint64_t capacity,
                                  uint64_t* out_count, hipStream_t s, char* base, size_t cap,
                                  const char* who) {
  set_detail("");
  if (!out_count) {
    set_detail("out_count is NULL");
    return DDM_E_INVALID_ARG;
  }
  *out_count = 0;
  ddm_status r = check_common(t, upd_lo, upd_hi, m);
  if (r != DDM_OK) return r;
  if (m == 0 || tree_n(t) == 0) {
    if (tree_n(t) != 0) return ddm_tree_check(t);
    return DDM_OK;
  }
  uint64_t need = 0;
  r = ddm_match_scratch_bytes(m, tree_d(t), DDM_SCRATCH_PLAIN, 0, &need);
  if (r != DDM_OK) return r;
  if (need > cap) {
    set_detail(std::string(who) + ": " + std::to_string(m) + " updates need " +
               std::to_string(need) + " bytes of scratch; it holds " + std::to_string(cap));
    return DDM_E_INVALID_ARG;
  }
  MatchPlan P;
  r = parse_opts(nullptr, &P);
  if (r != DDM_OK) return r;
  MatchState st(s);
  st.noalloc = true;
  st.sc.use_external(base, cap);
  uint32_t *lists = nullptr, *lists_count = nullptr;
  r = front_half(t, upd_lo, upd_hi, m, P, st, nullptr, &lists, &lists_count, s, nullptr, 0,
                 false, 0);
  if (r != DDM_OK) return r;
  *out_count = st.K;
  if (st.K > capacity) {
    set_detail("result larger than capacity");
    return DDM_E_CAPACITY;
  }
  if (st.K == 0) return DDM_OK;
  if (!out_pairs) {
    set_detail("out_pairs is NULL");
    return DDM_E_INVALID_ARG;
  }
  const size_t used = st.sc.used_;
  if (tree_n(t) > kMaxBitWords * 32 && st.maxseg > kSegMid &&
      ((sizeof(uint32_t) * st.K + 255) & ~size_t(255)) > cap - used) {
    set_detail(std::string(who) + ": sorting segments over " + std::to_string(kSegMid) +
               " pairs among more than 2^20 subscriptions needs 4 bytes per pair (" +
               std::to_string(st.K) + " pairs) beyond the scratch");
    return DDM_E_INVALID_ARG;
  }
  SegOut O{};
  O.base = st.off;
  O.out = out_pairs;
  const TreeDev T = tree_dev(t);
  r = traverse_any<true>(tree_d(t), P, T, upd_lo, upd_hi, m, st.all(), st.kstar, O, s);
  if (r != DDM_OK) return r;
  Scratch rest(s);
  rest.use_external(base + used, cap - used);
  return sort_segments(st.off, m, out_pairs, st.K, tree_n(t), lists, lists_count, s, SegSrc{},
                       st.maxseg, &rest);
}

}  // namespace ddm
