// Per-tree construction steps shared by the single-tree build (tree.hip) and
// the batched build (batch.hip).  Each step works on one tree (one
// dimension k of one subscription set) described by a TreeJob.
#pragma once

#include "ddm_internal.h"

namespace ddm {

struct TreeJob {
  const float* s_lo;       // the set's lower bounds, dimension-major [d][n]
  const float* s_hi;
  float* rec;              // (n+1) records of 2d floats (tree k order)
  float* maxhi;            // P+1
  float* bmax;             // C
  const uint32_t* id;      // n+1 (sorted payload at positions 1..n)
  const uint32_t* skey_lo; // n sorted keys of lo_k
  const uint32_t* skey_hi; // n sorted keys of hi_k, or null
  uint32_t* sidx_lo;       // ns samples
  uint32_t* sidx_hi;       // ns samples, or null
  uint32_t* quant;         // kQuant quantiles
  uint32_t* maxlen_bits;   // one word: bound of the lengths (float bits)
  uint32_t n, d, k, P, C, H, ns;
  const float* recin;      // optional: the set as n records (lo_0, hi_0, lo_1, ...)
};

constexpr int kChunk = 2048;        // positions per workgroup in a maxhi pass
constexpr int kChunkLog = 11;
constexpr int kTreeThreads = 1024;  // two positions per thread

// samples of the sorted keys for two-level searches, and quantiles; index c
__device__ __forceinline__ void tree_index_item(const TreeJob& J, uint32_t c) {
  if (c < J.ns) {
    J.sidx_lo[c] = J.skey_lo[(size_t)c << 6];
    if (J.skey_hi) J.sidx_hi[c] = J.skey_hi[(size_t)c << 6];
  }
  if (c < kQuant) J.quant[c] = J.skey_lo[(uint32_t)(((uint64_t)c * J.n) / kQuant)];
}

// Pass 0 on chunk c (2048 consecutive positions): gather the records (or,
// with GATHER false, read the records already in place, after extents have
// moved) and compute maxhi for heights 0..10 in LDS, the block maxima
// (height 5 plus the position above) and the length bound.
template <bool GATHER = true>
__device__ __forceinline__ void tree_low_chunk(const TreeJob& J, uint32_t c) {
  __shared__ float mx[kChunk];
  __shared__ uint32_t wlen[kTreeThreads / kWave];
  const uint32_t k = J.k;
  const uint32_t D = J.d;
  float* __restrict__ rec = J.rec;
  const uint32_t* __restrict__ ids = J.id;
  // bound of the segment lengths in dimension k: the float difference rounded
  // to nearest, moved one float up, is >= the exact difference; lengths are
  // >= 0, so their float bits order like unsigned integers
  uint32_t lenb = 0;
  if (GATHER) {
    // every id of the thread's positions is loaded first, then every
    // record (one contiguous record per subscription with recin, else the
    // bounds of each dimension), so that there are two rounds of loads in
    // flight instead of two per position; then the records are written in
    // tree-k order (dimension k first, then the others ascending)
    constexpr uint32_t IT = kChunk / kTreeThreads;
    static_assert(kChunk % kTreeThreads == 0, "whole rounds");
    const float* __restrict__ rin = J.recin;
    uint32_t idx[IT];
    bool ok[IT];
#pragma unroll
    for (uint32_t it = 0; it < IT; ++it) {
      const uint32_t p = c * kChunk + threadIdx.x + it * kTreeThreads;
      ok[it] = p >= 1 && p <= J.n;
      idx[it] = ok[it] ? ids[p] : 0u;
    }
    float val[IT][2 * DDM_MAX_D];
#pragma unroll
    for (uint32_t it = 0; it < IT; ++it)
#pragma unroll
      for (uint32_t q = 0; q < 2 * DDM_MAX_D; ++q)
        val[it][q] = !(ok[it] && q < 2 * D) ? 0.f
                     : rin               ? rin[(size_t)idx[it] * 2 * D + q]
                     : (q & 1u)          ? J.s_hi[(size_t)(q / 2) * J.n + idx[it]]
                                         : J.s_lo[(size_t)(q / 2) * J.n + idx[it]];
#pragma unroll
    for (uint32_t it = 0; it < IT; ++it) {
      const uint32_t r = threadIdx.x + it * kTreeThreads;
      const uint32_t p = c * kChunk + r;
      float h = -INFINITY;
      if (ok[it]) {
        float* dst = rec + (size_t)p * 2 * D;
        float l0 = 0.f;
#pragma unroll
        for (uint32_t kk = 0; kk < DDM_MAX_D; ++kk) {
          if (kk >= D) continue;
          const uint32_t slot = kk == k ? 0u : (kk < k ? kk + 1u : kk);
          dst[2 * slot] = val[it][2 * kk];
          dst[2 * slot + 1] = val[it][2 * kk + 1];
          if (kk == k) {
            l0 = val[it][2 * kk];
            h = val[it][2 * kk + 1];
          }
        }
        if (valid_extent(l0, h)) lenb = max(lenb, __float_as_uint(nextafterf(h - l0, INFINITY)));
      }
      mx[r] = h;
    }
  } else {
    // the records in place (extents moved): dimension k's bounds
    for (uint32_t r = threadIdx.x; r < kChunk; r += kTreeThreads) {
      const uint32_t p = c * kChunk + r;
      float h = -INFINITY;
      if (p >= 1 && p <= J.n) {
        const float* dst = rec + (size_t)p * 2 * D;
        const float l0 = dst[0];
        h = dst[1];
        if (valid_extent(l0, h)) lenb = max(lenb, __float_as_uint(nextafterf(h - l0, INFINITY)));
      }
      mx[r] = h;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lenb = max(lenb, (uint32_t)__shfl_xor((int)lenb, o, kWave));
  if (lane_id() == 0) wlen[threadIdx.x / kWave] = lenb;
  for (int h = 1; h < kChunkLog; ++h) {
    __syncthreads();
    if (h == 1 && threadIdx.x == 0) {
      uint32_t v = 0;
      for (int w = 0; w < kTreeThreads / kWave; ++w) v = max(v, wlen[w]);
      if (v) atomicMax(J.maxlen_bits, v);
    }
    if (h == (int)kBlockLog) {
      // heights < 6 are final and heights >= 6 still hold their own upper
      // bound: block b of the chunk is position 64b plus subtree(64b + 32)
      if (threadIdx.x < kChunk / 64) {
        const uint32_t b = threadIdx.x;
        const uint32_t blk = c * (kChunk / 64) + b;
        if (blk < J.C) J.bmax[blk] = fmaxf(mx[64 * b], mx[64 * b + 32]);
      }
      __syncthreads();
    }
    for (uint32_t r = threadIdx.x; r < kChunk; r += kTreeThreads) {
      if (r != 0 && (uint32_t)__builtin_ctz(r) == (uint32_t)h) {
        const uint32_t half = 1u << (h - 1);
        mx[r] = fmaxf(mx[r], fmaxf(mx[r - half], mx[r + half]));
      }
    }
  }
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < kChunk; r += kTreeThreads) {
    const uint32_t p = c * kChunk + r;
    if (r != 0 && p <= J.P) J.maxhi[p] = mx[r];
  }
}

// Pass with shift S >= 11 on chunk c: positions p = q << S (q in the chunk),
// real heights S .. S+10.  Leaves (odd q) combine the two children of height
// S-1 computed by the previous pass.
__device__ __forceinline__ void tree_high_chunk(const TreeJob& J, uint32_t c, uint32_t S) {
  __shared__ float mx[kChunk];
  const uint32_t D = J.d;
  const uint32_t qmax = J.P >> S;
  const float* __restrict__ rec = J.rec;
  float* __restrict__ maxhi = J.maxhi;
  for (uint32_t r = threadIdx.x; r < kChunk; r += kTreeThreads) {
    const uint32_t q = c * kChunk + r;
    float h = -INFINITY;
    if (r != 0 && q <= qmax) {
      const uint32_t p = q << S;
      if (p <= J.n) h = rec[(size_t)p * 2 * D + 1];
      if (q & 1u) {
        const uint32_t half = 1u << (S - 1);
        h = fmaxf(h, fmaxf(maxhi[p - half], maxhi[p + half]));
      }
    }
    mx[r] = h;
  }
  for (int h = 1; h < kChunkLog; ++h) {
    __syncthreads();
    for (uint32_t r = threadIdx.x; r < kChunk; r += kTreeThreads) {
      if (r != 0 && (uint32_t)__builtin_ctz(r) == (uint32_t)h) {
        const uint32_t half = 1u << (h - 1);
        mx[r] = fmaxf(mx[r], fmaxf(mx[r - half], mx[r + half]));
      }
    }
  }
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < kChunk; r += kTreeThreads) {
    const uint32_t q = c * kChunk + r;
    if (r != 0 && q <= qmax) maxhi[q << S] = mx[r];
  }
}

}  // namespace ddm
