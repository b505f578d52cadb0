// Device-side pieces shared by the single-instance and batched matchers:
// record/query loads, wavefront helpers, the update-set and output-segment
// descriptors, and the body of the tile traversal.
#pragma once

#include "ddm_internal.h"

namespace ddm {

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void load_rec(const float* __restrict__ p, float (&v)[2 * D]) {
  if constexpr (D == 1) {
    const float2 a = *reinterpret_cast<const float2*>(p);
    v[0] = a.x; v[1] = a.y;
  } else if constexpr (D == 2) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  } else if constexpr (D == 3) {
    const float2 a = reinterpret_cast<const float2*>(p)[0];
    const float2 b = reinterpret_cast<const float2*>(p)[1];
    const float2 c = reinterpret_cast<const float2*>(p)[2];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y; v[4] = c.x; v[5] = c.y;
  } else {
    const float4 a = reinterpret_cast<const float4*>(p)[0];
    const float4 b = reinterpret_cast<const float4*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  }
}

// Query j's bounds in record order: probe dimension k first, then the other
// dimensions ascending (slot s >= 1 holds dimension s-1 or s).
template <int D>
__device__ __forceinline__ void load_query(const float* __restrict__ ulo,
                                           const float* __restrict__ uhi, uint32_t m,
                                           uint32_t j, uint32_t k, float (&ql)[D],
                                           float (&qh)[D]) {
  ql[0] = ulo[(size_t)k * m + j];
  qh[0] = uhi[(size_t)k * m + j];
#pragma unroll
  for (int s = 1; s < D; ++s) {
    const uint32_t kk = (uint32_t)(s - 1) + (((uint32_t)(s - 1) >= k) ? 1u : 0u);
    ql[s] = ulo[(size_t)kk * m + j];
    qh[s] = uhi[(size_t)kk * m + j];
  }
}

// closed overlap of a record (2D floats) with query bounds, all dimensions
template <int D>
__device__ __forceinline__ bool overlaps(const float (&v)[2 * D], const float (&ql)[D],
                                         const float (&qh)[D]) {
  bool ok = true;
#pragma unroll
  for (int s = 0; s < D; ++s) ok = ok && (v[2 * s] <= qh[s]) && (ql[s] <= v[2 * s + 1]);
  return ok;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
  return uniform_f32(v);
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return uniform_f32(v);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, uint32_t lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)lane);
  return ((uint64_t)hi << 32) | lo;
}

// Which updates a traversal processes: group g (probe dimension g) holds
// gcount[g] updates at perm[gstart[g] ...].
struct UpdSet {
  const uint32_t* perm;
  const uint32_t* gstart;
  const uint32_t* gcount;
  uint32_t total;     // upper bound of sum(gcount), for the launch size
  uint32_t qpt = 64;  // updates per wavefront in the tile traversal (64 or 1)
  // bucket-aligned tiles (optional): bucket b holds perm[boff[b] ..
  // boff[b+1]) (the last ends at `total`), tiles of 64 updates never cross a
  // bucket, tile t belongs to bucket tmap[t], the buckets' first tiles are
  // tprefix[b] and there are tprefix[nbuckets] tiles
  const uint32_t* boff = nullptr;
  const uint32_t* tprefix = nullptr;
  const uint32_t* tmap = nullptr;
  // optional: per update j, pb[2j] <= the first and pb[2j+1] >= the last
  // position of its candidate range in its probe tree (bounds from the
  // probe's quantile searches); tiles then skip their own searches
  const uint32_t* pb = nullptr;
  // optional tile list (replaces the 64-update tiles of tprefix / tmap):
  // tile t holds perm[tstart[t] .. tstart[t+1]) (at most 64 updates, one
  // bucket), belongs to bucket tbuck[t], and there are *ntiles tiles
  const uint32_t* tstart = nullptr;
  const uint32_t* tbuck = nullptr;
  const uint64_t* ntiles = nullptr;
};

// Where a traversal writes.  COUNT (fill == false): cnt[j] = hits of j.
// FILL: hit r of update j goes to out[base[j] + r] if that is below the
// segment end: base[j+1] (final offsets, cap == nullptr) or
// min(base[j] + cap[j], limit) (slots of the single-pass form); with cnt
// non-null the total number of hits (written or not) is stored in cnt[j].
// COUNT with a stash (skey non-null, tile traversal only): every hit is also
// appended, with its rank among its update's hits, to chunks of kStashChunk
// entries.  Tile t owns chunks kStashStatic*t .. +kStashStatic-1 (no atomic
// for tiles with few hits); further chunks come from the slice
// t % kStashSlices of the counted chunks, at least kStashGrab at a time
// (the tile keeps the surplus for its next hits): slice s spans sslice
// chunks from sfirst + s*sslice and snext[s] is its next free chunk
// (separate counters, so that tiles do not queue on one address).  snext[kStashSlices] becomes
// non-zero once a slice is used up (the stash is then incomplete and the
// counts alone are valid).  sused[c] = entries written in chunk c; every
// tile writes it for each of its static chunks.
constexpr uint32_t kStashChunk = 64;
constexpr uint32_t kStashStatic = 2;
constexpr uint32_t kStashSlices = 256;
constexpr uint32_t kStashGrab = 4;  // at least this many counted chunks per request
// at most 2^28 stashed hits (4 GiB of stash); larger results overflow it and
// take the fill traversal
constexpr uint64_t kStashMaxEntries = 1ull << 28;
// a caller's capacity above this many hits per update means dense results,
// for which writing and moving every hit costs more than traversing again
// (measured: 2 hits per update gain, 18 lose); no stash then
constexpr uint64_t kStashMaxPerUpdate = 8;

struct SegOut {
  const uint64_t* base;
  const uint32_t* cap;
  uint64_t limit;
  uint32_t* cnt;
  uint64_t* out;
  // FILL, optional: the subscription id of each hit (4 bytes) at the same
  // place in this array instead of the key in out (the segment sort then
  // forms the keys as it writes them)
  uint32_t* ids = nullptr;
  uint64_t* skey = nullptr;
  uint32_t* srank = nullptr;
  uint32_t* sused = nullptr;
  uint32_t* snext = nullptr;
  uint32_t* sowner = nullptr;  // optional: tile of every counted chunk a tile takes
  uint32_t sfirst = 0;
  uint32_t sslice = 0;
};

__device__ __forceinline__ bool upd_index(const UpdSet& U, uint32_t t, uint32_t d,
                                          uint32_t* idx, uint32_t* grp = nullptr) {
  uint32_t acc = 0;
  for (uint32_t g = 0; g < d; ++g) {
    const uint32_t c = U.gcount[g];
    if (t < acc + c) {
      *idx = U.gstart[g] + (t - acc);
      if (grp) *grp = g;
      return true;
    }
    acc += c;
  }
  return false;
}

__device__ __forceinline__ void seg_bounds(const SegOut& O, uint32_t j, uint64_t* b,
                                           uint64_t* e) {
  *b = O.base[j];
  if (O.cap) {
    const uint64_t e0 = *b + O.cap[j];
    *e = e0 < O.limit ? e0 : (O.limit > *b ? O.limit : *b);
  } else {
    *e = O.base[j + 1];
  }
}

// --------------------------------------------------------------------------
// 3/5b. one wavefront per tile of 64 updates (same probe dimension k, ordered
// by bucket).
//
// The tile's candidates in tree k are confined to positions
// [Pbeg, Pend] = [min plo, max phi] of its updates.  The wave walks that
// range block by block (64 positions; the tree's maxupper of position 64c and
// of the height-5 subtree at 64c+32, i.e. Algorithm 4's pruning test cut at
// height 5): 64 lanes read 64 block maxima at once and a ballot keeps the
// blocks whose maxupper reaches the tile's smallest q.lower.  A kept block is
// read one position per lane; positions meeting the tile's enclosing box in
// every dimension are compacted into an LDS ring with a ballot and a prefix
// popcount.  Each time 64 candidates are pending, lane l takes candidate l
// and the wave tests the tile's updates one after the other against the 64
// candidates (Algorithm 1, closed, every dimension): the ballot of the test
// is the update's hits among them, and a prefix popcount places the hits
// contiguously in the update's own segment.
// --------------------------------------------------------------------------
constexpr int kTileWaves = 4;
constexpr int kRing = 128;

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, kWave));
  return uniform_u32(v);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, kWave));
  return uniform_u32(v);
}

// One tile of the traversal: updates perm[qbeg .. qbeg + nq) (global indices;
// qoff is subtracted to index the instance's coordinates), probe dimension k
// of tree set T.  LDS per wavefront: s_cand [2D][kRing] floats, s_cid
// [kRing], s_q [64][RV] float4.
// XP (count pass only, d >= 2, one instance): the flush is transposed.  The
// tile's updates are sorted once by their lower bound in record slot 1 (the
// first dimension after the probe dimension) into LDS (s_lo1, s_q, s_xj);
// each candidate lane binary-searches the window of updates whose slot-1
// extent can meet its own (lower bound in [c.lo1 - longest update, c.hi1],
// bounds rounded outwards, so the window is a superset) and tests only those
// exactly, in every dimension.  A cell of the tile spans a far wider range
// in the other dimensions than one update, so a window holds a few updates
// where the untransposed flush tests all 64.  Hits are counted per update
// in LDS (s_xcnt); the atomic's result is the hit's rank for the stash.
constexpr uint32_t kXpWindow = 8;  // widest window the transposed flush takes

struct XpLds {
  float* lo1;     // [64] sorted slot-1 lower bounds (+inf past nq)
  uint32_t* cnt;  // [64] hits per sorted update
  uint32_t* j;    // [64] update index of each sorted update
};

template <int D, bool FILL, bool STASH = false, bool XP = false>
__device__ __forceinline__ void tile_body(const TreeDev& T, const float* __restrict__ ulo,
                                          const float* __restrict__ uhi, uint32_t m,
                                          const uint32_t* __restrict__ perm, uint32_t qoff,
                                          uint32_t k, uint32_t qbeg, uint32_t nq, const SegOut& O,
                                          float* __restrict__ s_cand, uint32_t* __restrict__ s_cid,
                                          float4* __restrict__ s_q, uint32_t lane,
                                          uint32_t tile_id = 0,
                                          const uint32_t* __restrict__ pb = nullptr,
                                          XpLds xl = XpLds{}) {
  constexpr int R = 2 * D;
  constexpr int RV = (R + 3) / 4;
  static_assert(!XP || (!FILL && D >= 2), "the transposed flush counts, for d >= 2");
  const bool qv = lane < nq;
  const uint32_t gj = qv ? perm[qbeg + lane] : 0u;  // global update index
  const uint32_t j = gj - qoff;                      // index within the instance
  float ql[D], qh[D];
  if (qv) {
    load_query<D>(ulo, uhi, m, j, k, ql, qh);
  } else {
#pragma unroll
    for (int s = 0; s < D; ++s) {
      ql[s] = INFINITY;
      qh[s] = -INFINITY;
    }
  }
  float tmax1 = 0.f;  // XP: longest slot-1 extent of the tile, rounded up
  uint32_t jx = j;    // the update this lane stands for (XP: in sorted order)
  if constexpr (XP) {
    // bitonic sort of the lanes' (slot-1 lower bound, lane) pairs; lanes
    // past nq sort last
    float key = qv ? ql[1] : INFINITY;
    uint32_t src = lane;
#pragma unroll
    for (uint32_t kk = 2; kk <= (uint32_t)kWave; kk <<= 1) {
#pragma unroll
      for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
        const float ok = __shfl_xor(key, (int)jj, kWave);
        const uint32_t os = (uint32_t)__shfl_xor((int)src, (int)jj, kWave);
        const bool up = (lane & kk) == 0, lower = (lane & jj) == 0;
        const bool other_less = ok < key || (ok == key && os < src);
        if (lower == up ? other_less : !other_less) {
          key = ok;
          src = os;
        }
      }
    }
    // this lane now holds the rank-`lane` update: take its bounds
    float sl[D], sh[D];
#pragma unroll
    for (int s = 0; s < D; ++s) {
      sl[s] = __shfl(ql[s], (int)src, kWave);
      sh[s] = __shfl(qh[s], (int)src, kWave);
    }
    const uint32_t sj = (uint32_t)__shfl((int)j, (int)src, kWave);
#pragma unroll
    for (int s = 0; s < D; ++s) {
      ql[s] = sl[s];
      qh[s] = sh[s];
    }
    xl.lo1[lane] = qv ? sl[1] : INFINITY;
    xl.cnt[lane] = 0;
    xl.j[lane] = sj;
    jx = sj;
    tmax1 = nextafterf(wave_max(qv ? sh[1] - sl[1] : 0.f), INFINITY);
  }
  {
    float qr[4 * RV];
#pragma unroll
    for (int s = 0; s < D; ++s) {
      qr[2 * s] = ql[s];
      qr[2 * s + 1] = qh[s];
    }
#pragma unroll
    for (int r = R; r < 4 * RV; ++r) qr[r] = 0.f;
#pragma unroll
    for (int vv = 0; vv < RV; ++vv)
      s_q[lane * RV + vv] = make_float4(qr[4 * vv], qr[4 * vv + 1], qr[4 * vv + 2], qr[4 * vv + 3]);
  }
  float elo[D], ehi[D];
#pragma unroll
  for (int s = 0; s < D; ++s) {
    elo[s] = wave_min(ql[s]);
    ehi[s] = wave_max(qh[s]);
  }
  // candidate positions of the tile in tree k: lower bound in
  // [t, Ehi] with t <= Elo - maxlen (see the probe kernels).  With per-update
  // bounds from the probe (a superset of each update's range; every
  // position scanned is still tested exactly), the tile's range is their
  // union; otherwise two-level searches over the sorted lower bounds.
  uint32_t Pbeg, Pend;
  if (pb) {
    uint32_t b0 = 0xffffffffu, e0 = 0u;
    if (qv) {
      const uint2 be = reinterpret_cast<const uint2*>(pb)[j];
      b0 = be.x;
      e0 = be.y;
    }
    Pbeg = wave_min_u32(b0);
    Pend = wave_max_u32(e0);
  } else {
    const uint32_t* keys[2] = {T.skey_lo[k], T.skey_lo[k]};
    const uint32_t* idx[2] = {T.sidx_lo[k], T.sidx_lo[k]};
    const uint32_t x[2] = {f2key(ehi[0]), f2key(nextafterf(elo[0] - T.maxlen[k], -INFINITY))};
    const bool up[2] = {true, false};
    uint32_t res[2];
    count_2l<2>(keys, idx, x, up, T.n, T.ns, res);
    Pend = uniform_u32(res[0]);
    Pbeg = uniform_u32(res[1] + 1u);
  }
  uint32_t mycnt = 0;
  uint64_t mybase = 0, myend = 0;  // myend: segment end (write guard)
  if (FILL && qv) seg_bounds(O, gj, &mybase, &myend);
  const uint64_t mystart = mybase;
  uint64_t* __restrict__ out = O.out;
  uint32_t* __restrict__ oids = O.ids;
  const uint64_t jhi = (uint64_t)jx << 32;
  const uint32_t nq4 = (nq + 3u) & ~3u;
  wave_sync();

  const float* __restrict__ rec = T.rec[k];
  const float* __restrict__ bmx = T.bmax[k];
  const uint32_t* __restrict__ ids = T.id[k];
  uint32_t head = 0, tail = 0;
  // stash chunk of the wave (uniform): id, entries used, last static chunk,
  // still stashing
  uint32_t sch = tile_id * kStashStatic, sfill = 0;
  uint32_t slast = sch + kStashStatic - 1;  // last chunk the tile holds
  bool sok = STASH;
  uint64_t myhm = 0;  // this lane's update: hits among the flushed candidates

  // stash: room for `tot` more entries from this wave, in the current chunk
  // and (if needed) nnew more chunks starting at `first` (static ones of the
  // tile, else counted ones from the slices); false once the stash is full
  auto stash_room = [&](uint32_t tot, uint32_t* room_out, uint32_t* first_out,
                        uint32_t* nnew_out) {
    const uint32_t room = kStashChunk - sfill;
    uint32_t first = 0, nnew = 0;
    if (room < tot) {
      nnew = (tot - room + kStashChunk - 1) / kStashChunk;
      if (sch + nnew <= slast) {
        first = sch + 1;
      } else {
        // the tile's slice first, then the following ones; the part of a
        // slice too short for the request is marked empty
        const uint32_t take = max(nnew, kStashGrab);
        if (sch < slast && lane < slast - sch) O.sused[sch + 1 + lane] = 0;
        bool got = false;
        for (uint32_t a = 0, sl = tile_id % kStashSlices; a < kStashSlices && !got;
             ++a, sl = (sl + 1) % kStashSlices) {
          const uint32_t send = O.sfirst + (sl + 1) * O.sslice;
          uint32_t f = 0;
          if (lane == 0) {
            // a slice already used up is passed over without an atomic
            f = __hip_atomic_load(O.snext + sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (f < send) f = atomicAdd(O.snext + sl, take);
          }
          first = uniform_u32(f);
          if (first < send && take <= send - first) {
            got = true;
          } else if (first < send && lane < send - first) {
            O.sused[first + lane] = 0;
          }
        }
        if (!got) {
          sok = false;
          if (lane == 0) atomicOr(O.snext + kStashSlices, 1u);
        } else {
          if (O.sowner && lane < take) O.sowner[first + lane] = tile_id;
          slast = first + take - 1;
        }
      }
    }
    *room_out = room;
    *first_out = first;
    *nnew_out = nnew;
    return sok;
  };
  // the stash has taken `tot` entries (room, first, nnew as stash_room gave)
  auto stash_advance = [&](uint32_t tot, uint32_t room, uint32_t first, uint32_t nnew) {
    if (nnew) {
      if (lane == 0) O.sused[sch] = kStashChunk;
      if (lane + 1 < nnew) O.sused[first + lane] = kStashChunk;
      sch = first + nnew - 1;
      sfill = tot - room - (nnew - 1) * kStashChunk;
    } else {
      sfill += tot;
    }
  };

  auto flush_classic = [&](uint32_t c) {
    wave_sync();
    const uint64_t cvm = (c >= (uint32_t)kWave) ? ~0ull : ((1ull << c) - 1ull);
    const uint32_t slot = (head + lane) & (kRing - 1);
    float v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s_cand[r * kRing + slot];
    const uint32_t sid = s_cid[slot];
    for (uint32_t qi = 0; qi < nq4; qi += 4) {
      uint64_t hm[4];
      bool hit[4];  // this lane's bit of hm (the fill stores under it)
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) {
        float q[4 * RV];
#pragma unroll
        for (int vv = 0; vv < RV; ++vv) {
          const float4 t4 = s_q[(qi + u) * RV + vv];
          q[4 * vv] = t4.x;
          q[4 * vv + 1] = t4.y;
          q[4 * vv + 2] = t4.z;
          q[4 * vv + 3] = t4.w;
        }
        // one compare per lane mask, combined with scalar ANDs
        uint64_t h = cvm;
        bool hl = lane < c;
#pragma unroll
        for (int s = 0; s < D; ++s) {
          const bool c1 = v[2 * s] <= q[2 * s + 1], c2 = q[2 * s] <= v[2 * s + 1];
          h &= ballot(c1);
          h &= ballot(c2);
          hl = hl && c1 && c2;
        }
        hm[u] = h;
        hit[u] = hl;
      }
      if ((hm[0] | hm[1] | hm[2] | hm[3]) != 0) {
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
          if (hm[u] == 0) continue;
          const uint32_t qq = qi + u;
          const uint32_t pc = (uint32_t)__popcll(hm[u]);
          if (FILL) {
            const uint64_t b = readlane_u64(mybase, qq);
            const uint64_t e = readlane_u64(myend, qq);
            const uint64_t jq = readlane_u64(jhi, qq);
            const uint64_t dst = b + mask_rank(hm[u]);
            if (hit[u] && dst < e) {
              if (oids) oids[dst] = sid;
              else out[dst] = jq | sid;
            }
            if (lane == qq) mybase += pc;
          } else if constexpr (STASH || XP) {
            if (lane == qq) myhm = hm[u];
          } else {
            if (lane == qq) mycnt += pc;
          }
        }
      }
    }
    if constexpr (STASH) {
      // each lane stashes its own update's hits among these candidates: a
      // wave prefix of the hit counts places them, one chunk request (if
      // any) covers the whole flush (most flushes have no hit at all)
      if (ballot(myhm != 0) != 0) {
        const uint32_t pcl = (uint32_t)__popcll(myhm);
        uint32_t incl = pcl;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const uint32_t t = (uint32_t)__shfl_up((int)incl, o, kWave);
          if (lane >= (uint32_t)o) incl += t;
        }
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
        if (tot > 0 && sok) {
          const uint32_t room = kStashChunk - sfill;
          uint32_t first = 0, nnew = 0;
          if (room < tot) {
            // hits beyond the current chunk go to consecutive new ones: the
            // tile's next static chunks, else counted ones (the static
            // chunks left over are then marked empty)
            nnew = (tot - room + kStashChunk - 1) / kStashChunk;
            if (sch + nnew <= slast) {
              first = sch + 1;
            } else {
              // the tile's slice first, then the following ones; the part
              // of a slice too short for the request is marked empty
              const uint32_t take = max(nnew, kStashGrab);
              if (sch < slast && lane < slast - sch) O.sused[sch + 1 + lane] = 0;
              bool got = false;
              for (uint32_t a = 0, sl = tile_id % kStashSlices; a < kStashSlices && !got;
                   ++a, sl = (sl + 1) % kStashSlices) {
                const uint32_t send = O.sfirst + (sl + 1) * O.sslice;
                uint32_t f = 0;
                if (lane == 0) {
                  // a slice already used up is passed over without an atomic
                  f = __hip_atomic_load(O.snext + sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                  if (f < send) f = atomicAdd(O.snext + sl, take);
                }
                first = uniform_u32(f);
                if (first < send && take <= send - first) {
                  got = true;
                } else if (first < send && lane < send - first) {
                  O.sused[first + lane] = 0;
                }
              }
              if (!got) {
                sok = false;
                if (lane == 0) atomicOr(O.snext + kStashSlices, 1u);
              } else {
                if (O.sowner && lane < take) O.sowner[first + lane] = tile_id;
                slast = first + take - 1;
              }
            }
          }
          if (sok) {
            uint64_t hv = myhm;
            uint32_t v = incl - pcl, r = XP ? (lane < nq ? xl.cnt[lane] : 0u) : mycnt;
            while (hv) {
              const uint32_t ci = (uint32_t)__builtin_ctzll(hv);
              hv &= hv - 1;
              const uint64_t e = v < room ? (uint64_t)sch * kStashChunk + sfill + v
                                          : (uint64_t)first * kStashChunk + (v - room);
              O.skey[e] = jhi | s_cid[(head + ci) & (kRing - 1)];
              O.srank[e] = r;
              ++v;
              ++r;
            }
            if (nnew) {
              if (lane == 0) O.sused[sch] = kStashChunk;
              if (lane + 1 < nnew) O.sused[first + lane] = kStashChunk;
              sch = first + nnew - 1;
              sfill = tot - room - (nnew - 1) * kStashChunk;
            } else {
              sfill += tot;
            }
          }
        }
        if constexpr (XP) {
          if (lane < nq) xl.cnt[lane] += pcl;
        } else {
          mycnt += pcl;
        }
        myhm = 0;
      }
    } else if constexpr (XP) {
      if (lane < nq) xl.cnt[lane] += (uint32_t)__popcll(myhm);
      myhm = 0;
    }
    head += c;
    wave_sync();
  };
  auto flush_xp = [&](uint32_t c) {
    wave_sync();
    const bool in = lane < c;
    const uint32_t slot = (head + lane) & (kRing - 1);
    float v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s_cand[r * kRing + slot];
    const uint32_t sid = s_cid[slot];
    // window [a, b) of the sorted updates that may meet the candidate in
    // slot 1: lower bound >= c.lo1 - tmax1 (rounded down) and <= c.hi1
    const float klo = nextafterf(v[2] - tmax1, -INFINITY), khi = v[3];
    uint32_t a = 0, b = 0;
#pragma unroll
    for (uint32_t step = kWave; step > 0; step >>= 1) {
      if (a + step <= (uint32_t)kWave && xl.lo1[a + step - 1] < klo) a += step;
      if (b + step <= (uint32_t)kWave && xl.lo1[b + step - 1] <= khi) b += step;
    }
    if (!in) b = a;
    // dense cells (wide windows): the untransposed loop over all updates is
    // cheaper; it keeps its counts and ranks in the same LDS counters
    if (wave_max_u32(b - a) > kXpWindow) {
      flush_classic(c);
      return;
    }
    auto meets = [&](uint32_t u) {
      float q[4 * RV];
#pragma unroll
      for (int vv = 0; vv < RV; ++vv) {
        const float4 t4 = s_q[u * RV + vv];
        q[4 * vv] = t4.x;
        q[4 * vv + 1] = t4.y;
        q[4 * vv + 2] = t4.z;
        q[4 * vv + 3] = t4.w;
      }
      bool ok = true;
#pragma unroll
      for (int s2 = 0; s2 < D; ++s2)
        ok = ok && (v[2 * s2] <= q[2 * s2 + 1]) && (q[2 * s2] <= v[2 * s2 + 1]);
      return ok;
    };
    if constexpr (!STASH) {
      for (uint32_t u = a; u < b; ++u)
        if (meets(u)) atomicAdd(&xl.cnt[u], 1u);
    } else {
      uint32_t nh = 0;
      for (uint32_t u = a; u < b; ++u) nh += meets(u) ? 1u : 0u;
      if (ballot(nh != 0) != 0) {
        uint32_t incl = nh;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const uint32_t t = (uint32_t)__shfl_up((int)incl, o, kWave);
          if (lane >= (uint32_t)o) incl += t;
        }
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
        uint32_t room = 0, first = 0, nnew = 0;
        const bool keep = sok && stash_room(tot, &room, &first, &nnew);
        uint32_t vpos = incl - nh;
        for (uint32_t u = a; u < b; ++u) {
          if (!meets(u)) continue;
          const uint32_t r = atomicAdd(&xl.cnt[u], 1u);
          if (keep) {
            const uint64_t e = vpos < room ? (uint64_t)sch * kStashChunk + sfill + vpos
                                           : (uint64_t)first * kStashChunk + (vpos - room);
            O.skey[e] = ((uint64_t)xl.j[u] << 32) | sid;
            O.srank[e] = r;
          }
          ++vpos;
        }
        if (keep) stash_advance(tot, room, first, nnew);
      }
    }
    head += c;
    wave_sync();
  };

  auto flush = [&](uint32_t c) {
    if constexpr (XP) flush_xp(c);
    else flush_classic(c);
  };

  // one block of 64 candidate positions: test against the tile's box in
  // every dimension, compact the survivors into the ring
  auto stage = [&](const float (&v)[R], uint32_t id, bool inb) {
    bool cnd = inb;
#pragma unroll
    for (int s = 0; s < D; ++s) cnd = cnd & (v[2 * s] <= ehi[s]) & (elo[s] <= v[2 * s + 1]);
    const uint64_t cm = ballot(cnd);
    if (cnd) {
      const uint32_t slot = (tail + mask_rank(cm)) & (kRing - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) s_cand[r * kRing + slot] = v[r];
      s_cid[slot] = id;
    }
    tail += (uint32_t)__popcll(cm);
    if (tail - head >= (uint32_t)kWave) flush(kWave);
  };

  if (Pbeg <= Pend) {
    const uint32_t c0 = Pbeg >> kBlockLog, c1 = Pend >> kBlockLog;
    for (uint32_t cb = c0; cb <= c1; cb += kWave) {
      const uint32_t c = cb + lane;
      const bool keep = (c <= c1) && (bmx[c] >= elo[0]);
      uint64_t bm = ballot(keep);
      while (bm != 0) {
        // two kept blocks at a time: both loads are in flight together
        const uint32_t b0 = (uint32_t)__builtin_ctzll(bm);
        bm &= bm - 1;
        const bool two = bm != 0;
        const uint32_t b1 = two ? (uint32_t)__builtin_ctzll(bm) : b0;
        if (two) bm &= bm - 1;
        const uint32_t blkA = cb + b0, blkB = cb + b1;
        const uint32_t pA = max(blkA << kBlockLog, Pbeg) + lane;
        const uint32_t pB = max(blkB << kBlockLog, Pbeg) + lane;
        const bool inA = pA <= min((blkA << kBlockLog) + (1u << kBlockLog) - 1u, Pend);
        const bool inB = two && pB <= min((blkB << kBlockLog) + (1u << kBlockLog) - 1u, Pend);
        float vA[R], vB[R];
        uint32_t idA = 0, idB = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) vA[r] = vB[r] = 0.f;
        if (inA) {
          load_rec<D>(rec + (size_t)pA * R, vA);
          idA = ids[pA];
        }
        if (inB) {
          load_rec<D>(rec + (size_t)pB * R, vB);
          idB = ids[pB];
        }
        stage(vA, idA, inA);
        stage(vB, idB, inB);
      }
    }
    if (tail != head) flush(tail - head);
  }
  if (STASH && sok) {
    if (lane == 0) O.sused[sch] = sfill;
    if (sch < slast && lane < slast - sch) O.sused[sch + 1 + lane] = 0;
  }
  if constexpr (XP) {
    wave_sync();
    if (qv) O.cnt[xl.j[lane] + qoff] = xl.cnt[lane];
  } else if (qv) {
    if (!FILL) O.cnt[gj] = mycnt;
    else if (O.cnt) O.cnt[gj] = (uint32_t)(mybase - mystart);
  }
}

// Quantiles held in LDS are padded by one word after every 64: the lanes of
// a binary search read indices a power of two apart, which without padding
// fall into one LDS bank at the middle levels of the search.
constexpr uint32_t kQuantPad = kQuant + kQuant / 64;
__device__ __forceinline__ uint32_t qslot(uint32_t i) { return i + (i >> 6); }

// number of quantiles <= x (upper) or < x, LDS binary lifting over the
// padded copy
__device__ __forceinline__ uint32_t quant_count(const uint32_t* __restrict__ q, uint32_t x,
                                                bool upper) {
  uint32_t pos = 0;
#pragma unroll
  for (uint32_t step = kQuant; step > 0; step >>= 1) {
    const uint32_t c = pos + step;
    if (c <= kQuant) {
      const uint32_t v = q[qslot(c - 1)];
      if (upper ? (v <= x) : (v < x)) pos = c;
    }
  }
  return pos;
}

}  // namespace ddm
