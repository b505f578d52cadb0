// Interval tree construction on the device (Sec. IV, Interval-Tree-Create).
//
// The paper builds an augmented AVL tree by insertion.  Here the tree over a
// static subscription set is flat and implicit: segments sorted by lower
// bound occupy in-order positions 1..n of a complete binary tree with
// P = 2^H - 1 >= n positions, where position p has height ctz(p), children
// p -/+ 2^(h-1) and subtree span [p - 2^h + 1, p + 2^h - 1].  The order is
// the paper's (lower bound first); equal lower bounds keep subscription id
// order (stable sort) instead of the upper-bound tie-break, which changes
// no query result.  Each position stores maxupper of its subtree, computed
// bottom-up; minlower is the lower bound at the leftmost position of the
// subtree and needs no storage.  Positions beyond n are padding, recognised
// by index only.
#include "ddm_internal.h"
#include "tree_dev.h"

#include <algorithm>
#include <mutex>
#include <new>

struct ddm_tree {
  int device = 0;
  hipStream_t stream = nullptr;
  uint32_t n = 0, d = 0, H = 0, P = 0;
  char* block = nullptr;  // one device allocation for everything below
  float* rec[DDM_MAX_D] = {};
  float* maxhi[DDM_MAX_D] = {};
  uint32_t* id[DDM_MAX_D] = {};
  uint32_t* skey_lo[DDM_MAX_D] = {};
  uint32_t* skey_hi[DDM_MAX_D] = {};
  float* bmax[DDM_MAX_D] = {};
  uint32_t* sidx_lo[DDM_MAX_D] = {};
  uint32_t* sidx_hi[DDM_MAX_D] = {};
  uint32_t* quant[DDM_MAX_D] = {};
  uint32_t ns = 0;              // ceil(n / 64) search samples
  uint32_t C = 0;               // blocks of 64 positions
  float* maxlen = nullptr;      // d floats (device)
  float* fstat = nullptr;       // feature statistics (learned sizing)
  uint32_t* fcum = nullptr;
  uint32_t* sat = nullptr;
  int32_t* flag = nullptr;  // device: nonzero if a coordinate was invalid
  // feature statistics are computed on the first learned match (they are
  // not needed otherwise); `fstats_ready` marks them enqueued on the stream
  // of that match, `fstats_event` lets other streams wait for them
  std::mutex fmu;
  bool fstats_ready = false;
  hipEvent_t fstats_event = nullptr;
};

namespace ddm {

TreeDev tree_dev(const ddm_tree* t) {
  TreeDev T{};
  for (uint32_t k = 0; k < t->d; ++k) {
    T.rec[k] = t->rec[k];
    T.maxhi[k] = t->maxhi[k];
    T.id[k] = t->id[k];
    T.skey_lo[k] = t->skey_lo[k];
    T.skey_hi[k] = t->skey_hi[k];
    T.bmax[k] = t->bmax[k];
    T.sidx_lo[k] = t->sidx_lo[k];
    T.sidx_hi[k] = t->sidx_hi[k];
    T.quant[k] = t->quant[k];
  }
  T.ns = t->ns;
  T.maxlen = t->maxlen;
  T.n = t->n;
  T.d = t->d;
  T.H = t->H;
  return T;
}

FeatDev tree_feat(const ddm_tree* t) { return FeatDev{t->fstat, t->fcum, t->sat, t->n, t->d}; }
const int32_t* tree_flag(const ddm_tree* t) { return t->flag; }
uint32_t tree_n(const ddm_tree* t) { return t->n; }
uint32_t tree_d(const ddm_tree* t) { return t->d; }
int tree_device(const ddm_tree* t) { return t->device; }

// validate, order-preserving keys, identity payload (id arrays shifted by one
// so that the sorted payload lands directly at positions 1..n)
// keys, identity payload and validity of every coordinate; with recin, the
// set is also written as n records (lo_0, hi_0, lo_1, hi_1, ...) so that the
// tree's gather reads one contiguous record per position
__global__ void build_keys_kernel(const float* __restrict__ lo, const float* __restrict__ hi,
                                  uint32_t n, uint32_t d, uint32_t* __restrict__ klo,
                                  uint32_t* __restrict__ khi, uint32_t* __restrict__ id_base,
                                  int32_t* __restrict__ flag, float* __restrict__ recin) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t total = (uint64_t)n * d;
  bool bad = false;
  if (idx < total) {
    const uint32_t k = (uint32_t)(idx / n);
    const uint32_t i = (uint32_t)(idx - (uint64_t)k * n);
    const float a = lo[idx], b = hi[idx];
    bad = !valid_extent(a, b);
    klo[idx] = f2key(a);
    if (khi) khi[idx] = f2key(b);
    id_base[(size_t)k * (n + 1) + 1 + i] = i;
    if (recin) *reinterpret_cast<float2*>(recin + ((size_t)i * d + k) * 2) = make_float2(a, b);
  }
  if (ballot(bad) != 0 && lane_id() == 0) atomicOr(flag, 1);
}

// up to DDM_MAX_D tree jobs passed by value (one build)
struct TreeJobs {
  TreeJob j[DDM_MAX_D];
};

// samples and quantiles: job blockIdx.y, items blockIdx.x * 256 + tid
__global__ void build_index_kernel(TreeJobs J) {
  tree_index_item(J.j[blockIdx.y], blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void tree_init_kernel(int32_t* __restrict__ flag, uint32_t* __restrict__ maxlen_bits,
                                 uint32_t d) {
  if (threadIdx.x == 0) *flag = 0;
  if (threadIdx.x < d) maxlen_bits[threadIdx.x] = 0;
}

// job blockIdx.y, chunk blockIdx.x
__global__ __launch_bounds__(kTreeThreads) void tree_low_kernel(TreeJobs J) {
  tree_low_chunk(J.j[blockIdx.y], blockIdx.x);
}

// the same pass over records already in place (extents moved)
__global__ __launch_bounds__(kTreeThreads) void tree_refit_kernel(TreeJobs J) {
  tree_low_chunk<false>(J.j[blockIdx.y], blockIdx.x);
}

__global__ __launch_bounds__(kTreeThreads) void tree_high_kernel(TreeJobs J, uint32_t S) {
  tree_high_chunk(J.j[blockIdx.y], blockIdx.x, S);
}

static size_t al(size_t b) { return (b + 255) & ~size_t(255); }

// device bytes of a tree over n subscriptions in d dimensions (one block)
size_t tree_bytes_estimate(uint32_t n, uint32_t d) {
  if (n == 0) return 0;
  uint32_t H = 0;
  while (H < 32 && ((1ull << H) - 1) < n) ++H;
  const uint64_t P = (1ull << H) - 1;
  const size_t rec_b = al(sizeof(float) * (size_t)(n + 1) * 2 * d);
  const size_t mx_b = al(sizeof(float) * ((size_t)P + 1));
  const size_t id_b = al(sizeof(uint32_t) * (size_t)(n + 1) * d);
  const size_t key_b = al(sizeof(uint32_t) * (size_t)n * d);
  const size_t bm_b = al(sizeof(float) * std::max<uint64_t>(1, (P + 1) >> kBlockLog));
  const size_t si_b = al(sizeof(uint32_t) * (size_t)((n + 63) / 64) * d);
  const size_t qu_b = al(sizeof(uint32_t) * kQuant * d);
  return rec_b * d + mx_b * d + id_b + 2 * key_b + bm_b * d + 2 * si_b + qu_b + 256 + 256 +
         al(sizeof(float) * 4 * DDM_MAX_D) + al(sizeof(uint32_t) * DDM_MAX_D * 2 * (kFeatBins + 1)) +
         al(sizeof(uint32_t) * kSatWords);
}

static TreeJobs make_jobs(const ddm_tree* t, const float* lo, const float* hi) {
  const bool sort_hi = t->d == 1;
  TreeJobs J{};
  for (uint32_t k = 0; k < t->d; ++k) {
    TreeJob& j = J.j[k];
    j.s_lo = lo;
    j.s_hi = hi;
    j.rec = t->rec[k];
    j.maxhi = t->maxhi[k];
    j.bmax = t->bmax[k];
    j.id = t->id[k];
    j.skey_lo = t->skey_lo[k];
    j.skey_hi = sort_hi ? t->skey_hi[k] : nullptr;
    j.sidx_lo = t->sidx_lo[k];
    j.sidx_hi = sort_hi ? t->sidx_hi[k] : nullptr;
    j.quant = t->quant[k];
    j.maxlen_bits = (uint32_t*)t->maxlen + k;
    j.n = t->n;
    j.d = t->d;
    j.k = k;
    j.P = t->P;
    j.C = t->C;
    j.H = t->H;
    j.ns = t->ns;
  }
  return J;
}

// samples/quantiles of the sorted keys, then maxupper and block maxima; the
// records are gathered from the inputs (gather) or already in place
static ddm_status enqueue_tree_passes(const ddm_tree* t, const TreeJobs& J, bool gather,
                                      hipStream_t s) {
  const uint32_t d = t->d;
  {
    dim3 g((std::max(t->ns, kQuant) + 255) / 256, d);
    build_index_kernel<<<g, 256, 0, s>>>(J);
    DDM_LAUNCHED("build_index_kernel");
  }
  ProfScope ps("tree_build", s);
  dim3 g((t->P + 1 + kChunk - 1) / kChunk, d);
  if (gather)
    tree_low_kernel<<<g, kTreeThreads, 0, s>>>(J);
  else
    tree_refit_kernel<<<g, kTreeThreads, 0, s>>>(J);
  DDM_LAUNCHED("tree_low_kernel");
  for (uint32_t S = kChunkLog; S < t->H; S += kChunkLog) {
    const uint32_t q_end = (t->P >> S) + 1;
    dim3 g2((q_end + kChunk - 1) / kChunk, d);
    tree_high_kernel<<<g2, kTreeThreads, 0, s>>>(J, S);
    DDM_LAUNCHED("tree_high_kernel");
  }
  return DDM_OK;
}

ddm_status enqueue_tree_build(ddm_tree* t, const float* lo, const float* hi, hipStream_t s) {
  const uint32_t n = t->n, d = t->d;
  // scratch: ping-pong key buffers (lo and hi), payload ping-pong, sort tables
  // upper bounds are sorted only for d == 1, where the BITS counts are the
  // final counts; for d > 1 the probe dimension comes from lower bounds only
  const bool sort_hi = d == 1;
  const uint32_t narr = sort_hi ? 2 * d : d;
  // the sort's arrays (buffer 1 of each is filled in once scratch exists)
  SortArr host[2 * DDM_MAX_D];
  for (uint32_t i = 0; i < narr; ++i) host[i] = SortArr{{nullptr, nullptr}, {nullptr, nullptr}, n, 0};
  const size_t sort_bytes = radix_onesweep_scratch_bytes(host, narr, 4);
  Scratch sc(s);
  sc.reserve(sizeof(uint32_t) * (size_t)n * d);  // lo keys tmp
  sc.reserve(sizeof(uint32_t) * (size_t)n * d);  // hi keys tmp
  sc.reserve(sizeof(uint32_t) * (size_t)n * d);  // payload tmp
  sc.reserve(sort_bytes);
  sc.reserve(sizeof(float) * 2 * (size_t)n * d);  // the set as records
  if (!sc.commit()) return DDM_E_NOMEM;
  uint32_t* klo_tmp = sc.take<uint32_t>((size_t)n * d);
  uint32_t* khi_tmp = sc.take<uint32_t>((size_t)n * d);
  uint32_t* val_tmp = sc.take<uint32_t>((size_t)n * d);
  char* sort_scratch = sc.take<char>(sort_bytes);
  float* recin = sc.take<float>(2 * (size_t)n * d);
  if (!sc.fits()) return scratch_overrun("tree build");

  {
    ProfScope ps("build_keys", s);
    const uint64_t total = (uint64_t)n * d;
    build_keys_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(
        lo, hi, n, d, t->skey_lo[0], sort_hi ? t->skey_hi[0] : nullptr, t->id[0], t->flag,
        recin);
    DDM_LAUNCHED("build_keys_kernel");
  }
  uint32_t na = 0;
  for (uint32_t k = 0; k < d; ++k) {
    SortArr& a = host[na++];
    a.k[0] = t->skey_lo[k];
    a.k[1] = klo_tmp + (size_t)k * n;
    a.v[0] = t->id[k] + 1;
    a.v[1] = val_tmp + (size_t)k * n;
    if (!sort_hi) continue;
    SortArr& b = host[na++];
    b.k[0] = t->skey_hi[k];
    b.k[1] = khi_tmp + (size_t)k * n;
  }
  ddm_status st = radix_sort_onesweep(host, narr, 4, sort_scratch, t->flag, s);
  if (st != DDM_OK) return st;
  TreeJobs J = make_jobs(t, lo, hi);
  for (uint32_t k = 0; k < d; ++k) J.j[k].recin = recin;
  return enqueue_tree_passes(t, J, true, s);
}

// ---------------------------------------------------------------------------
// Moving subscriptions of a resident tree (dynamic DDM: extents move between
// matches, Sec. I and Sec. VI).  If the moved lower bounds keep every tree's
// (lower bound, id) order, the records are rewritten in place and maxupper,
// block maxima, samples and quantiles are recomputed over the records
// (refit, no sort); otherwise the subscription set is read back from the
// records, the moves applied, and the tree rebuilt.
// ---------------------------------------------------------------------------
struct TreePtrs {
  float* rec[DDM_MAX_D];
  const uint32_t* id[DDM_MAX_D];
  uint32_t* pos[DDM_MAX_D];  // position of every subscription in tree k
  uint32_t* key[DDM_MAX_D];  // sorted lower keys with the moves applied
  uint32_t n, d;
};

__global__ void upd_pos_kernel(TreePtrs A) {
  const uint32_t k = blockIdx.y;
  const uint32_t p = 1 + blockIdx.x * blockDim.x + threadIdx.x;
  if (p <= A.n) A.pos[k][A.id[k][p]] = p;
}

// ids in range and new extents valid (flag bit 2)
__global__ void upd_check_kernel(const uint32_t* __restrict__ ids, const float* __restrict__ lo,
                                 const float* __restrict__ hi, uint32_t count, uint32_t n,
                                 uint32_t d, int32_t* __restrict__ flag) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  bool bad = ids[c] >= n;
  for (uint32_t k = 0; k < d; ++k)
    bad = bad || !valid_extent(lo[(size_t)k * count + c], hi[(size_t)k * count + c]);
  if (bad) atomicOr(flag, 4);
}

__global__ void upd_keys_kernel(TreePtrs A, const uint32_t* __restrict__ ids,
                                const float* __restrict__ lo, uint32_t count) {
  const uint32_t k = blockIdx.y;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  const uint32_t i = ids[c];
  if (i >= A.n) return;
  A.key[k][A.pos[k][i] - 1] = f2key(lo[(size_t)k * count + c]);
}

// (key, id) strictly increasing along every tree after the moves? (bit 3)
__global__ void upd_order_kernel(TreePtrs A, int32_t* __restrict__ flag) {
  const uint32_t k = blockIdx.y;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i + 1 >= A.n) return;
  const uint32_t a = A.key[k][i], b = A.key[k][i + 1];
  if (a > b || (a == b && A.id[k][i + 1] > A.id[k][i + 2])) atomicOr(flag, 8);
}

// the moved extents into their record of every tree
__global__ void upd_apply_kernel(TreePtrs A, const uint32_t* __restrict__ ids,
                                 const float* __restrict__ lo, const float* __restrict__ hi,
                                 uint32_t count) {
  const uint32_t k = blockIdx.y;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  const uint32_t D = A.d;
  float* r = A.rec[k] + (size_t)A.pos[k][ids[c]] * 2 * D;
  r[0] = lo[(size_t)k * count + c];
  r[1] = hi[(size_t)k * count + c];
  uint32_t slot = 1;
  for (uint32_t kk = 0; kk < D; ++kk) {
    if (kk == k) continue;
    r[2 * slot] = lo[(size_t)kk * count + c];
    r[2 * slot + 1] = hi[(size_t)kk * count + c];
    ++slot;
  }
}

__global__ void upd_zero_maxlen_kernel(uint32_t* __restrict__ maxlen_bits, uint32_t d) {
  if (threadIdx.x < d) maxlen_bits[threadIdx.x] = 0;
}

// d = 1: upper keys of the records, to be sorted again
__global__ void upd_hi_keys_kernel(const float* __restrict__ rec, uint32_t n,
                                   uint32_t* __restrict__ khi) {
  const uint32_t p = 1 + blockIdx.x * blockDim.x + threadIdx.x;
  if (p <= n) khi[p - 1] = f2key(rec[(size_t)p * 2 + 1]);
}

// the subscription set back from tree 0's records (slot s holds dimension s)
__global__ void upd_gather_kernel(const float* __restrict__ rec, const uint32_t* __restrict__ id,
                                  uint32_t n, uint32_t d, float* __restrict__ lo,
                                  float* __restrict__ hi) {
  const uint32_t p = 1 + blockIdx.x * blockDim.x + threadIdx.x;
  if (p > n) return;
  const uint32_t i = id[p];
  const float* r = rec + (size_t)p * 2 * d;
  for (uint32_t k = 0; k < d; ++k) {
    lo[(size_t)k * n + i] = r[2 * k];
    hi[(size_t)k * n + i] = r[2 * k + 1];
  }
}

__global__ void upd_scatter_kernel(const uint32_t* __restrict__ ids,
                                   const float* __restrict__ nlo, const float* __restrict__ nhi,
                                   uint32_t count, uint32_t n, uint32_t d,
                                   float* __restrict__ lo, float* __restrict__ hi) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  const uint32_t i = ids[c];
  for (uint32_t k = 0; k < d; ++k) {
    lo[(size_t)k * n + i] = nlo[(size_t)k * count + c];
    hi[(size_t)k * n + i] = nhi[(size_t)k * count + c];
  }
}

static ddm_status tree_update(ddm_tree* t, const uint32_t* ids, const float* nlo,
                              const float* nhi, uint32_t count, hipStream_t s, int* rebuilt) {
  const uint32_t n = t->n, d = t->d;
  Scratch sc(s);
  sc.reserve(sizeof(uint32_t) * (size_t)n * d);  // positions
  sc.reserve(sizeof(uint32_t) * (size_t)n * d);  // keys with the moves
  sc.reserve(sizeof(int32_t));                   // flag
  if (!sc.commit()) return DDM_E_NOMEM;
  uint32_t* pos = sc.take<uint32_t>((size_t)n * d);
  uint32_t* keys = sc.take<uint32_t>((size_t)n * d);
  int32_t* flag = sc.take<int32_t>(1);
  if (!sc.fits()) return scratch_overrun("tree update");
  TreePtrs A{};
  for (uint32_t k = 0; k < d; ++k) {
    A.rec[k] = t->rec[k];
    A.id[k] = t->id[k];
    A.pos[k] = pos + (size_t)k * n;
    A.key[k] = keys + (size_t)k * n;
    DDM_HIP(hipMemcpyAsync(A.key[k], t->skey_lo[k], sizeof(uint32_t) * n,
                           hipMemcpyDeviceToDevice, s));
  }
  A.n = n;
  A.d = d;
  tree_init_kernel<<<1, 64, 0, s>>>(flag, nullptr, 0);
  DDM_LAUNCHED("tree_init_kernel");
  upd_pos_kernel<<<dim3((n + 255) / 256, d), 256, 0, s>>>(A);
  DDM_LAUNCHED("upd_pos_kernel");
  upd_check_kernel<<<(count + 255) / 256, 256, 0, s>>>(ids, nlo, nhi, count, n, d, flag);
  DDM_LAUNCHED("upd_check_kernel");
  upd_keys_kernel<<<dim3((count + 255) / 256, d), 256, 0, s>>>(A, ids, nlo, count);
  DDM_LAUNCHED("upd_keys_kernel");
  upd_order_kernel<<<dim3((n + 255) / 256, d), 256, 0, s>>>(A, flag);
  DDM_LAUNCHED("upd_order_kernel");
  int32_t f = 0;
  DDM_HIP(hipMemcpyAsync(&f, flag, sizeof(f), hipMemcpyDeviceToHost, s));
  DDM_HIP(hipStreamSynchronize(s));
  if (f & 4) {
    set_detail("ddm_tree_update: id out of range, or NaN/inf or lo > hi in the new extents");
    return DDM_E_INVALID_INPUT;
  }
  {
    // learned-sizing statistics describe the old set
    std::lock_guard<std::mutex> lk(t->fmu);
    t->fstats_ready = false;
  }
  if (!(f & 8)) {
    *rebuilt = 0;
    upd_apply_kernel<<<dim3((count + 255) / 256, d), 256, 0, s>>>(A, ids, nlo, nhi, count);
    DDM_LAUNCHED("upd_apply_kernel");
    for (uint32_t k = 0; k < d; ++k)
      DDM_HIP(hipMemcpyAsync(t->skey_lo[k], A.key[k], sizeof(uint32_t) * n,
                             hipMemcpyDeviceToDevice, s));
    upd_zero_maxlen_kernel<<<1, 64, 0, s>>>((uint32_t*)t->maxlen, d);
    DDM_LAUNCHED("upd_zero_maxlen_kernel");
    if (d == 1) {
      // the upper keys stay a sorted multiset for the exact counts
      SortArr h{{nullptr, nullptr}, {nullptr, nullptr}, n, 0};
      const size_t sort_bytes = radix_onesweep_scratch_bytes(&h, 1, 4);
      Scratch ss(s);
      ss.reserve(sizeof(uint32_t) * n);
      ss.reserve(sort_bytes);
      if (!ss.commit()) return DDM_E_NOMEM;
      uint32_t* ktmp = ss.take<uint32_t>(n);
      char* sort_scratch = ss.take<char>(sort_bytes);
      if (!ss.fits()) return scratch_overrun("tree update");
      upd_hi_keys_kernel<<<(n + 255) / 256, 256, 0, s>>>(t->rec[0], n, t->skey_hi[0]);
      DDM_LAUNCHED("upd_hi_keys_kernel");
      h.k[0] = t->skey_hi[0];
      h.k[1] = ktmp;
      ddm_status st = radix_sort_onesweep(&h, 1, 4, sort_scratch, t->flag, s);
      if (st != DDM_OK) return st;
      return enqueue_tree_passes(t, make_jobs(t, nullptr, nullptr), false, s);
    }
    return enqueue_tree_passes(t, make_jobs(t, nullptr, nullptr), false, s);
  }
  *rebuilt = 1;
  Scratch sr(s);
  sr.reserve(sizeof(float) * (size_t)n * d);
  sr.reserve(sizeof(float) * (size_t)n * d);
  if (!sr.commit()) return DDM_E_NOMEM;
  float* lo = sr.take<float>((size_t)n * d);
  float* hi = sr.take<float>((size_t)n * d);
  if (!sr.fits()) return scratch_overrun("tree update");
  upd_gather_kernel<<<(n + 255) / 256, 256, 0, s>>>(t->rec[0], t->id[0], n, d, lo, hi);
  DDM_LAUNCHED("upd_gather_kernel");
  upd_scatter_kernel<<<(count + 255) / 256, 256, 0, s>>>(ids, nlo, nhi, count, n, d, lo, hi);
  DDM_LAUNCHED("upd_scatter_kernel");
  tree_init_kernel<<<1, 64, 0, s>>>(t->flag, (uint32_t*)t->maxlen, d);
  DDM_LAUNCHED("tree_init_kernel");
  return enqueue_tree_build(t, lo, hi, s);
}

// Enqueue the feature statistics on stream s the first time a learned match
// uses the tree; later users on other streams wait for the recorded event.
ddm_status tree_ensure_features(const ddm_tree* tc, hipStream_t s) {
  ddm_tree* t = const_cast<ddm_tree*>(tc);
  std::lock_guard<std::mutex> lk(t->fmu);
  if (t->fstats_ready) {
    DDM_HIP(hipStreamWaitEvent(s, t->fstats_event, 0));
    return DDM_OK;
  }
  ProfScope ps("feature_stats", s);
  FeatArgs F{};
  for (uint32_t k = 0; k < t->d; ++k) {
    F.rec[k] = t->rec[k];
    F.maxhi[k] = t->maxhi[k];
    F.skey_lo[k] = t->skey_lo[k];
    F.sidx_lo[k] = t->sidx_lo[k];
  }
  F.n = t->n;
  F.d = t->d;
  F.ns = t->ns;
  F.root = 1u << (t->H - 1);
  F.fstat = t->fstat;
  F.fcum = t->fcum;
  F.sat = t->sat;
  ddm_status st = enqueue_feature_stats(F, s);
  if (st != DDM_OK) return st;
  if (!t->fstats_event) t->fstats_event = pooled_event();
  if (!t->fstats_event) {
    set_detail("event creation failed");
    return DDM_E_DEVICE;
  }
  DDM_HIP(hipEventRecord(t->fstats_event, s));
  t->fstats_ready = true;
  return DDM_OK;
}

}  // namespace ddm

using namespace ddm;

extern "C" ddm_status ddm_build(const float* sub_lo, const float* sub_hi, uint32_t n, uint32_t d,
                                void* stream, ddm_tree** out_tree) {
  set_detail("");
  if (!out_tree) {
    set_detail("ddm_build: out_tree is NULL");
    return DDM_E_INVALID_ARG;
  }
  *out_tree = nullptr;
  if (d < 1 || d > DDM_MAX_D) {
    set_detail("ddm_build: d must be in [1, DDM_MAX_D]");
    return DDM_E_INVALID_ARG;
  }
  if (n > 0 && (!sub_lo || !sub_hi)) {
    set_detail("ddm_build: NULL coordinate pointer");
    return DDM_E_INVALID_ARG;
  }
  if (n >= 0x40000000u) {
    set_detail("ddm_build: n must be below 2^30");
    return DDM_E_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  ddm_tree* t = new (std::nothrow) ddm_tree();
  if (!t) return DDM_E_NOMEM;
  DDM_HIP(hipGetDevice(&t->device));
  t->stream = s;
  t->n = n;
  t->d = d;
  if (n == 0) {
    *out_tree = t;
    return DDM_OK;
  }
  uint32_t H = 0;
  while (H < 32 && ((1ull << H) - 1) < n) ++H;
  t->H = H;
  t->P = (uint32_t)((1ull << H) - 1);
  const size_t rec_b = al(sizeof(float) * (size_t)(n + 1) * 2 * d);
  const size_t mx_b = al(sizeof(float) * ((size_t)t->P + 1));
  const size_t id_b = al(sizeof(uint32_t) * (size_t)(n + 1) * d);
  const size_t key_b = al(sizeof(uint32_t) * (size_t)n * d);
  t->C = std::max<uint32_t>(1u, (uint32_t)(((uint64_t)t->P + 1) >> kBlockLog));
  const size_t bm_b = al(sizeof(float) * t->C);
  t->ns = (n + 63) / 64;
  const size_t si_b = al(sizeof(uint32_t) * (size_t)t->ns * d);
  const size_t qu_b = al(sizeof(uint32_t) * kQuant * d);
  const size_t total = tree_bytes_estimate(n, d);
  void* blk = dev_alloc(total, s);
  hipError_t e = hipSuccess;
  if (!blk) {
    delete t;
    set_detail("ddm_build: device allocation failed");
    return DDM_E_NOMEM;
  }
  t->block = (char*)blk;
  char* p = t->block;
  for (uint32_t k = 0; k < d; ++k) { t->rec[k] = (float*)p; p += rec_b; }
  for (uint32_t k = 0; k < d; ++k) { t->maxhi[k] = (float*)p; p += mx_b; }
  uint32_t* idb = (uint32_t*)p;
  p += id_b;
  for (uint32_t k = 0; k < d; ++k) t->id[k] = idb + (size_t)k * (n + 1);
  uint32_t* klo = (uint32_t*)p;
  p += key_b;
  uint32_t* khi = (uint32_t*)p;
  p += key_b;
  for (uint32_t k = 0; k < d; ++k) {
    t->skey_lo[k] = klo + (size_t)k * n;
    t->skey_hi[k] = khi + (size_t)k * n;
  }
  for (uint32_t k = 0; k < d; ++k) { t->bmax[k] = (float*)p; p += bm_b; }
  {
    uint32_t* ilo = (uint32_t*)p;
    p += si_b;
    uint32_t* ihi = (uint32_t*)p;
    p += si_b;
    for (uint32_t k = 0; k < d; ++k) {
      t->sidx_lo[k] = ilo + (size_t)k * t->ns;
      t->sidx_hi[k] = ihi + (size_t)k * t->ns;
    }
    uint32_t* qu = (uint32_t*)p;
    p += qu_b;
    for (uint32_t k = 0; k < d; ++k) t->quant[k] = qu + (size_t)k * kQuant;
  }
  t->maxlen = (float*)p;
  p += 256;
  t->fstat = (float*)p;
  p += al(sizeof(float) * 4 * DDM_MAX_D);
  t->fcum = (uint32_t*)p;
  p += al(sizeof(uint32_t) * DDM_MAX_D * 2 * (kFeatBins + 1));
  t->sat = (uint32_t*)p;
  p += al(sizeof(uint32_t) * kSatWords);
  t->flag = (int32_t*)p;
  tree_init_kernel<<<1, 64, 0, s>>>(t->flag, (uint32_t*)t->maxlen, d);
  e = hipGetLastError();
  if (e != hipSuccess) {
    dev_free(t->block, s);
    delete t;
    return hip_fail(e, "tree_init_kernel", __FILE__, __LINE__);
  }
  ddm_status st = enqueue_tree_build(t, sub_lo, sub_hi, s);
  if (st != DDM_OK) {
    dev_free(t->block, s);
    delete t;
    return st;
  }
  *out_tree = t;
  return DDM_OK;
}

extern "C" ddm_status ddm_tree_update(ddm_tree* t, const uint32_t* ids, const float* new_lo,
                                      const float* new_hi, uint32_t count, void* stream,
                                      int* out_rebuilt) {
  set_detail("");
  if (!t || (count && (!ids || !new_lo || !new_hi))) {
    set_detail("ddm_tree_update: NULL argument");
    return DDM_E_INVALID_ARG;
  }
  if (out_rebuilt) *out_rebuilt = 0;
  if (count == 0) return DDM_OK;
  if (t->n == 0 || count > t->n) {
    set_detail("ddm_tree_update: more moves than subscriptions");
    return DDM_E_INVALID_ARG;
  }
  int cur = -1;
  DDM_HIP(hipGetDevice(&cur));
  if (cur != t->device) {
    set_detail("ddm_tree_update: the current device is not the tree's device");
    return DDM_E_INVALID_ARG;
  }
  int rb = 0;
  ddm_status st = tree_update(t, ids, new_lo, new_hi, count, (hipStream_t)stream, &rb);
  if (out_rebuilt) *out_rebuilt = rb;
  return st;
}

extern "C" void ddm_tree_free(ddm_tree* t) {
  if (!t) return;
  release_event(t->fstats_event);
  if (t->block) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != t->device) (void)hipSetDevice(t->device);
    dev_free(t->block, t->stream);
    if (cur != t->device) (void)hipSetDevice(cur);
  }
  delete t;
}

extern "C" ddm_status ddm_tree_check(const ddm_tree* t) {
  set_detail("");
  if (!t) return DDM_E_INVALID_ARG;
  if (t->n == 0) return DDM_OK;
  int32_t f = 0;
  DDM_HIP(hipStreamSynchronize(t->stream));
  DDM_HIP(hipMemcpy(&f, t->flag, sizeof(f), hipMemcpyDeviceToHost));
  if (f & kFlagSortTimeout) {
    set_detail("tree build: a radix sort look-back wait gave up");
    return DDM_E_DEVICE;
  }
  if (f) {
    set_detail("subscription coordinates: NaN/inf or lo > hi");
    return DDM_E_INVALID_INPUT;
  }
  return DDM_OK;
}

extern "C" ddm_status ddm_tree_prepare_learned(const ddm_tree* t, void* stream) {
  set_detail("");
  if (!t) return DDM_E_INVALID_ARG;
  if (t->d > 3) {
    set_detail("features are defined for d <= 3");
    return DDM_E_INVALID_ARG;
  }
  if (t->n == 0) {
    set_detail("features need a non-empty subscription set");
    return DDM_E_INVALID_ARG;
  }
  return tree_ensure_features(t, (hipStream_t)stream);
}

extern "C" ddm_status ddm_tree_info(const ddm_tree* t, uint32_t* n, uint32_t* d, uint32_t* height) {
  if (!t) return DDM_E_INVALID_ARG;
  if (n) *n = t->n;
  if (d) *d = t->d;
  if (height) *height = t->H;
  return DDM_OK;
}

extern "C" ddm_status ddm_tree_export(const ddm_tree* t, uint32_t k, float* lo, float* hi,
                                      uint32_t* ids, float* maxhi) {
  set_detail("");
  if (!t || k >= t->d) return DDM_E_INVALID_ARG;
  if (t->n == 0) return DDM_OK;
  DDM_HIP(hipStreamSynchronize(t->stream));
  const uint32_t n = t->n, D = t->d;
  if (lo || hi) {
    float* recs = (float*)malloc(sizeof(float) * (size_t)(n + 1) * 2 * D);
    if (!recs) return DDM_E_NOMEM;
    hipError_t e = hipMemcpy(recs, t->rec[k], sizeof(float) * (size_t)(n + 1) * 2 * D,
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      free(recs);
      return hip_fail(e, "hipMemcpy", __FILE__, __LINE__);
    }
    for (uint32_t p = 1; p <= n; ++p) {
      if (lo) lo[p - 1] = recs[(size_t)p * 2 * D];
      if (hi) hi[p - 1] = recs[(size_t)p * 2 * D + 1];
    }
    free(recs);
  }
  if (ids) DDM_HIP(hipMemcpy(ids, t->id[k] + 1, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
  if (maxhi)
    DDM_HIP(hipMemcpy(maxhi, t->maxhi[k] + 1, sizeof(float) * t->P, hipMemcpyDeviceToHost));
  return DDM_OK;
}
