// Sort-Based Matching on the device (Algorithm 3, Sec. III-D), the paper's
// sweep-line comparison system, for measuring Interval Tree Matching
// against on the same GPU.  Results are the same keys, in the same order, as
// ddm_match.
//
// The sequential algorithm sorts all endpoints and sweeps them while keeping
// the sets of active subscriptions and updates; each pair is reported when
// the first of its two upper endpoints is passed.  The loop-carried sets are
// what the paper names as the obstacle to parallelism.  Here the sweep runs
// in dimension 0 and is cut into segments of kSbmSeg consecutive subscription
// lower endpoints (in sweep order); the active subscription set at the start
// of every segment comes from a prefix instead of from the previous segment:
//
//   A(b) = { ranks r < bG : hi_r >= x_b },  x_b = lower endpoint of rank bG
//   |A(b)| = bG - #{hi < x_b}   (hi < x_b implies rank < bG)
//
// so the segment sizes are one binary search each, their offsets a scan, and
// every subscription enters the lists of the segments its span covers.  An
// update u then resumes the sweep at the last segment start not after its
// lower endpoint: the subscriptions active there that are still active at
// lo_u, plus every subscription whose lower endpoint the sweep passes before
// reaching hi_u and whose upper endpoint is not before lo_u.  That is the set
// of subscriptions the sequential sweep pairs with u (at u's upper endpoint,
// or at theirs while u is active), each exactly once.  The other dimensions
// are tested on every reported pair (the combine of Sec. III-A), so no
// per-dimension list is formed.
//
// One lane per update, updates in sweep order so that a wave's lanes resume
// at neighbouring segments.  Count pass, scan, fill pass, per-update sort.
#include "ddm_internal.h"

namespace ddm {

constexpr uint32_t kSbmSeg = 64;  // subscription lower endpoints per segment
constexpr uint32_t kSbmThreads = 256;

// keys of the sweep dimension and validation of every dimension; bit 0 of
// *flag: a subscription is invalid, bit 1: an update is
__global__ void sbm_keys_kernel(const float* __restrict__ slo, const float* __restrict__ shi,
                                uint32_t n, const float* __restrict__ ulo,
                                const float* __restrict__ uhi, uint32_t m, uint32_t d,
                                uint32_t* __restrict__ klo, uint32_t* __restrict__ kid,
                                uint32_t* __restrict__ khi, uint32_t* __restrict__ ukey,
                                uint32_t* __restrict__ uid, int32_t* __restrict__ flag) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  bool bad_s = false, bad_u = false;
  if (t < n) {
    for (uint32_t k = 0; k < d; ++k)
      bad_s = bad_s || !valid_extent(slo[(size_t)k * n + t], shi[(size_t)k * n + t]);
    klo[t] = f2key(slo[t]);
    khi[t] = f2key(shi[t]);
    kid[t] = t;
  }
  if (t < m) {
    for (uint32_t k = 0; k < d; ++k)
      bad_u = bad_u || !valid_extent(ulo[(size_t)k * m + t], uhi[(size_t)k * m + t]);
    ukey[t] = f2key(ulo[t]);
    uid[t] = t;
  }
  const uint64_t bs = ballot(bad_s), bu = ballot(bad_u);
  if (lane_id() == 0 && (bs | bu)) atomicOr(flag, (bs ? 1 : 0) | (bu ? 2 : 0));
}

// subscriptions in sweep order: rank r holds (lo_0, hi_0, lo_1, hi_1, ...)
__global__ void sbm_records_kernel(const float* __restrict__ slo, const float* __restrict__ shi,
                                   uint32_t n, uint32_t d, const uint32_t* __restrict__ sid,
                                   float* __restrict__ rec) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t i = sid[r];
  float* dst = rec + (size_t)r * 2 * d;
  for (uint32_t k = 0; k < d; ++k) {
    dst[2 * k] = slo[(size_t)k * n + i];
    dst[2 * k + 1] = shi[(size_t)k * n + i];
  }
}

__global__ void sbm_init_kernel(uint32_t* __restrict__ acur, uint32_t B,
                                uint32_t* __restrict__ lists_count, int32_t* __restrict__ flag) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < B) acur[t] = 0;
  if (t < 2) lists_count[t] = 0;
  if (t == 0) *flag = 0;
}

// |A(b)| for every segment start b
__global__ void sbm_active_count_kernel(const uint32_t* __restrict__ klo,
                                        const uint32_t* __restrict__ khi, uint32_t n, uint32_t B,
                                        uint32_t* __restrict__ acnt) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const uint32_t r0 = b * kSbmSeg;
  acnt[b] = r0 - lower_bound_u32(khi, n, klo[r0]);
}

// rank r joins A(b) for r < bG and x_b <= hi_r: b in [r/G + 1, (c - 1)/G]
// with c = #{lo <= hi_r} >= r + 1
__global__ void sbm_lists_kernel(const uint32_t* __restrict__ klo, uint32_t n,
                                 const float* __restrict__ rec, uint32_t d, uint32_t B,
                                 const uint64_t* __restrict__ aoff, uint32_t* __restrict__ acur,
                                 uint32_t* __restrict__ alist) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t c = upper_bound_u32(klo, n, f2key(rec[(size_t)r * 2 * d + 1]));
  if (c == 0) return;  // only for lo > hi, rejected before this kernel runs
  const uint32_t b1 = min((c - 1) / kSbmSeg, B - 1);
  for (uint32_t b = r / kSbmSeg + 1; b <= b1; ++b) {
    const uint32_t slot = atomicAdd(&acur[b], 1u);
    if (aoff[b] + slot < aoff[b + 1]) alist[aoff[b] + slot] = r;
  }
}

template <int D>
__device__ __forceinline__ bool sbm_meets(const float* __restrict__ rec, uint32_t r,
                                          const float (&ql)[D], const float (&qh)[D]) {
  const float* p = rec + (size_t)r * 2 * D;
  bool hit = true;
#pragma unroll
  for (int k = 0; k < D; ++k) hit = hit & (p[2 * k] <= qh[k]) & (ql[k] <= p[2 * k + 1]);
  return hit;
}

// the resumed sweep of one update per lane (count pass, then fill pass)
template <int D, bool FILL>
__global__ __launch_bounds__(kSbmThreads) void sbm_match_kernel(
    const float* __restrict__ ulo, const float* __restrict__ uhi, uint32_t m,
    const uint32_t* __restrict__ uorder, const uint32_t* __restrict__ klo, uint32_t n,
    const float* __restrict__ rec, const uint32_t* __restrict__ sid,
    const uint64_t* __restrict__ aoff, const uint32_t* __restrict__ alist,
    uint32_t* __restrict__ cnt, const uint64_t* __restrict__ off, uint64_t* __restrict__ out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  const uint32_t j = uorder[t];
  float ql[D], qh[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    ql[k] = ulo[(size_t)k * m + j];
    qh[k] = uhi[(size_t)k * m + j];
  }
  const uint32_t cl = upper_bound_u32(klo, n, f2key(ql[0]));  // #{lo <= lo_u}
  const uint32_t ch = upper_bound_u32(klo, n, f2key(qh[0]));  // #{lo <= hi_u}
  const uint32_t b = cl ? (cl - 1) / kSbmSeg : 0;
  uint32_t c = 0;
  const uint64_t base = FILL ? off[j] : 0;
  const uint64_t jhi = (uint64_t)j << 32;
  // subscriptions active at the segment start that are still active at lo_u
  for (uint64_t e = aoff[b]; e < aoff[b + 1]; ++e) {
    const uint32_t r = alist[e];
    if (r >= n) continue;  // every slot is written when the inputs are valid
    if (sbm_meets<D>(rec, r, ql, qh)) {
      if (FILL) out[base + c] = jhi | sid[r];
      ++c;
    }
  }
  // lower endpoints passed from the segment start up to hi_u
  for (uint32_t r = b * kSbmSeg; r < ch; ++r) {
    if (sbm_meets<D>(rec, r, ql, qh)) {
      if (FILL) out[base + c] = jhi | sid[r];
      ++c;
    }
  }
  if (!FILL) cnt[j] = c;
}

template <bool FILL>
static void launch_sbm(uint32_t d, const float* ulo, const float* uhi, uint32_t m,
                       const uint32_t* uorder, const uint32_t* klo, uint32_t n, const float* rec,
                       const uint32_t* sid, const uint64_t* aoff, const uint32_t* alist,
                       uint32_t* cnt, const uint64_t* off, uint64_t* out, hipStream_t s) {
  ProfScope ps(FILL ? "sbm_fill" : "sbm_count", s);
  const dim3 g((m + kSbmThreads - 1) / kSbmThreads);
#define DDM_SBM(DD)                                                                          \
  sbm_match_kernel<DD, FILL><<<g, kSbmThreads, 0, s>>>(ulo, uhi, m, uorder, klo, n, rec, sid, \
                                                       aoff, alist, cnt, off, out)
  switch (d) {
    case 1: DDM_SBM(1); break;
    case 2: DDM_SBM(2); break;
    case 3: DDM_SBM(3); break;
    default: DDM_SBM(4); break;
  }
#undef DDM_SBM
}

__global__ void sbm_words_kernel(const uint64_t* __restrict__ a, uint32_t ia,
                                 const int32_t* __restrict__ flag, uint64_t* __restrict__ w) {
  if (threadIdx.x == 0) {
    w[0] = a[ia];
    w[1] = (uint64_t)(uint32_t)*flag;
  }
}

}  // namespace ddm

using namespace ddm;

extern "C" ddm_status ddm_match_sbm(const float* sub_lo, const float* sub_hi, uint32_t n,
                                    const float* upd_lo, const float* upd_hi, uint32_t m,
                                    uint32_t d, uint64_t* out_pairs, uint64_t capacity,
                                    uint64_t* out_count, void* stream) {
  set_detail("");
  if (!out_count) {
    set_detail("ddm_match_sbm: out_count is NULL");
    return DDM_E_INVALID_ARG;
  }
  *out_count = 0;
  if (d < 1 || d > DDM_MAX_D || (n && (!sub_lo || !sub_hi)) || (m && (!upd_lo || !upd_hi)) ||
      m >= 0x80000000u || n >= 0x80000000u) {
    set_detail("ddm_match_sbm: d in [1, DDM_MAX_D], coordinate pointers, n, m < 2^31");
    return DDM_E_INVALID_ARG;
  }
  if (n == 0 || m == 0) return DDM_OK;
  hipStream_t s = (hipStream_t)stream;
  const uint32_t B = (n + kSbmSeg - 1) / kSbmSeg;
  SortArr host[3] = {SortArr{{nullptr, nullptr}, {nullptr, nullptr}, n, 0},
                     SortArr{{nullptr, nullptr}, {nullptr, nullptr}, n, 0},
                     SortArr{{nullptr, nullptr}, {nullptr, nullptr}, m, 0}};
  const size_t sort_bytes = radix_onesweep_scratch_bytes(host, 3, 4);
  Scratch sc(s);
  for (int i = 0; i < 6; ++i) sc.reserve(sizeof(uint32_t) * n);  // lower keys, ids, upper keys
  for (int i = 0; i < 4; ++i) sc.reserve(sizeof(uint32_t) * m);  // update keys, ids
  sc.reserve(sort_bytes);
  sc.reserve(sizeof(float) * 2 * (size_t)d * n);
  sc.reserve(sizeof(uint32_t) * B);  // acnt
  sc.reserve(sizeof(uint32_t) * B);  // acur
  sc.reserve(sizeof(uint64_t) * (B + 1));
  sc.reserve(sizeof(uint64_t) * scan_tmp_words(B));
  sc.reserve(sizeof(uint32_t) * m);
  sc.reserve(sizeof(uint64_t) * (m + 1));
  sc.reserve(sizeof(uint64_t) * scan_tmp_words(m));
  sc.reserve(sizeof(uint32_t) * 2 * (size_t)m);
  sc.reserve(sizeof(uint32_t) * 2);
  sc.reserve(sizeof(int32_t));
  sc.reserve(sizeof(uint64_t) * 2);
  if (!sc.commit()) return DDM_E_NOMEM;
  uint32_t* klo[2] = {sc.take<uint32_t>(n), sc.take<uint32_t>(n)};
  uint32_t* kid[2] = {sc.take<uint32_t>(n), sc.take<uint32_t>(n)};
  uint32_t* khi[2] = {sc.take<uint32_t>(n), sc.take<uint32_t>(n)};
  uint32_t* ukey[2] = {sc.take<uint32_t>(m), sc.take<uint32_t>(m)};
  uint32_t* uid[2] = {sc.take<uint32_t>(m), sc.take<uint32_t>(m)};
  char* sort_scratch = sc.take<char>(sort_bytes);
  float* rec = sc.take<float>(2 * (size_t)d * n);
  uint32_t* acnt = sc.take<uint32_t>(B);
  uint32_t* acur = sc.take<uint32_t>(B);
  uint64_t* aoff = sc.take<uint64_t>(B + 1);
  uint64_t* atmp = sc.take<uint64_t>(scan_tmp_words(B));
  uint32_t* cnt = sc.take<uint32_t>(m);
  uint64_t* off = sc.take<uint64_t>(m + 1);
  uint64_t* stmp = sc.take<uint64_t>(scan_tmp_words(m));
  uint32_t* lists = sc.take<uint32_t>(2 * (size_t)m);
  uint32_t* lists_count = sc.take<uint32_t>(2);
  int32_t* flag = sc.take<int32_t>(1);
  uint64_t* words = sc.take<uint64_t>(2);
  if (!sc.fits()) return scratch_overrun("ddm_match_sbm");

  const uint32_t nm = n > m ? n : m;
  {
    ProfScope ps("sbm_keys", s);
    const uint32_t z = B > 2 ? B : 2;
    sbm_init_kernel<<<(z + 255) / 256, 256, 0, s>>>(acur, B, lists_count, flag);
    DDM_LAUNCHED("sbm_init_kernel");
    sbm_keys_kernel<<<(nm + 255) / 256, 256, 0, s>>>(sub_lo, sub_hi, n, upd_lo, upd_hi, m, d,
                                                     klo[0], kid[0], khi[0], ukey[0], uid[0],
                                                     flag);
    DDM_LAUNCHED("sbm_keys_kernel");
  }
  // the sorted endpoint list: lower and upper endpoints of the subscriptions
  // (ties of the lower keys broken by id: the radix sort is stable) and the
  // updates' lower endpoints, which give the order of the update lanes
  host[0] = SortArr{{klo[0], klo[1]}, {kid[0], kid[1]}, n, 0};
  host[1] = SortArr{{khi[0], khi[1]}, {nullptr, nullptr}, n, 0};
  host[2] = SortArr{{ukey[0], ukey[1]}, {uid[0], uid[1]}, m, 0};
  ddm_status r = radix_sort_onesweep(host, 3, 4, sort_scratch, flag, s);
  if (r != DDM_OK) return r;
  {
    ProfScope ps("sbm_segments", s);
    sbm_records_kernel<<<(n + 255) / 256, 256, 0, s>>>(sub_lo, sub_hi, n, d, kid[0], rec);
    DDM_LAUNCHED("sbm_records_kernel");
    sbm_active_count_kernel<<<(B + 255) / 256, 256, 0, s>>>(klo[0], khi[0], n, B, acnt);
    DDM_LAUNCHED("sbm_active_count_kernel");
  }
  r = scan_u32_u64(acnt, aoff, B, atmp, s);
  if (r != DDM_OK) return r;
  sbm_words_kernel<<<1, 64, 0, s>>>(aoff, B, flag, words);
  DDM_LAUNCHED("sbm_words_kernel");
  uint64_t h[2] = {0, 0};
  DDM_HIP(hipMemcpyAsync(h, words, sizeof(h), hipMemcpyDeviceToHost, s));
  DDM_HIP(hipStreamSynchronize(s));
  if (h[1] & (uint32_t)kFlagSortTimeout) {
    set_detail("ddm_match_sbm: a radix sort look-back wait gave up");
    return DDM_E_DEVICE;
  }
  if (h[1]) {
    set_detail(h[1] & 1 ? "subscription coordinates: NaN/inf or lo > hi"
                        : "update coordinates: NaN/inf or lo > hi");
    return DDM_E_INVALID_INPUT;
  }
  const uint64_t A = h[0];
  Scratch sa(s);
  sa.reserve(sizeof(uint32_t) * (A ? A : 1));
  if (!sa.commit()) return DDM_E_NOMEM;
  uint32_t* alist = sa.take<uint32_t>(A ? A : 1);
  if (!sa.fits()) return scratch_overrun("ddm_match_sbm lists");
  {
    ProfScope ps("sbm_lists", s);
    sbm_lists_kernel<<<(n + 255) / 256, 256, 0, s>>>(klo[0], n, rec, d, B, aoff, acur, alist);
    DDM_LAUNCHED("sbm_lists_kernel");
  }
  launch_sbm<false>(d, upd_lo, upd_hi, m, uid[0], klo[0], n, rec, kid[0], aoff, alist, cnt,
                    nullptr, nullptr, s);
  DDM_LAUNCHED("sbm_match_kernel");
  r = scan_u32_u64(cnt, off, m, stmp, s);
  if (r != DDM_OK) return r;
  sbm_words_kernel<<<1, 64, 0, s>>>(off, m, flag, words);
  DDM_LAUNCHED("sbm_words_kernel");
  DDM_HIP(hipMemcpyAsync(h, words, sizeof(h), hipMemcpyDeviceToHost, s));
  DDM_HIP(hipStreamSynchronize(s));
  *out_count = h[0];
  if (h[0] > capacity) {
    set_detail("result larger than capacity");
    return DDM_E_CAPACITY;
  }
  if (h[0] == 0) return DDM_OK;
  if (!out_pairs) return DDM_E_INVALID_ARG;
  launch_sbm<true>(d, upd_lo, upd_hi, m, uid[0], klo[0], n, rec, kid[0], aoff, alist, nullptr,
                   off, out_pairs, s);
  DDM_LAUNCHED("sbm_match_kernel");
  return sort_segments_keys(off, m, out_pairs, h[0], n, lists, lists_count, s);
}
