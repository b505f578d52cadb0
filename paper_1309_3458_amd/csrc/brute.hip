// Brute-Force Matching on the device (Algorithm 2): every update is tested
// against every subscription with the closed predicate in every dimension
// (Sec. III-A).  It is the paper's embarrassingly parallel baseline, kept
// here to measure Interval Tree Matching against on the same GPU; results
// are the same keys in the same order as ddm_match.
//
// One lane per update; a workgroup stages 1024 subscriptions at a time in
// LDS (coalesced loads, broadcast reads) and every lane tests them in id
// order, so each update's hits come out already sorted: count pass, scan,
// fill pass, no segment sort.
#include "ddm_internal.h"

namespace ddm {

constexpr uint32_t kBfChunk = 1024;
constexpr uint32_t kBfThreads = 256;

template <int D, bool FILL>
__global__ __launch_bounds__(kBfThreads) void brute_kernel(
    const float* __restrict__ slo, const float* __restrict__ shi, uint32_t n,
    const float* __restrict__ ulo, const float* __restrict__ uhi, uint32_t m,
    uint32_t* __restrict__ cnt, const uint64_t* __restrict__ off, uint64_t* __restrict__ out,
    int32_t* __restrict__ flag) {
  __shared__ float ss[kBfChunk * 2 * D];
  const uint32_t j = blockIdx.x * kBfThreads + threadIdx.x;
  const bool act = j < m;
  float ql[D], qh[D];
  bool bad = false;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    ql[k] = act ? ulo[(size_t)k * m + j] : INFINITY;
    qh[k] = act ? uhi[(size_t)k * m + j] : -INFINITY;
    if (act) bad = bad || !valid_extent(ql[k], qh[k]);
  }
  uint32_t c = 0;
  uint64_t base = (FILL && act) ? off[j] : 0;
  const uint64_t jhi = (uint64_t)j << 32;
  for (uint32_t c0 = 0; c0 < n; c0 += kBfChunk) {
    const uint32_t lim = min(kBfChunk, n - c0);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < lim; i += kBfThreads) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const float a = slo[(size_t)k * n + c0 + i], b = shi[(size_t)k * n + c0 + i];
        ss[i * 2 * D + 2 * k] = a;
        ss[i * 2 * D + 2 * k + 1] = b;
        // the subscriptions are validated once, by the first workgroup
        if (!FILL && blockIdx.x == 0 && !valid_extent(a, b)) atomicOr(flag, 1);
      }
    }
    __syncthreads();
    for (uint32_t i = 0; i < lim; ++i) {
      bool hit = true;
#pragma unroll
      for (int k = 0; k < D; ++k)
        hit = hit & (ss[i * 2 * D + 2 * k] <= qh[k]) & (ql[k] <= ss[i * 2 * D + 2 * k + 1]);
      if (hit) {
        if (FILL) out[base + c] = jhi | (c0 + i);
        ++c;
      }
    }
  }
  if (!FILL && act) cnt[j] = c;
  if (!FILL && ballot(bad) != 0 && lane_id() == 0) atomicOr(flag, 2);
}

template <bool FILL>
static ddm_status launch_brute(uint32_t d, const float* slo, const float* shi, uint32_t n,
                               const float* ulo, const float* uhi, uint32_t m, uint32_t* cnt,
                               const uint64_t* off, uint64_t* out, int32_t* flag,
                               hipStream_t s) {
  ProfScope ps(FILL ? "brute_fill" : "brute_count", s);
  const dim3 g((m + kBfThreads - 1) / kBfThreads);
  switch (d) {
    case 1: brute_kernel<1, FILL><<<g, kBfThreads, 0, s>>>(slo, shi, n, ulo, uhi, m, cnt, off, out, flag); break;
    case 2: brute_kernel<2, FILL><<<g, kBfThreads, 0, s>>>(slo, shi, n, ulo, uhi, m, cnt, off, out, flag); break;
    case 3: brute_kernel<3, FILL><<<g, kBfThreads, 0, s>>>(slo, shi, n, ulo, uhi, m, cnt, off, out, flag); break;
    default: brute_kernel<4, FILL><<<g, kBfThreads, 0, s>>>(slo, shi, n, ulo, uhi, m, cnt, off, out, flag); break;
  }
  DDM_LAUNCHED("brute_kernel");
  return DDM_OK;
}

__global__ void brute_init_kernel(int32_t* __restrict__ flag) {
  if (threadIdx.x == 0) *flag = 0;
}

__global__ void brute_words_kernel(const uint64_t* __restrict__ off, uint32_t m,
                                   const int32_t* __restrict__ flag, uint64_t* __restrict__ w) {
  if (threadIdx.x == 0) {
    w[0] = off[m];
    w[1] = (uint64_t)(uint32_t)*flag;
  }
}

}  // namespace ddm

using namespace ddm;

extern "C" ddm_status ddm_match_brute(const float* sub_lo, const float* sub_hi, uint32_t n,
                                      const float* upd_lo, const float* upd_hi, uint32_t m,
                                      uint32_t d, uint64_t* out_pairs, uint64_t capacity,
                                      uint64_t* out_count, void* stream) {
  set_detail("");
  if (!out_count) {
    set_detail("ddm_match_brute: out_count is NULL");
    return DDM_E_INVALID_ARG;
  }
  *out_count = 0;
  if (d < 1 || d > DDM_MAX_D || (n && (!sub_lo || !sub_hi)) || (m && (!upd_lo || !upd_hi)) ||
      m >= 0x80000000u) {
    set_detail("ddm_match_brute: d in [1, DDM_MAX_D], coordinate pointers, m < 2^31");
    return DDM_E_INVALID_ARG;
  }
  if (n == 0 || m == 0) return DDM_OK;
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  sc.reserve(sizeof(uint32_t) * m);
  sc.reserve(sizeof(uint64_t) * (m + 1));
  sc.reserve(sizeof(uint64_t) * scan_tmp_words(m));
  sc.reserve(sizeof(int32_t));
  sc.reserve(sizeof(uint64_t) * 2);
  if (!sc.commit()) return DDM_E_NOMEM;
  uint32_t* cnt = sc.take<uint32_t>(m);
  uint64_t* off = sc.take<uint64_t>(m + 1);
  uint64_t* tmp = sc.take<uint64_t>(scan_tmp_words(m));
  int32_t* flag = sc.take<int32_t>(1);
  uint64_t* words = sc.take<uint64_t>(2);
  if (!sc.fits()) return scratch_overrun("ddm_match_brute");
  brute_init_kernel<<<1, 64, 0, s>>>(flag);
  DDM_LAUNCHED("brute_init_kernel");
  ddm_status r = launch_brute<false>(d, sub_lo, sub_hi, n, upd_lo, upd_hi, m, cnt, nullptr,
                                     nullptr, flag, s);
  if (r != DDM_OK) return r;
  r = scan_u32_u64(cnt, off, m, tmp, s);
  if (r != DDM_OK) return r;
  brute_words_kernel<<<1, 64, 0, s>>>(off, m, flag, words);
  DDM_LAUNCHED("brute_words_kernel");
  uint64_t h[2] = {0, 0};
  DDM_HIP(hipMemcpyAsync(h, words, sizeof(h), hipMemcpyDeviceToHost, s));
  DDM_HIP(hipStreamSynchronize(s));
  if (h[1]) {
    set_detail(h[1] & 1 ? "subscription coordinates: NaN/inf or lo > hi"
                        : "update coordinates: NaN/inf or lo > hi");
    return DDM_E_INVALID_INPUT;
  }
  *out_count = h[0];
  if (h[0] > capacity) {
    set_detail("result larger than capacity");
    return DDM_E_CAPACITY;
  }
  if (h[0] == 0) return DDM_OK;
  if (!out_pairs) return DDM_E_INVALID_ARG;
  return launch_brute<true>(d, sub_lo, sub_hi, n, upd_lo, upd_hi, m, nullptr, off, out_pairs,
                            flag, s);
}
