// Learned output sizing: a small MLP (18 -> 64 -> 64 -> 1, FP32, ReLU) that
// predicts log1p(number of subscriptions an update meets) from the update's
// extent and coarse prefix histograms of the subscription endpoints.  It
// only sizes the output of the single-pass matcher; every pair still comes
// from the exact traversal, and an update whose prediction falls short is
// redone by the plain count -> scan -> fill path, so results never depend on
// the network.
//
// Kernels: per-tree feature statistics (built with the tree), per-update
// features, forward (inference and capacities), forward + backward with
// per-workgroup partial gradients reduced in a fixed order (deterministic),
// and Adam.
#include "ddm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

namespace ddm {

// ---------------------------------------------------------------------------
// parameter layout (row-major W[out][in])
// ---------------------------------------------------------------------------
constexpr int kIn = kFeatures;
constexpr int kHid = 64;
constexpr int oW1 = 0;
constexpr int oB1 = oW1 + kHid * kIn;    // 1152
constexpr int oW2 = oB1 + kHid;          // 1216
constexpr int oB2 = oW2 + kHid * kHid;   // 5312
constexpr int oW3 = oB2 + kHid;          // 5376
constexpr int oB3 = oW3 + kHid;          // 5440
static_assert(oB3 + 1 == kParams, "parameter count");

// ---------------------------------------------------------------------------
// per-tree feature statistics (enqueued by the tree build)
//   fstat[k] = {min lower bound, width = max upper - min lower, mean length}
//   fcum[k][0][b] = #{lo < e_b}, fcum[k][1][b] = #{hi in bins < b},
//   e_b = min + width * b / 64, b = 0..64
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t hist_bin(float x, float mn, float w) {
  const float u = (x - mn) / w * (float)kFeatBins;
  if (!(u > 0.f)) return 0u;
  return min((uint32_t)u, (uint32_t)kFeatBins - 1u);
}

__global__ __launch_bounds__(256) void feat_hist_kernel(FeatArgs A, double* __restrict__ part) {
  __shared__ uint32_t h[kFeatBins];
  __shared__ double ws[256 / kWave];
  const uint32_t k = blockIdx.y;
  const uint32_t D = A.d;
  const uint32_t tid = threadIdx.x;
  if (tid < kFeatBins) h[tid] = 0;
  __syncthreads();
  const float mn = A.rec[k][2 * D];  // lower bound at in-order position 1
  const float mx = A.maxhi[k][A.root];
  const float w = fmaxf(mx - mn, 1e-30f);
  double ext = 0.0;
  for (uint32_t p = 1 + blockIdx.x * 256 + tid; p <= A.n; p += gridDim.x * 256) {
    const float lo = A.rec[k][(size_t)p * 2 * D];
    const float hi = A.rec[k][(size_t)p * 2 * D + 1];
    atomicAdd(&h[hist_bin(hi, mn, w)], 1u);
    ext += (double)hi - (double)lo;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ext += __shfl_xor(ext, o, kWave);
  if (lane_id() == 0) ws[tid / kWave] = ext;
  __syncthreads();
  if (tid < kFeatBins && h[tid]) atomicAdd(&A.fcum[(k * 2 + 1) * (kFeatBins + 1) + tid + 1], h[tid]);
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < 256 / kWave; ++i) t += ws[i];
    part[(size_t)k * gridDim.x + blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(128) void feat_final_kernel(FeatArgs A, const double* __restrict__ part,
                                                         uint32_t nparts) {
  const uint32_t k = blockIdx.x;
  const uint32_t D = A.d;
  const float mn = A.rec[k][2 * D];
  const float mx = A.maxhi[k][A.root];
  const float w = fmaxf(mx - mn, 1e-30f);
  const uint32_t b = threadIdx.x;
  if (b <= kFeatBins) {
    const float e = (b == kFeatBins) ? mx : mn + w * (float)b / (float)kFeatBins;
    const uint32_t* keys[1] = {A.skey_lo[k]};
    const uint32_t* idx[1] = {A.sidx_lo[k]};
    const uint32_t x[1] = {f2key(e)};
    const bool up[1] = {b == kFeatBins};
    uint32_t res[1];
    count_2l<1>(keys, idx, x, up, A.n, A.ns, res);
    A.fcum[(k * 2) * (kFeatBins + 1) + b] = res[0];
  }
  __syncthreads();
  if (b == 0) {
    uint32_t* c = A.fcum + (k * 2 + 1) * (kFeatBins + 1);
    c[0] = 0;
    for (uint32_t i = 1; i <= (uint32_t)kFeatBins; ++i) c[i] += c[i - 1];
    double t = 0.0;
    for (uint32_t i = 0; i < nparts; ++i) t += part[(size_t)k * nparts + i];
    A.fstat[k * 4 + 0] = mn;
    A.fstat[k * 4 + 1] = w;
    A.fstat[k * 4 + 2] = (float)(t / (double)A.n);
    A.fstat[k * 4 + 3] = 0.f;
  }
}

__global__ void feat_zero_kernel(uint32_t* __restrict__ fcum, uint32_t count,
                                 uint32_t* __restrict__ sat) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) fcum[i] = 0;
  if (i < kSatWords) sat[i] = 0;
}

// joint histogram of the subscriptions' lower corners on a G^d grid over the
// bounding box; entry (i0+1, i1+1, ...) of the (G+1)^d array counts the
// corners of cell (i0, i1, ...).  Corners are read from tree 0's records
// (lower bound of dimension 0, then those of the other dimensions).  Each
// workgroup counts into LDS and adds its nonzero cells to the global array.
__global__ __launch_bounds__(256) void sat_hist_kernel(FeatArgs A) {
  __shared__ uint32_t h[kSatWords];
  const uint32_t D = A.d;
  if (D > 3) return;
  const uint32_t G = sat_grid(D);
  uint32_t cells = 1;
  for (uint32_t k = 0; k < D; ++k) cells *= G + 1;
  for (uint32_t i = threadIdx.x; i < cells; i += 256) h[i] = 0;
  __syncthreads();
  for (uint32_t p = 1 + blockIdx.x * 256 + threadIdx.x; p <= A.n; p += gridDim.x * 256) {
    uint32_t idx = 0, stride = 1;
    for (uint32_t k = 0; k < D; ++k) {
      const float lo = A.rec[0][(size_t)p * 2 * D + 2 * k];
      const float u = (lo - A.fstat[k * 4 + 0]) / A.fstat[k * 4 + 1] * (float)G;
      const uint32_t c = !(u > 0.f) ? 0u : min((uint32_t)u, G - 1u);
      idx += (c + 1) * stride;
      stride *= G + 1;
    }
    atomicAdd(&h[idx], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < cells; i += 256)
    if (h[i]) atomicAdd(&A.sat[i], h[i]);
}

// prefix sums along every axis in LDS: sat[i...] = corners in cells < i
__global__ __launch_bounds__(1024) void sat_prefix_kernel(FeatArgs A) {
  __shared__ uint32_t h[kSatWords];
  const uint32_t D = A.d;
  if (D > 3) return;
  const uint32_t G1 = sat_grid(D) + 1;
  uint32_t cells = 1;
  for (uint32_t k = 0; k < D; ++k) cells *= G1;
  for (uint32_t i = threadIdx.x; i < cells; i += blockDim.x) h[i] = A.sat[i];
  __syncthreads();
  const uint32_t lines = cells / G1;
  uint32_t stride = 1;
  for (uint32_t ax = 0; ax < D; ++ax) {
    for (uint32_t l = threadIdx.x; l < lines; l += blockDim.x) {
      // base index: l enumerates the other axes
      uint32_t base = 0, rem = l, st = 1;
      for (uint32_t k = 0; k < D; ++k) {
        if (k != ax) {
          base += (rem % G1) * st;
          rem /= G1;
        }
        st *= G1;
      }
      uint32_t run = 0;
      for (uint32_t i = 0; i < G1; ++i) {
        run += h[base + i * stride];
        h[base + i * stride] = run;
      }
    }
    stride *= G1;
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < cells; i += blockDim.x) A.sat[i] = h[i];
}

ddm_status enqueue_feature_stats(const FeatArgs& A, hipStream_t s) {
  const uint32_t nparts = 64;
  Scratch sc(s);
  sc.reserve(sizeof(double) * nparts * A.d);
  if (!sc.commit()) return DDM_E_NOMEM;
  double* part = sc.take<double>(nparts * A.d);
  if (!sc.fits()) return scratch_overrun("feature statistics");
  const uint32_t cnt = A.d * 2 * (kFeatBins + 1);
  feat_zero_kernel<<<(std::max(cnt, kSatWords) + 255) / 256, 256, 0, s>>>(A.fcum, cnt, A.sat);
  DDM_LAUNCHED("feat_zero_kernel");
  feat_hist_kernel<<<dim3(nparts, A.d), 256, 0, s>>>(A, part);
  DDM_LAUNCHED("feat_hist_kernel");
  feat_final_kernel<<<A.d, 128, 0, s>>>(A, part, nparts);
  DDM_LAUNCHED("feat_final_kernel");
  if (A.d <= 3) {
    sat_hist_kernel<<<nparts, 256, 0, s>>>(A);
    DDM_LAUNCHED("sat_hist_kernel");
    sat_prefix_kernel<<<1, 1024, 0, s>>>(A);
    DDM_LAUNCHED("sat_prefix_kernel");
  }
  return DDM_OK;
}

// ---------------------------------------------------------------------------
// features of one update (d <= 3), see the header for their definition
// ---------------------------------------------------------------------------
__device__ __forceinline__ float interp_cum(const uint32_t* __restrict__ c, float u) {
  if (!(u > 0.f)) return (float)c[0];
  if (u >= (float)kFeatBins) return (float)c[kFeatBins];
  const uint32_t b = (uint32_t)u;
  const float fr = u - (float)b;
  return (float)c[b] + fr * ((float)c[b + 1] - (float)c[b]);
}

// corners counted by the prefix array below the point u (grid units, one per
// dimension), multilinear inside a cell (corners spread evenly in a cell).
// Evaluated in double: the box count below is a signed sum of 2^d such
// values that can cancel to a small number.
template <int D>
__device__ __forceinline__ double sat_at(const uint32_t* __restrict__ sat, const float (&u)[D]) {
  constexpr uint32_t G = sat_grid(D);
  uint32_t i[D];
  double f[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float uk = fminf(fmaxf(u[k], 0.f), (float)G);
    i[k] = min((uint32_t)uk, G - 1u);
    f[k] = (double)uk - (double)i[k];
  }
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < (1 << D); ++c) {
    double w = 1.0;
    uint32_t idx = 0, st = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const bool hi = (c >> k) & 1;
      w *= hi ? f[k] : 1.0 - f[k];
      idx += (i[k] + (hi ? 1u : 0u)) * st;
      st *= G + 1;
    }
    acc += w * (double)sat[idx];
  }
  return acc;
}

// corners in the box [a, b] (grid units), by inclusion-exclusion
template <int D>
__device__ __forceinline__ double sat_box(const uint32_t* __restrict__ sat, const float (&a)[D],
                                          const float (&b)[D]) {
  double tot = 0.0;
#pragma unroll
  for (int c = 0; c < (1 << D); ++c) {
    float u[D];
    int neg = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const bool hi = (c >> k) & 1;
      u[k] = hi ? b[k] : a[k];
      neg += hi ? 0 : 1;
    }
    const double v = sat_at<D>(sat, u);
    tot += (neg & 1) ? -v : v;
  }
  return tot;
}

template <int D>
__global__ __launch_bounds__(256) void features_kernel(FeatDev F, const float* __restrict__ ulo,
                                                       const float* __restrict__ uhi, uint32_t m,
                                                       float* __restrict__ X) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  float f[kFeatures];
#pragma unroll
  for (int i = 0; i < kFeatures; ++i) f[i] = 0.f;
  const float n = (float)F.n;
  constexpr float G = (float)sat_grid(D);
  float ga[D], gb[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float ql = ulo[(size_t)k * m + j], qh = uhi[(size_t)k * m + j];
    const float mn = F.fstat[k * 4 + 0], w = F.fstat[k * 4 + 1], me = F.fstat[k * 4 + 2];
    const uint32_t* clo = F.fcum + (k * 2) * (kFeatBins + 1);
    const uint32_t* chi = F.fcum + (k * 2 + 1) * (kFeatBins + 1);
    const float c_le = interp_cum(clo, (qh - mn) / w * (float)kFeatBins);
    const float c_lt = interp_cum(chi, (ql - mn) / w * (float)kFeatBins);
    const float c = fminf(fmaxf(c_le - c_lt, 0.f), n);
    f[5 * k + 0] = (qh - ql) / w;
    f[5 * k + 1] = (0.5f * (ql + qh) - mn) / w;
    f[5 * k + 2] = c / n;
    f[5 * k + 3] = log1pf(c) * (1.f / 16.f);
    f[5 * k + 4] = me / w;
    // lower corners that can meet q in this dimension: [q.lo - mean length, q.hi]
    ga[k] = (ql - me - mn) / w * G;
    gb[k] = (qh - mn) / w * G;
  }
  f[15] = log2f(n) * (1.f / 20.f);
  f[16] = (float)D * (1.f / 3.f);
  f[17] = log1pf((float)fmax(sat_box<D>(F.sat, ga, gb), 0.0)) * (1.f / 16.f);
#pragma unroll
  for (int i = 0; i < kFeatures; ++i) X[(size_t)j * kFeatures + i] = f[i];
}

ddm_status launch_features(const FeatDev& F, uint32_t d, const float* ulo, const float* uhi,
                           uint32_t m, float* X, hipStream_t s) {
  if (m == 0) return DDM_OK;
  ProfScope ps("features", s);
  switch (d) {
    case 1: features_kernel<1><<<(m + 255) / 256, 256, 0, s>>>(F, ulo, uhi, m, X); break;
    case 2: features_kernel<2><<<(m + 255) / 256, 256, 0, s>>>(F, ulo, uhi, m, X); break;
    case 3: features_kernel<3><<<(m + 255) / 256, 256, 0, s>>>(F, ulo, uhi, m, X); break;
    default:
      set_detail("features: d must be at most 3");
      return DDM_E_INVALID_ARG;
  }
  DDM_LAUNCHED("features_kernel");
  return DDM_OK;
}

// ---------------------------------------------------------------------------
// MLP forward: one thread per sample, parameters in LDS (broadcast reads)
//   out_mode 0: yhat[s] = prediction
//   out_mode 1: cap[s] = min(ceil(expm1(prediction + delta)), capmax)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ params,
                                                          const float* __restrict__ X, uint32_t N,
                                                          int out_mode, float delta,
                                                          uint32_t capmax,
                                                          float* __restrict__ yhat,
                                                          uint32_t* __restrict__ cap) {
  __shared__ float P[kParams];
  for (uint32_t i = threadIdx.x; i < (uint32_t)kParams; i += blockDim.x) P[i] = params[i];
  __syncthreads();
  const uint32_t sidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (sidx >= N) return;
  float x[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = X[(size_t)sidx * kIn + i];
  float h1[kHid];
#pragma unroll
  for (int o = 0; o < kHid; ++o) {
    float a = P[oB1 + o];
#pragma unroll
    for (int i = 0; i < kIn; ++i) a = fmaf(P[oW1 + o * kIn + i], x[i], a);
    h1[o] = fmaxf(a, 0.f);
  }
  float y = P[oB3];
  for (int o = 0; o < kHid; ++o) {
    float a = P[oB2 + o];
#pragma unroll
    for (int i = 0; i < kHid; ++i) a = fmaf(P[oW2 + o * kHid + i], h1[i], a);
    y = fmaf(P[oW3 + o], fmaxf(a, 0.f), y);
  }
  if (out_mode == 0) {
    yhat[sidx] = y;
  } else {
    const float e = expm1f(fminf(y + delta, 30.f));
    const float c = ceilf(fmaxf(e, 0.f));
    cap[sidx] = c >= (float)capmax ? capmax : (uint32_t)c;
  }
}

ddm_status launch_mlp_forward(const float* params, const float* X, uint32_t N, int out_mode,
                              float delta, uint32_t capmax, float* yhat, uint32_t* cap,
                              hipStream_t s) {
  if (N == 0) return DDM_OK;
  ProfScope ps("mlp_forward", s);
  mlp_forward_kernel<<<(N + 255) / 256, 256, 0, s>>>(params, X, N, out_mode, delta, capmax, yhat,
                                                       cap);
  DDM_LAUNCHED("mlp_forward_kernel");
  return DDM_OK;
}

// ---------------------------------------------------------------------------
// MLP forward + backward of the mean squared error over N samples.
// One workgroup of 128 threads handles 128 samples (one per thread) and
// writes its partial gradient; mlp_reduce_kernel sums the partials in a
// fixed order.
// ---------------------------------------------------------------------------
constexpr int kGB = 128;   // samples per workgroup
constexpr int kPad = 65;   // LDS row stride (bank-conflict padding)

__global__ __launch_bounds__(kGB) void mlp_grad_kernel(const float* __restrict__ params,
                                                       const float* __restrict__ X,
                                                       const float* __restrict__ Y, uint32_t N,
                                                       float* __restrict__ part,
                                                       float* __restrict__ part_loss) {
  __shared__ float P[kParams];
  __shared__ float H1[kGB][kPad];
  __shared__ float H2[kGB][kPad];
  __shared__ float D2[kGB][kPad];
  __shared__ float XS[kGB][kIn + 1];
  __shared__ float DY[kGB];
  __shared__ float LS[kGB];
  const uint32_t t = threadIdx.x;
  for (uint32_t i = t; i < (uint32_t)kParams; i += kGB) P[i] = params[i];
  __syncthreads();
  const uint32_t sidx = blockIdx.x * kGB + t;
  const bool valid = sidx < N;
  const float invN = 1.f / (float)N;
  float x[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = valid ? X[(size_t)sidx * kIn + i] : 0.f;
  const float ylab = valid ? Y[sidx] : 0.f;
  // forward
  float h1[kHid];
#pragma unroll
  for (int o = 0; o < kHid; ++o) {
    float a = P[oB1 + o];
#pragma unroll
    for (int i = 0; i < kIn; ++i) a = fmaf(P[oW1 + o * kIn + i], x[i], a);
    h1[o] = fmaxf(a, 0.f);
    H1[t][o] = h1[o];
  }
  float y = P[oB3];
  for (int o = 0; o < kHid; ++o) {
    float a = P[oB2 + o];
#pragma unroll
    for (int i = 0; i < kHid; ++i) a = fmaf(P[oW2 + o * kHid + i], h1[i], a);
    const float h2 = fmaxf(a, 0.f);
    H2[t][o] = h2;
    y = fmaf(P[oW3 + o], h2, y);
  }
  const float r = valid ? (y - ylab) : 0.f;
  const float dy = 2.f * r * invN;
  DY[t] = dy;
  LS[t] = r * r * invN;
#pragma unroll
  for (int i = 0; i < kIn; ++i) XS[t][i] = x[i];
  for (int o = 0; o < kHid; ++o) D2[t][o] = H2[t][o] > 0.f ? dy * P[oW3 + o] : 0.f;
  __syncthreads();
  float* g = part + (size_t)blockIdx.x * kParams;
  // output layer and second-layer bias
  if (t < (uint32_t)kHid) {
    float a = 0.f, b = 0.f;
    for (int q = 0; q < kGB; ++q) {
      a = fmaf(DY[q], H2[q][t], a);
      b += D2[q][t];
    }
    g[oW3 + t] = a;
    g[oB2 + t] = b;
  }
  if (t == kHid) {
    float a = 0.f, l = 0.f;
    for (int q = 0; q < kGB; ++q) {
      a += DY[q];
      l += LS[q];
    }
    g[oB3] = a;
    part_loss[blockIdx.x] = l;
  }
  // dW2[o][i] = sum_q D2[q][o] H1[q][i]: thread t owns a 4 x 8 tile
  {
    const int o0 = (t / 8) * 4, i0 = (t % 8) * 8;
    float acc[4][8];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 8; ++b) acc[a][b] = 0.f;
    for (int q = 0; q < kGB; ++q) {
      float dv[4], hv[8];
#pragma unroll
      for (int a = 0; a < 4; ++a) dv[a] = D2[q][o0 + a];
#pragma unroll
      for (int b = 0; b < 8; ++b) hv[b] = H1[q][i0 + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = fmaf(dv[a], hv[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 8; ++b) g[oW2 + (o0 + a) * kHid + i0 + b] = acc[a][b];
  }
  __syncthreads();
  // back to the first layer: dz1 = (W2^T dz2) * [z1 > 0], stored over H1
  {
    float dz2[kHid];
#pragma unroll
    for (int o = 0; o < kHid; ++o) dz2[o] = D2[t][o];
    for (int i = 0; i < kHid; ++i) {
      float a = 0.f;
#pragma unroll
      for (int o = 0; o < kHid; ++o) a = fmaf(P[oW2 + o * kHid + i], dz2[o], a);
      H1[t][i] = H1[t][i] > 0.f ? a : 0.f;
    }
  }
  __syncthreads();
  // dW1[o][i] = sum_q dz1[q][o] x[q][i], db1[o] = sum_q dz1[q][o]
  {
    const int o = t / 2, ib = (t % 2) * (kIn / 2);
    float acc[kIn / 2], b = 0.f;
#pragma unroll
    for (int i = 0; i < kIn / 2; ++i) acc[i] = 0.f;
    for (int q = 0; q < kGB; ++q) {
      const float dz = H1[q][o];
      b += dz;
#pragma unroll
      for (int i = 0; i < kIn / 2; ++i) acc[i] = fmaf(dz, XS[q][ib + i], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < kIn / 2; ++i) g[oW1 + o * kIn + ib + i] = acc[i];
    if (t % 2 == 0) g[oB1 + o] = b;
  }
}

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ part,
                                                         const float* __restrict__ part_loss,
                                                         uint32_t nb, float* __restrict__ grad,
                                                         float* __restrict__ loss) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < (uint32_t)kParams) {
    float a = 0.f;
    for (uint32_t b = 0; b < nb; ++b) a += part[(size_t)b * kParams + p];
    grad[p] = a;
  }
  if (p == 0 && loss) {
    float l = 0.f;
    for (uint32_t b = 0; b < nb; ++b) l += part_loss[b];
    *loss = l;
  }
}

ddm_status launch_mlp_grad(const float* params, const float* X, const float* Y, uint32_t N,
                           float* grad, float* loss, hipStream_t s) {
  if (N == 0) {
    set_detail("mlp gradient of an empty batch");
    return DDM_E_INVALID_ARG;
  }
  const uint32_t nb = (N + kGB - 1) / kGB;
  Scratch sc(s);
  sc.reserve(sizeof(float) * kParams * (size_t)nb);
  sc.reserve(sizeof(float) * nb);
  if (!sc.commit()) return DDM_E_NOMEM;
  float* part = sc.take<float>(kParams * (size_t)nb);
  float* pl = sc.take<float>(nb);
  if (!sc.fits()) return scratch_overrun("predictor gradient");
  ProfScope ps("mlp_grad", s);
  mlp_grad_kernel<<<nb, kGB, 0, s>>>(params, X, Y, N, part, pl);
  DDM_LAUNCHED("mlp_grad_kernel");
  mlp_reduce_kernel<<<(kParams + 255) / 256, 256, 0, s>>>(part, pl, nb, grad, loss);
  DDM_LAUNCHED("mlp_reduce_kernel");
  return DDM_OK;
}

__global__ void adam_kernel(float* __restrict__ params, float* __restrict__ m1,
                            float* __restrict__ m2, const float* __restrict__ grad, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (uint32_t)kParams) return;
  const float g = grad[p];
  const float a = b1 * m1[p] + (1.f - b1) * g;
  const float v = b2 * m2[p] + (1.f - b2) * g * g;
  m1[p] = a;
  m2[p] = v;
  params[p] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// counter-based uniform numbers for the initial weights (splitmix64)
__device__ __forceinline__ float init_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (float)(z >> 40) * (1.f / 16777216.f);
}

// U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases of each layer
__global__ void mlp_init_kernel(float* __restrict__ params, uint64_t seed) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (uint32_t)kParams) return;
  const float fan = p < (uint32_t)oW2 ? (float)kIn : (p < (uint32_t)oW3 ? (float)kHid : (float)kHid);
  const float bound = 1.f / sqrtf(fan);
  params[p] = (2.f * init_uniform(seed, p) - 1.f) * bound;
}

__global__ void fill_f32_kernel(float* __restrict__ p, float v, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

}  // namespace ddm

using namespace ddm;

struct ddm_predictor {
  int device = 0;
  float* block = nullptr;  // params | adam m | adam v | grad | loss
  float* params = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* grad = nullptr;
  float* loss = nullptr;
  uint64_t step = 0;
  float delta = 0.f;
};

namespace ddm {
const float* predictor_params(const ddm_predictor* p) { return p->params; }
float predictor_delta(const ddm_predictor* p) { return p->delta; }
int predictor_device(const ddm_predictor* p) { return p->device; }
}  // namespace ddm

extern "C" ddm_status ddm_predictor_create(uint64_t seed, ddm_predictor** out) {
  set_detail("");
  if (!out) return DDM_E_INVALID_ARG;
  *out = nullptr;
  ddm_predictor* p = new (std::nothrow) ddm_predictor();
  if (!p) return DDM_E_NOMEM;
  DDM_HIP(hipGetDevice(&p->device));
  const size_t words = (size_t)kParams * 4 + 64;
  hipError_t e = hipMalloc((void**)&p->block, words * sizeof(float));
  if (e != hipSuccess) {
    delete p;
    (void)hipGetLastError();
    set_detail("predictor allocation failed");
    return DDM_E_NOMEM;
  }
  p->params = p->block;
  p->m1 = p->params + kParams;
  p->m2 = p->m1 + kParams;
  p->grad = p->m2 + kParams;
  p->loss = p->grad + kParams;
  mlp_init_kernel<<<(kParams + 255) / 256, 256>>>(p->params, seed);
  fill_f32_kernel<<<(2 * kParams + 255) / 256, 256>>>(p->m1, 0.f, 2 * kParams);
  e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(p->block);
    delete p;
    return hip_fail(e, "ddm_predictor_create", __FILE__, __LINE__);
  }
  *out = p;
  return DDM_OK;
}

extern "C" void ddm_predictor_free(ddm_predictor* p) {
  if (!p) return;
  if (p->block) (void)hipFree(p->block);
  delete p;
}

extern "C" ddm_status ddm_predictor_get_params(const ddm_predictor* p, float* host,
                                               uint32_t count, float* delta) {
  set_detail("");
  if (!p || (count && !host)) return DDM_E_INVALID_ARG;
  if (count != 0 && count != (uint32_t)kParams) {
    set_detail("count must be DDM_PREDICTOR_PARAMS");
    return DDM_E_INVALID_ARG;
  }
  if (count) DDM_HIP(hipMemcpy(host, p->params, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  if (delta) *delta = p->delta;
  return DDM_OK;
}

extern "C" ddm_status ddm_predictor_set_params(ddm_predictor* p, const float* host,
                                               uint32_t count, float delta) {
  set_detail("");
  if (!p || (count && !host)) return DDM_E_INVALID_ARG;
  if (count != 0 && count != (uint32_t)kParams) {
    set_detail("count must be DDM_PREDICTOR_PARAMS");
    return DDM_E_INVALID_ARG;
  }
  if (!std::isfinite(delta)) {
    set_detail("delta must be finite");
    return DDM_E_INVALID_ARG;
  }
  if (count) {
    for (uint32_t i = 0; i < count; ++i)
      if (!std::isfinite(host[i])) {
        set_detail("parameters must be finite");
        return DDM_E_INVALID_ARG;
      }
    DDM_HIP(hipMemcpy(p->params, host, sizeof(float) * kParams, hipMemcpyHostToDevice));
  }
  p->delta = delta;
  return DDM_OK;
}

// Predictor file: "DDMP", format version, parameter count, delta (as its
// float bits), each a little-endian 32-bit word, then the parameters.
static const char kPredMagic[4] = {'D', 'D', 'M', 'P'};
constexpr uint32_t kPredVersion = 1;

extern "C" ddm_status ddm_predictor_save(const ddm_predictor* p, const char* path) {
  set_detail("");
  if (!p || !path) return DDM_E_INVALID_ARG;
  std::vector<float> w(kParams);
  float delta = 0.f;
  ddm_status st = ddm_predictor_get_params(p, w.data(), (uint32_t)kParams, &delta);
  if (st != DDM_OK) return st;
  uint32_t hdr[4];
  std::memcpy(&hdr[0], kPredMagic, 4);
  hdr[1] = kPredVersion;
  hdr[2] = (uint32_t)kParams;
  std::memcpy(&hdr[3], &delta, 4);
  FILE* f = std::fopen(path, "wb");
  if (!f) {
    set_detail(std::string("ddm_predictor_save: cannot open ") + path);
    return DDM_E_INVALID_ARG;
  }
  const bool ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
                  std::fwrite(w.data(), sizeof(float), w.size(), f) == w.size();
  if (std::fclose(f) != 0 || !ok) {
    set_detail(std::string("ddm_predictor_save: write failed: ") + path);
    return DDM_E_INVALID_ARG;
  }
  return DDM_OK;
}

extern "C" ddm_status ddm_predictor_load(const char* path, ddm_predictor** out) {
  set_detail("");
  if (!path || !out) return DDM_E_INVALID_ARG;
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    set_detail(std::string("ddm_predictor_load: cannot open ") + path);
    return DDM_E_INVALID_ARG;
  }
  uint32_t hdr[4];
  std::vector<float> w(kParams);
  bool ok = std::fread(hdr, sizeof(hdr), 1, f) == 1 && std::memcmp(&hdr[0], kPredMagic, 4) == 0 &&
            hdr[1] == kPredVersion && hdr[2] == (uint32_t)kParams &&
            std::fread(w.data(), sizeof(float), w.size(), f) == w.size();
  char extra;
  ok = ok && std::fread(&extra, 1, 1, f) == 0;  // nothing after the parameters
  std::fclose(f);
  if (!ok) {
    set_detail(std::string("ddm_predictor_load: not a predictor file of this version: ") + path);
    return DDM_E_INVALID_INPUT;
  }
  float delta;
  std::memcpy(&delta, &hdr[3], 4);
  ddm_predictor* p = nullptr;
  ddm_status st = ddm_predictor_create(0, &p);
  if (st != DDM_OK) return st;
  st = ddm_predictor_set_params(p, w.data(), (uint32_t)kParams, delta);
  if (st != DDM_OK) {
    const std::string why = ddm_last_error_detail();
    ddm_predictor_free(p);
    set_detail("ddm_predictor_load: " + why);
    return DDM_E_INVALID_INPUT;
  }
  *out = p;
  return DDM_OK;
}

extern "C" ddm_status ddm_predictor_forward(const ddm_predictor* p, const float* X, uint32_t N,
                                            float* yhat, void* stream) {
  set_detail("");
  if (!p || (N && (!X || !yhat))) return DDM_E_INVALID_ARG;
  return launch_mlp_forward(p->params, X, N, 0, 0.f, 0, yhat, nullptr, (hipStream_t)stream);
}

extern "C" ddm_status ddm_predictor_grad(const ddm_predictor* p, const float* X, const float* Y,
                                         uint32_t N, float* grad, float* loss, void* stream) {
  set_detail("");
  if (!p || !X || !Y || !grad || N == 0) return DDM_E_INVALID_ARG;
  return launch_mlp_grad(p->params, X, Y, N, grad, loss, (hipStream_t)stream);
}

extern "C" ddm_status ddm_predictor_adam(ddm_predictor* p, const float* grad, float lr,
                                         void* stream) {
  set_detail("");
  if (!p || !grad || !(lr > 0.f)) return DDM_E_INVALID_ARG;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  p->step += 1;
  const float c1 = 1.f - (float)std::pow((double)b1, (double)p->step);
  const float c2 = 1.f - (float)std::pow((double)b2, (double)p->step);
  adam_kernel<<<(kParams + 255) / 256, 256, 0, (hipStream_t)stream>>>(p->params, p->m1, p->m2,
                                                                     grad, lr, b1, b2, eps, c1, c2);
  DDM_LAUNCHED("adam_kernel");
  return DDM_OK;
}

extern "C" ddm_status ddm_predictor_train(ddm_predictor* p, const float* X, const float* Y,
                                          uint32_t N, uint32_t batch, uint32_t epochs, float lr,
                                          void* stream, float* epoch_loss) {
  set_detail("");
  if (!p || !X || !Y || N == 0 || batch == 0 || epochs == 0 || !(lr > 0.f))
    return DDM_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const uint32_t nbat = (N + batch - 1) / batch;
  Scratch sc(s);
  sc.reserve(sizeof(float) * (size_t)nbat * epochs);
  if (!sc.commit()) return DDM_E_NOMEM;
  float* losses = sc.take<float>((size_t)nbat * epochs);
  if (!sc.fits()) return scratch_overrun("predictor training");
  for (uint32_t e = 0; e < epochs; ++e) {
    for (uint32_t b = 0; b < nbat; ++b) {
      const uint32_t s0 = b * batch;
      const uint32_t nb = std::min(batch, N - s0);
      ddm_status r = launch_mlp_grad(p->params, X + (size_t)s0 * kIn, Y + s0, nb, p->grad,
                                     losses + (size_t)e * nbat + b, s);
      if (r != DDM_OK) return r;
      r = ddm_predictor_adam(p, p->grad, lr, stream);
      if (r != DDM_OK) return r;
    }
  }
  if (epoch_loss) {
    std::vector<float> h((size_t)nbat * epochs);
    DDM_HIP(hipMemcpyAsync(h.data(), losses, sizeof(float) * h.size(), hipMemcpyDeviceToHost, s));
    DDM_HIP(hipStreamSynchronize(s));
    for (uint32_t e = 0; e < epochs; ++e) {
      double t = 0.0, w = 0.0;
      for (uint32_t b = 0; b < nbat; ++b) {
        const double nb = std::min(batch, N - b * batch);
        t += h[(size_t)e * nbat + b] * nb;
        w += nb;
      }
      epoch_loss[e] = (float)(t / w);
    }
  }
  return DDM_OK;
}
