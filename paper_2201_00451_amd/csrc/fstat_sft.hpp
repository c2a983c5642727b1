// Steps (i)-(ii) of Sec. 3 on the GPU: short Fourier transforms (SFTs) of
// the detector strain to the heterodyned, low-passed, downsampled series
// x_h(t_k) the resampling starts from.
//
// SFT s covers [t_s, t_s + T), t_s = t_start + s T, and holds the K bins
// k = k0 .. k0 + K - 1 (frequency k / T) of its segment's DFT, normalised by
// the raw time step.  Combining the SFTs into one transform and keeping the
// band is the low-pass; heterodyning at the band's centre f_h = (k0 + K/2)/T
// and transforming back over the band's K bins downsamples to dt = T / K.
// Sample j of SFT s is then
//   x_h(t_s + j dt) = (1/T) exp(-2 pi i f_h t_start) (-1)^j
//                     sum_q X_s[k0 + q] exp(+2 pi i q j / K)
// (f_h T is a whole number, so the heterodyne phase at t_s is the one at
// t_start, and f_h j dt = (k0 + K/2) j / K leaves (-1)^j after the bins'
// own phases): one K-point inverse DFT per SFT.
//
// One workgroup per SFT: a mixed-radix (4, 2, 3, 5) Stockham autosort in LDS
// (two buffers of K points and the K twiddles exp(+2 pi i e / K), written
// from FP64 phases), then the scaled, phased samples to HBM.  A missing SFT
// writes zeros and clears its validity.
#pragma once

#include "fstat_common.hpp"

namespace fstat {

constexpr int kSftMaxBins = 4096;
constexpr int kSftMaxStages = 16;
constexpr int kSftThreads = 256;

struct SftPlan {
  int32_t K, nstages;
  int32_t radix[kSftMaxStages];
  float scale;        // 1 / T
  float2 het;         // exp(-2 pi i f_h t_start)
};

// Inverse r-point DFT in registers: y_p = sum_q v_q exp(+2 pi i p q / r).
__device__ __forceinline__ float2 imul_i(float2 a) { return make_float2(-a.y, a.x); }

__device__ inline void idft2(float2* v) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
__device__ inline void idft4(float2* v) {
  const float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
  const float2 s13 = cadd(v[1], v[3]), d13 = imul_i(csub(v[1], v[3]));
  v[0] = cadd(s02, s13);
  v[1] = cadd(d02, d13);
  v[2] = csub(s02, s13);
  v[3] = csub(d02, d13);
}
__device__ inline void idft3(float2* v) {
  constexpr float kS3 = 0.86602540378443864676f;  // sin(2 pi / 3)
  const float2 t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
  const float2 a = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
  const float2 b = imul_i(cscale(t2, kS3));
  v[0] = cadd(v[0], t1);
  v[1] = cadd(a, b);
  v[2] = csub(a, b);
}
__device__ inline void idft5(float2* v) {
  constexpr float c1 = 0.30901699437494742410f, s1 = 0.95105651629515357212f;    // 2 pi / 5
  constexpr float c2 = -0.80901699437494742410f, s2 = 0.58778525229247312917f;   // 4 pi / 5
  const float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  const float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  const float2 a1 = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
  const float2 a2 = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
  const float2 b1 = imul_i(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
  const float2 b2 = imul_i(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
  v[0] = cadd(v[0], cadd(t1, t2));
  v[1] = cadd(a1, b1);
  v[4] = csub(a1, b1);
  v[2] = cadd(a2, b2);
  v[3] = csub(a2, b2);
}

// One Stockham stage of radix R: with L the length of the transforms built
// so far and m = K / R, butterfly b (j = b mod L, kb = b / L) combines
// in[b + q m], q < R, twiddled by W^{j q K / (L R)}, into
// out[kb L R + j + L p], p < R.
template <int R>
__device__ inline void sft_stage(const float2* in, float2* out, const float2* tw, int K, int L) {
  const int m = K / R;
  const int step = K / (L * R);
  for (int b = threadIdx.x; b < m; b += kSftThreads) {
    const int j = b % L, kb = b / L;
    float2 v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      v[q] = in[b + q * m];
      if (q > 0) v[q] = cmul(v[q], tw[j * q * step]);
    }
    if constexpr (R == 2) idft2(v);
    if constexpr (R == 3) idft3(v);
    if constexpr (R == 4) idft4(v);
    if constexpr (R == 5) idft5(v);
    const int o = kb * L * R + j;
#pragma unroll
    for (int p = 0; p < R; ++p) out[o + L * p] = v[p];
  }
}

__global__ __launch_bounds__(kSftThreads) void k_sft_series(SftPlan sp,
                                                             const float2* __restrict__ sfts,
                                                             const uint8_t* __restrict__ present,
                                                             float2* __restrict__ x,
                                                             uint8_t* __restrict__ valid) {
  extern __shared__ float2 sbuf[];
  const int K = sp.K;
  const int64_t seg = blockIdx.x;
  float2* out = x + seg * K;
  const bool have = present == nullptr || present[seg] != 0;
  if (!have) {
    for (int j = threadIdx.x; j < K; j += kSftThreads) {
      out[j] = make_float2(0.f, 0.f);
      if (valid) valid[seg * K + j] = 0;
    }
    return;
  }
  float2* b0 = sbuf;
  float2* b1 = sbuf + K;
  float2* tw = sbuf + 2 * K;
  for (int e = threadIdx.x; e < K; e += kSftThreads) {
    tw[e] = cis_cycles(double(e) / double(K));
    b0[e] = sfts[seg * K + e];
  }
  __syncthreads();
  int L = 1;
  for (int s = 0; s < sp.nstages; ++s) {
    const int r = sp.radix[s];
    if (r == 4) sft_stage<4>(b0, b1, tw, K, L);
    else if (r == 2) sft_stage<2>(b0, b1, tw, K, L);
    else if (r == 3) sft_stage<3>(b0, b1, tw, K, L);
    else sft_stage<5>(b0, b1, tw, K, L);
    __syncthreads();
    float2* t = b0;
    b0 = b1;
    b1 = t;
    L *= r;
  }
  const float2 h = cscale(sp.het, sp.scale);
  for (int j = threadIdx.x; j < K; j += kSftThreads) {
    float2 v = cmul(b0[j], h);
    if (j & 1) v = make_float2(-v.x, -v.y);
    out[j] = v;
    if (valid) valid[seg * K + j] = 1;
  }
}

}  // namespace fstat
