// Step (vi) of Sec. 3 (forward DFT, negative exponent, no 1/N) as a
// two-pass four-step Stockham FFT, with step (vii) fused into the last pass.
//
// View the length-N series (N = Rr * C) as Rr rows of C: y[r C + c].
//   Column pass: for each column c, an Rr-point FFT over r, then the twiddle
//     W_N^{q c}; written back in place (each workgroup owns whole columns).
//   Row pass: for each row q, a C-point FFT over c gives X[q + Rr p].  The
//     same workgroup transforms rows of y_a' and y_b', so it holds Fa' and
//     Fb' of every bin it produces and writes 2F directly (ascending
//     frequency: output index (m + N/2) mod N).
// Inside a pass, lines are transformed in LDS by a mixed-radix Stockham
// autosort: every thread holds whole radix-R butterflies (R <= 16) in
// registers.  Twiddles come from FP32 tables written from FP64 once per call.
// The HBM traffic is one read and one write of the series per pass.
// Workgroups are remapped so that the ones an XCD runs together handle
// neighbouring columns (rows), whose partial cache lines then meet in that
// XCD's L2.
#pragma once

#include "fstat_common.hpp"

namespace fstat {

// cos(pi i / 8), sin(pi i / 8) for i = 0..7
__host__ __device__ constexpr float c16(int i) {
  return i == 0 ? 1.0f
         : i == 1 ? 0.92387953251128674f
         : i == 2 ? 0.70710678118654752f
         : i == 3 ? 0.38268343236508977f
         : i == 4 ? 0.0f
         : i == 5 ? -0.38268343236508977f
         : i == 6 ? -0.70710678118654752f
                  : -0.92387953251128674f;
}
__host__ __device__ constexpr float s16(int i) {
  return i == 0 ? 0.0f
         : i == 1 ? 0.38268343236508977f
         : i == 2 ? 0.70710678118654752f
         : i == 3 ? 0.92387953251128674f
         : i == 4 ? 1.0f
         : i == 5 ? 0.92387953251128674f
         : i == 6 ? 0.70710678118654752f
                  : 0.38268343236508977f;
}

// x * W_R^m, W_R = exp(-2 pi i / R), R <= 16, m < R/2
template <int R>
__device__ __forceinline__ float2 mul_wr(float2 x, int m) {
  const int i = 16 / R * m;
  if (i == 0) return x;
  if (i == 4) return make_float2(x.y, -x.x);
  const float c = c16(i), s = s16(i);
  return make_float2(x.x * c + x.y * s, x.y * c - x.x * s);
}

// In-register forward DFT of R points by radix-2 decimation in time.
template <int R>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
  if constexpr (R == 2) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R > 2) {
    constexpr int H = R / 2;
    float2 e[H], o[H];
#pragma unroll
    for (int m = 0; m < H; ++m) {
      e[m] = v[2 * m];
      o[m] = v[2 * m + 1];
    }
    dft<H>(e);
    dft<H>(o);
#pragma unroll
    for (int m = 0; m < H; ++m) {
      float2 t = mul_wr<R>(o[m], m);
      v[m] = cadd(e[m], t);
      v[m + H] = csub(e[m], t);
    }
  }
}

// Radix plan: log2 L split into ceil(log2 L / 4) stages as evenly as possible.
__host__ __device__ constexpr int stage_count(int logl) { return (logl + 3) / 4; }
__host__ __device__ constexpr int stage_logr(int logl, int s) {
  return s < logl % stage_count(logl) ? logl / stage_count(logl) + 1 : logl / stage_count(logl);
}
__host__ __device__ constexpr int stage_logp(int logl, int s) {
  return s == 0 ? 0 : stage_logp(logl, s - 1) + stage_logr(logl, s - 1);
}

// Workgroups are dispatched round-robin over the 8 XCDs: give the ones an
// XCD holds at the same time consecutive logical indices.
__device__ inline uint32_t xcd_remap(uint32_t id, uint32_t total) {
  const uint32_t full = total & ~7u;
  if (id >= full) return id;
  return (id & 7u) * (full >> 3) + (id >> 3);
}

// One Stockham stage over NL interleaved lines: element (idx, line) lives at
// buf[idx * NL + line].  Stage twiddle W_{PR}^{jk} = W_4096^{jk 4096/(PR)}.
template <int LOGL, int NL, int NT, int S>
__device__ __forceinline__ void fft_stage(float2* buf, const float2* __restrict__ tw) {
  constexpr int LOGR = stage_logr(LOGL, S), R = 1 << LOGR;
  constexpr int P = 1 << stage_logp(LOGL, S);
  constexpr int L = 1 << LOGL;
  constexpr int NB = NL * (L / R);
  constexpr int PER = (NB + NT - 1) / NT;
  constexpr int TWS = kTwLen / (P * R);
  const int tid = threadIdx.x;
  float2 v[PER][R];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if (NB % NT == 0 || b < NB) {
      const int line = b % NL, i = b / NL;
#pragma unroll
      for (int j = 0; j < R; ++j) v[s][j] = buf[(i + j * (L / R)) * NL + line];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if (NB % NT == 0 || b < NB) {
      const int line = b % NL, i = b / NL;
      const int k = i & (P - 1);
      if (P > 1) {
#pragma unroll
        for (int j = 1; j < R; ++j) v[s][j] = cmul(v[s][j], tw[j * k * TWS]);
      }
      dft<R>(v[s]);
      const int base = (i - k) * R + k;
#pragma unroll
      for (int m = 0; m < R; ++m) buf[(base + m * P) * NL + line] = v[s][m];
    }
  }
  __syncthreads();
}

template <int LOGL, int NL, int NT, int S>
__device__ __forceinline__ void fft_stages(float2* buf, const float2* __restrict__ tw) {
  if constexpr (S < stage_count(LOGL)) {
    fft_stage<LOGL, NL, NT, S>(buf, tw);
    fft_stages<LOGL, NL, NT, S + 1>(buf, tw);
  }
}

// FP32 twiddle tables from FP64 (see the workspace header layout).
__global__ void k_twiddles(void* ws, int64_t n_fft) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kTwLen) return;
  double s, c;
  sincospi(-2.0 * double(e) / double(kTwLen), &s, &c);
  tw_stage(ws)[e] = make_float2(float(c), float(s));
  sincospi(-2.0 * double(e) / double(n_fft), &s, &c);
  tw_lo(ws)[e] = make_float2(float(c), float(s));
  const int64_t eh = int64_t(e) * kTwLen;
  if (eh < n_fft) {
    sincospi(-2.0 * double(eh) / double(n_fft), &s, &c);
    tw_hi(ws)[e] = make_float2(float(c), float(s));
  }
}

// Column pass: lines are NL consecutive columns [c0, c0 + NL) of one array of
// one template slot; line length Rr = 2^LOGL.  Rows at or beyond rows_act are
// zero padding and are not read.  Grid: (C / NL) x 2 arrays x templates.
template <int LOGL, int NL, int NT>
__global__ __launch_bounds__(NT) void k_fft_cols(PlanConst P, void* ws, int log_c,
                                                 int64_t rows_act) {
  extern __shared__ float2 lds[];
  constexpr int L = 1 << LOGL;
  const uint32_t total = gridDim.x * gridDim.y * gridDim.z;
  const uint32_t id = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                total);
  const uint32_t gx = id % gridDim.x, rest = id / gridDim.x;
  const int arr = int(rest % gridDim.y), g = int(rest / gridDim.y);
  if (slot_params(ws, P.n_fft, g)->status != 0) return;
  const int64_t C = int64_t(1) << log_c;
  const int64_t c0 = int64_t(gx) * NL;
  float2* buf = slot_buf(ws, P.n_fft, g, arr);
  for (int e = threadIdx.x; e < L * NL; e += NT) {
    const int r = e / NL, line = e % NL;
    float2 v = make_float2(0.f, 0.f);
    if (r < rows_act) v = buf[int64_t(r) * C + c0 + line];
    lds[e] = v;
  }
  __syncthreads();
  fft_stages<LOGL, NL, NT, 0>(lds, tw_stage(ws));
  const int64_t nmask = P.n_fft - 1;
  const float2* __restrict__ wlo = tw_lo(ws);
  const float2* __restrict__ whi = tw_hi(ws);
  for (int e = threadIdx.x; e < L * NL; e += NT) {
    const int q = e / NL, line = e % NL;
    const int64_t c = c0 + line;
    const int64_t ex = (int64_t(q) * c) & nmask;
    const float2 w = cmul(wlo[ex & (kTwLen - 1)], whi[ex >> 12]);
    buf[int64_t(q) * C + c] = cmul(lds[e], w);
  }
}

// Row pass with the 2F epilogue (eq. Fstat, normalised as 2F = 2 F^T M^-1 F,
// which is 2 (|Fa'|^2 + |Fb'|^2) for the whitened antenna patterns).  Lines
// 0..RQ-1 are rows q0..q0+RQ-1 of y_a', lines RQ..2RQ-1 the same rows of y_b';
// line length C = 2^LOGL.  Grid: (Rr / RQ) x templates.
template <int LOGL, int RQ, int NT>
__global__ __launch_bounds__(NT) void k_fft_rows_2f(PlanConst P, void* ws, int log_rr,
                                                    float* __restrict__ twoF, float2* fafb,
                                                    int64_t t_first) {
  extern __shared__ float2 lds[];
  constexpr int L = 1 << LOGL;
  constexpr int NL = 2 * RQ;
  const uint32_t total = gridDim.x * gridDim.y;
  const uint32_t id = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, total);
  const uint32_t gx = id % gridDim.x;
  const int g = int(id / gridDim.x);
  const TmplParams& tp = *slot_params(ws, P.n_fft, g);
  const int64_t tmpl = t_first + g;
  const int64_t q0 = int64_t(gx) * RQ;
  const int64_t Rr = int64_t(1) << log_rr;
  const int64_t N = P.n_fft;
  const int status = tp.status;
  if (status == 0) {
    const float2* ba = slot_buf(ws, N, g, 0);
    const float2* bb = slot_buf(ws, N, g, 1);
    for (int e = threadIdx.x; e < L * NL; e += NT) {
      const int line = e / L, c = e % L;
      const int ql = line % RQ;
      const float2* src = line < RQ ? ba : bb;
      lds[c * NL + line] = src[(q0 + ql) * L + c];
    }
    __syncthreads();
    fft_stages<LOGL, NL, NT, 0>(lds, tw_stage(ws));
  }
  const float l11 = tp.l11, l21 = tp.l21, l22 = tp.l22;
  const float qnan = __builtin_nanf("");
  for (int e = threadIdx.x; e < L * RQ; e += NT) {
    const int ql = e % RQ, p = e / RQ;
    const int64_t m = q0 + ql + Rr * p;
    const int64_t i = (m + N / 2) & (N - 1);
    if (i < P.bin_lo || i >= P.bin_lo + P.n_bins) continue;
    const int64_t o = i - P.bin_lo;
    float2 fa = make_float2(qnan, qnan), fb = fa;
    float v = qnan;
    if (status == 0) {
      // whitened Fa', Fb': 2F = 2 (|Fa'|^2 + |Fb'|^2)
      fa = lds[p * NL + ql];
      fb = lds[p * NL + RQ + ql];
      v = 2.0f * ((fa.x * fa.x + fa.y * fa.y) + (fb.x * fb.x + fb.y * fb.y));
    }
    twoF[tmpl * P.n_bins + o] = v;
    if (fafb) {
      // undo the whitening: Fa = l11 Fa', Fb = l21 Fa' + l22 Fb'
      const float2 wa = fa, wb = fb;
      fa = cscale(wa, l11);
      fb = make_float2(l21 * wa.x + l22 * wb.x, l21 * wa.y + l22 * wb.y);
      fafb[(tmpl * 2 + 0) * P.n_bins + o] = fa;
      fafb[(tmpl * 2 + 1) * P.n_bins + o] = fb;
    }
  }
}

// Copy of the resampled series for the diagnostic entry point: y_a, y_b of
// slot g into out[t][2][n_fft], zero beyond the computed grid, with the
// whitening undone (y_a = l11 y_a', y_b = l21 y_a' + l22 y_b').
__global__ void k_copy_series(PlanConst P, void* ws, float2* out, int64_t t_first) {
  const int g = blockIdx.y;
  const TmplParams& tp = *slot_params(ws, P.n_fft, g);
  const float2* sa = slot_buf(ws, P.n_fft, g, 0);
  const float2* sb = slot_buf(ws, P.n_fft, g, 1);
  float2* da = out + ((t_first + g) * 2 + 0) * P.n_fft;
  float2* db = out + ((t_first + g) * 2 + 1) * P.n_fft;
  const float l11 = tp.l11, l21 = tp.l21, l22 = tp.l22;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < P.n_fft;
       k += int64_t(gridDim.x) * blockDim.x) {
    float2 a = make_float2(0.f, 0.f), b = a;
    if (k < P.k_pad) {
      const float2 wa = sa[k], wb = sb[k];
      a = cscale(wa, l11);
      b = make_float2(l21 * wa.x + l22 * wb.x, l21 * wa.y + l22 * wb.y);
    }
    da[k] = a;
    db[k] = b;
  }
}

}  // namespace fstat
