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

// LDS layout of NL lines of length L: line-major with one pad element every
// 16 and an odd-ish pitch, addr(idx, line) = line * pitch + idx + idx / 16,
// pitch = L + L / 16 + 1.  Consecutive butterflies of a stage, consecutive
// elements of a line and the same element of consecutive lines all land in
// different LDS banks (the radix-R decimation stride R becomes R + R/16).
template <int L>
struct LdsLayout {
  static constexpr int pitch = L + L / 16 + 1;
  __device__ static __forceinline__ int at(int idx, int line) {
    return line * pitch + idx + (idx >> 4);
  }
};

// Butterfly of a Stockham stage with P > 1: twiddle W_{PR}^{jk} (table
// W_4096^{jk 4096/(PR)}), then the R-point DFT in registers.
template <int R, int P>
__device__ __forceinline__ void twiddle_dft(float2 (&v)[R], int k, const float2* __restrict__ tw) {
  if constexpr (P > 1) {
    constexpr int TWS = kTwLen / (P * R);
#pragma unroll
    for (int j = 1; j < R; ++j) v[j] = cmul(v[j], tw[j * k * TWS]);
  }
  dft<R>(v);
}

// A middle Stockham stage (LDS to LDS) over NL lines.  Butterfly b covers
// index i = b mod (L/R) of line b div (L/R); reads finish (barrier) before
// the in-place writes, which finish (barrier) before the next stage.
template <int LOGL, int NL, int NT, int S>
__device__ __forceinline__ void fft_stage(float2* buf, const float2* __restrict__ tw) {
  constexpr int LOGR = stage_logr(LOGL, S), R = 1 << LOGR;
  constexpr int P = 1 << stage_logp(LOGL, S);
  constexpr int L = 1 << LOGL;
  constexpr int NBL = L / R;
  constexpr int NB = NL * NBL;
  constexpr int PER = (NB + NT - 1) / NT;
  using Lay = LdsLayout<L>;
  const int tid = threadIdx.x;
  float2 v[PER][R];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if (NB % NT == 0 || b < NB) {
      const int i = b % NBL, line = b / NBL;
#pragma unroll
      for (int j = 0; j < R; ++j) v[s][j] = buf[Lay::at(i + j * NBL, line)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if (NB % NT == 0 || b < NB) {
      const int i = b % NBL, line = b / NBL;
      const int k = i & (P - 1);
      twiddle_dft<R, P>(v[s], k, tw);
      const int base = (i - k) * R + k;
#pragma unroll
      for (int m = 0; m < R; ++m) buf[Lay::at(base + m * P, line)] = v[s][m];
    }
  }
  __syncthreads();
}

// Middle stages 1 .. last-1.
template <int LOGL, int NL, int NT, int S>
__device__ __forceinline__ void fft_middle(float2* buf, const float2* __restrict__ tw) {
  if constexpr (S < stage_count(LOGL) - 1) {
    fft_stage<LOGL, NL, NT, S>(buf, tw);
    fft_middle<LOGL, NL, NT, S + 1>(buf, tw);
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
// zero padding and are not read.  The first Stockham stage reads its inputs
// straight from HBM and the last one writes its outputs, times the four-step
// twiddle W_N^{q c}, straight back (both with columns fastest across
// threads: NL-element contiguous runs); only the middle stages go through
// LDS.  Grid: (C / NL) x 2 arrays x template slots.
// GROUPED: the input is the unphased series of the slot's sky/orbit group;
// stage 0 applies the template's spin-down phase while loading and the
// output goes to the slot's own buffer.
template <int LOGL, int NL, int NT, bool GROUPED>
__global__ __launch_bounds__(NT) void k_fft_cols(PlanConst P, void* ws, ChunkMap map, int slots,
                                                 int arr_base, int log_c, int64_t rows_act) {
  extern __shared__ float2 lds[];
  constexpr int L = 1 << LOGL;
  constexpr int NS = stage_count(LOGL);
  constexpr int R0 = 1 << stage_logr(LOGL, 0), NB0 = NL * (L / R0);
  constexpr int RL = 1 << stage_logr(LOGL, NS - 1), PL = L / RL, NBL = NL * PL;
  using Lay = LdsLayout<L>;
  const uint32_t total = gridDim.x * gridDim.y * gridDim.z;
  const uint32_t id = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                total);
  const uint32_t gx = id % gridDim.x, rest = id / gridDim.x;
  const int arr = int(rest % gridDim.y), g = int(rest / gridDim.y);
  TmplParams* tpp = slot_params(ws, P, g);
  int32_t status = tpp->status;
  if (GROUPED) {
    const int32_t gs = *group_status(ws, P, slots, map.tmpl_buf[g]);
    if (gs != 0 && threadIdx.x == 0) atomicOr(&tpp->status, gs);
    status |= gs;
  }
  if (status != 0) return;
  const int64_t C = int64_t(1) << log_c;
  const int64_t c0 = int64_t(gx) * NL;
  float2* buf = slot_buf(ws, P, g, arr_base + arr);
  const float2* src =
      GROUPED ? group_buf(ws, P, slots, map.tmpl_buf[g], arr) : buf;
  const double f1dot = tpp->f1dot, f2dot = tpp->f2dot, df = tpp->df;
  const float2* __restrict__ tw = tw_stage(ws);
  const int tid = threadIdx.x;
  // stage 0: HBM -> registers -> DFT -> LDS
  {
    constexpr int PER = (NB0 + NT - 1) / NT;
    float2 v[PER][R0];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int b = tid + s * NT;
      if (NB0 % NT == 0 || b < NB0) {
        const int line = b % NL, i = b / NL;
#pragma unroll
        for (int j = 0; j < R0; ++j) {
          const int r = i + j * (L / R0);
          v[s][j] = r < rows_act ? src[int64_t(r) * C + c0 + line] : make_float2(0.f, 0.f);
        }
      }
    }
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int b = tid + s * NT;
      if (NB0 % NT == 0 || b < NB0) {
        const int line = b % NL, i = b / NL;
        if (GROUPED) {
#pragma unroll
          for (int j = 0; j < R0; ++j) {
            const int r = i + j * (L / R0);
            if (r < rows_act)
              v[s][j] = cmul_exact(
                  v[s][j], spindown_rotation(P, f1dot, f2dot, df, int64_t(r) * C + c0 + line));
          }
        }
        dft<R0>(v[s]);
#pragma unroll
        for (int m = 0; m < R0; ++m) lds[Lay::at(i * R0 + m, line)] = v[s][m];
      }
    }
  }
  __syncthreads();
  fft_middle<LOGL, NL, NT, 1>(lds, tw);
  // last stage: LDS -> registers -> DFT -> x W_N^{q c} -> HBM
  {
    constexpr int PER = (NBL + NT - 1) / NT;
    const int64_t nmask = P.n_fft - 1;
    const float2* __restrict__ wlo = tw_lo(ws);
    const float2* __restrict__ whi = tw_hi(ws);
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int b = tid + s * NT;
      if (NBL % NT == 0 || b < NBL) {
        const int line = b % NL, i = b / NL;
        float2 v[RL];
#pragma unroll
        for (int j = 0; j < RL; ++j) v[j] = lds[Lay::at(i + j * PL, line)];
        twiddle_dft<RL, PL>(v, i, tw);
        const int64_t c = c0 + line;
        // W_N^{c (i + m PL)} = W_N^{c i} (W_N^{c PL})^m
        const int64_t e0 = (int64_t(i) * c) & nmask, e1 = (int64_t(PL) * c) & nmask;
        float2 w = cmul(wlo[e0 & (kTwLen - 1)], whi[e0 >> 12]);
        const float2 step = cmul(wlo[e1 & (kTwLen - 1)], whi[e1 >> 12]);
#pragma unroll
        for (int m = 0; m < RL; ++m) {
          buf[int64_t(i + m * PL) * C + c] = cmul(v[m], w);
          w = cmul(w, step);
        }
      }
    }
  }
}

// Row pass with the 2F epilogue (eq. Fstat, normalised as 2F = 2 F^T M^-1 F,
// which is 2 (|Fa'|^2 + |Fb'|^2) for the whitened antenna patterns).  Lines
// 0..RQ-1 are rows q0..q0+RQ-1 of y_a', lines RQ..2RQ-1 the same rows of y_b';
// line length C = 2^LOGL.  The first stage reads the rows straight from HBM
// (contiguous across threads); the last stage transforms the a and b rows of
// the same bins in one thread and writes 2F (rows fastest across threads:
// RQ-element runs of the output).  Grid: (Rr / RQ) x templates.
// Row-pass epilogues: 2F (forward); the adjoint spectrum H = g conj(F') of
// both arrays at every natural FFT index m (zero outside the band), written to
// arrays 2 and 3 of the slot, with 2F if twoF is not null; or the complex
// transform itself, conjugated, written to arrays 0 and 1 at the natural
// index for indices below k_pad (the inverse transform of the adjoint).
enum RowMode { kRow2F = 0, kRowAdjoint = 1, kRowConj = 2 };

template <int LOGL, int RQ, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_fft_rows(PlanConst P, void* ws, ChunkMap map, int log_rr,
                                                 float* __restrict__ twoF, float2* fafb,
                                                 const float* __restrict__ gin) {
  extern __shared__ float2 lds[];
  constexpr int L = 1 << LOGL;
  constexpr int NL = 2 * RQ;
  constexpr int NS = stage_count(LOGL);
  constexpr int R0 = 1 << stage_logr(LOGL, 0), NBL0 = L / R0, NB0 = NL * NBL0;
  constexpr int RL = 1 << stage_logr(LOGL, NS - 1), PL = L / RL, NBL = RQ * PL;
  using Lay = LdsLayout<L>;
  const uint32_t total = gridDim.x * gridDim.y;
  const uint32_t id = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, total);
  const uint32_t gx = id % gridDim.x;
  const int g = int(id / gridDim.x);
  const TmplParams& tp = *slot_params(ws, P, g);
  const int64_t tmpl = map.tmpl[g];
  const int64_t q0 = int64_t(gx) * RQ;
  const int64_t Rr = int64_t(1) << log_rr;
  const int64_t N = P.n_fft;
  const int status = tp.status;
  const float2* __restrict__ tw = tw_stage(ws);
  const int tid = threadIdx.x;
  const float qnan = __builtin_nanf("");
  if (status != 0) {
    if (MODE == kRowConj) return;
    // flagged template: NaN in every bin it owns
    for (int e = tid; e < L * RQ; e += NT) {
      const int ql = e % RQ, p = e / RQ;
      const int64_t i = (q0 + ql + Rr * p + N / 2) & (N - 1);
      if (i < P.bin_lo || i >= P.bin_lo + P.n_bins) continue;
      const int64_t o = i - P.bin_lo;
      if (twoF) twoF[tmpl * P.n_bins + o] = qnan;
      if (fafb) {
        fafb[(tmpl * 2 + 0) * P.n_bins + o] = make_float2(qnan, qnan);
        fafb[(tmpl * 2 + 1) * P.n_bins + o] = make_float2(qnan, qnan);
      }
    }
    return;
  }
  // stage 0: HBM -> registers -> DFT -> LDS
  {
    const float2* ba = slot_buf(ws, P, g, MODE == kRowConj ? 2 : 0);
    const float2* bb = slot_buf(ws, P, g, MODE == kRowConj ? 3 : 1);
    constexpr int PER = (NB0 + NT - 1) / NT;
    float2 v[PER][R0];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int b = tid + s * NT;
      if (NB0 % NT == 0 || b < NB0) {
        const int i = b % NBL0, line = b / NBL0;
        const float2* src = (line < RQ ? ba : bb) + (q0 + line % RQ) * L;
#pragma unroll
        for (int j = 0; j < R0; ++j) v[s][j] = src[i + j * NBL0];
      }
    }
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int b = tid + s * NT;
      if (NB0 % NT == 0 || b < NB0) {
        const int i = b % NBL0, line = b / NBL0;
        dft<R0>(v[s]);
#pragma unroll
        for (int m = 0; m < R0; ++m) lds[Lay::at(i * R0 + m, line)] = v[s][m];
      }
    }
  }
  __syncthreads();
  fft_middle<LOGL, NL, NT, 1>(lds, tw);
  // last stage of both arrays + 2F
  const float l11 = tp.l11, l21 = tp.l21, l22 = tp.l22;
  constexpr int PER = (NBL + NT - 1) / NT;
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if (NBL % NT == 0 || b < NBL) {
      const int ql = b % RQ, i = b / RQ;
      float2 va[RL], vb[RL];
#pragma unroll
      for (int j = 0; j < RL; ++j) {
        va[j] = lds[Lay::at(i + j * PL, ql)];
        vb[j] = lds[Lay::at(i + j * PL, RQ + ql)];
      }
      twiddle_dft<RL, PL>(va, i, tw);
      twiddle_dft<RL, PL>(vb, i, tw);
#pragma unroll
      for (int m = 0; m < RL; ++m) {
        const int64_t nat = q0 + ql + Rr * int64_t(i + m * PL);
        if (MODE == kRowConj) {
          if (nat < P.k_pad) {
            slot_buf(ws, P, g, 0)[nat] = make_float2(va[m].x, -va[m].y);
            slot_buf(ws, P, g, 1)[nat] = make_float2(vb[m].x, -vb[m].y);
          }
          continue;
        }
        const int64_t ib = (nat + N / 2) & (N - 1);
        const bool in_band = ib >= P.bin_lo && ib < P.bin_lo + P.n_bins;
        const int64_t o = ib - P.bin_lo;
        const float2 fa = va[m], fb = vb[m];
        if (MODE == kRowAdjoint) {
          const float gv = in_band ? gin[tmpl * P.n_bins + o] : 0.0f;
          slot_buf(ws, P, g, 2)[nat] = make_float2(gv * fa.x, -gv * fa.y);
          slot_buf(ws, P, g, 3)[nat] = make_float2(gv * fb.x, -gv * fb.y);
        }
        if (!in_band) continue;
        if (twoF)
          twoF[tmpl * P.n_bins + o] =
              2.0f * ((fa.x * fa.x + fa.y * fa.y) + (fb.x * fb.x + fb.y * fb.y));
        if (fafb) {
          // undo the whitening: Fa = l11 Fa', Fb = l21 Fa' + l22 Fb'
          fafb[(tmpl * 2 + 0) * P.n_bins + o] = cscale(fa, l11);
          fafb[(tmpl * 2 + 1) * P.n_bins + o] =
              make_float2(l21 * fa.x + l22 * fb.x, l21 * fa.y + l22 * fb.y);
        }
      }
    }
  }
}

// Copy of the resampled series for the diagnostic entry point: y_a, y_b of
// slot g into out[t][2][n_fft], zero beyond the computed grid, with the
// whitening undone (y_a = l11 y_a', y_b = l21 y_a' + l22 y_b').
__global__ void k_copy_series(PlanConst P, void* ws, ChunkMap map, float2* out) {
  const int g = blockIdx.y;
  const TmplParams& tp = *slot_params(ws, P, g);
  const float2* sa = slot_buf(ws, P, g, 0);
  const float2* sb = slot_buf(ws, P, g, 1);
  float2* da = out + (map.tmpl[g] * 2 + 0) * P.n_fft;
  float2* db = out + (map.tmpl[g] * 2 + 1) * P.n_fft;
  const float l11 = tp.l11, l21 = tp.l21, l22 = tp.l22;
  const float qnan = __builtin_nanf("");
  const bool flagged = tp.status != 0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < P.n_fft;
       k += int64_t(gridDim.x) * blockDim.x) {
    float2 a = make_float2(0.f, 0.f), b = a;
    if (flagged) {
      a = b = make_float2(qnan, qnan);
    } else if (k < P.k_pad) {
      const float2 wa = sa[k], wb = sb[k];
      a = cscale(wa, l11);
      b = make_float2(l21 * wa.x + l22 * wb.x, l21 * wa.y + l22 * wb.y);
    }
    da[k] = a;
    db[k] = b;
  }
}

}  // namespace fstat
