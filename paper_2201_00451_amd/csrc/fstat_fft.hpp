// Step (vi) of Sec. 3 (forward DFT, negative exponent, no 1/N) as a
// two-pass four-step Stockham FFT, with step (vii) fused into the last pass.
//
// View the length-N series (N = Rr * C) as Rr rows of C: y[r C + c].
//   Column pass: for each column c, an Rr-point FFT over r, then the twiddle
//     W_N^{q c}; written back in place (each workgroup owns whole columns).
//   Row pass: for each row q, a C-point FFT over c gives X[q + Rr p].  The
//     same workgroup transforms the rows of y_a' and y_b', so it holds Fa'
//     and Fb' of every bin it produces and writes 2F directly (ascending
//     frequency: output index (m + N/2) mod N).
// Inside a pass, lines are transformed in LDS by a mixed-radix Stockham
// autosort: every thread holds whole radix-R butterflies (R <= 32) in
// registers; the first stage reads HBM and the last one writes it.  Stage
// twiddles come from an FP32 table written from FP64 once per call and
// copied to LDS; the four-step twiddles from the exact quarter-turn split of
// their exponent and the rotation polynomials.  The HBM traffic is one read
// and one write of the series per pass.
#pragma once

#include "fstat_common.hpp"

namespace fstat {

// cos(pi i / 16), sin(pi i / 16) for i = 0..15 (32nd roots of unity)
__host__ __device__ constexpr float c32(int i) {
  constexpr float t[16] = {1.0f,
                           0.98078528040323044913f,
                           0.92387953251128675613f,
                           0.83146961230254523708f,
                           0.70710678118654752440f,
                           0.55557023301960222474f,
                           0.38268343236508977173f,
                           0.19509032201612826785f,
                           0.0f,
                           -0.19509032201612826785f,
                           -0.38268343236508977173f,
                           -0.55557023301960222474f,
                           -0.70710678118654752440f,
                           -0.83146961230254523708f,
                           -0.92387953251128675613f,
                           -0.98078528040323044913f};
  return t[i];
}
__host__ __device__ constexpr float s32(int i) { return i <= 8 ? c32(8 - i) : c32(i - 8); }

// x * W_R^m, W_R = exp(-2 pi i / R), R <= 32, m < R/2
template <int R>
__device__ __forceinline__ float2 mul_wr(float2 x, int m) {
  const int i = 32 / R * m;
  if (i == 0) return x;
  if (i == 8) return make_float2(x.y, -x.x);
  const float c = c32(i), s = s32(i);
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

// Radix plan: log2 L split into ceil(log2 L / MLR) stages as evenly as
// possible (radix at most 2^MLR, MLR = 4 or 5).
__host__ __device__ constexpr int stage_count(int logl, int mlr) { return (logl + mlr - 1) / mlr; }
__host__ __device__ constexpr int stage_logr(int logl, int s, int mlr) {
  return s < logl % stage_count(logl, mlr) ? logl / stage_count(logl, mlr) + 1
                                            : logl / stage_count(logl, mlr);
}
__host__ __device__ constexpr int stage_logp(int logl, int s, int mlr) {
  return s == 0 ? 0 : stage_logp(logl, s - 1, mlr) + stage_logr(logl, s - 1, mlr);
}

// Workgroups are dispatched round-robin over the 8 XCDs: give the ones an
// XCD holds at the same time consecutive logical indices.
__device__ inline uint32_t xcd_remap(uint32_t id, uint32_t total) {
  const uint32_t full = total & ~7u;
  if (id >= full) return id;
  return (id & 7u) * (full >> 3) + (id >> 3);
}

// LDS layout of lines of length L: line-major, one pad element after every
// PAD elements of a line, addr(idx, line) = line * pitch + idx + idx / PAD.
// PAD is the first stage's radix R0, whose butterflies write idx = R0 i + m
// across lanes: the pad turns that stride into R0 + 1, an odd number of bank
// pairs.  The stages that face HBM run F lines fastest across lanes (F
// lines times 16 / F consecutive butterflies in every 16 lanes); the pitch is
// L + L / PAD rounded up to 16 / F modulo 16 (to 1 if F >= 16), so those 16
// lanes touch 16 different 8-byte bank pairs.  The middle stages run one
// line's butterflies across lanes.
template <int L, int PAD, int F>
struct LdsLayout {
  static constexpr int kBank = F >= 16 ? 1 : 16 / F;
  static constexpr int kBase = L + L / PAD;
  static constexpr int pitch = kBase + ((kBank - kBase % 16) % 16 + 16) % 16;
  __device__ static __forceinline__ int at(int idx, int line) {
    return line * pitch + idx + idx / PAD;
  }
  // at(i + j STEP, line) for STEP a multiple of PAD: the pad of the strided
  // part is a constant stride, so the unrolled accesses of one thread differ
  // by compile-time offsets (one address register per butterfly)
  template <int STEP>
  __device__ static __forceinline__ int at_step(int i, int j, int line) {
    static_assert(STEP % PAD == 0, "stride must be a multiple of the pad period");
    return line * pitch + i + i / PAD + j * (STEP + STEP / PAD);
  }
  // at(i PAD + m, line) for m < PAD (a first-stage butterfly's outputs)
  __device__ static __forceinline__ int at_block(int i, int m, int line) {
    return line * pitch + i * (PAD + 1) + m;
  }
};
// Bytes of LDS of a pass: NL padded lines and the half twiddle table.
template <int L, int PAD, int F, int NL>
constexpr size_t kLdsBytes = (size_t(NL) * LdsLayout<L, PAD, F>::pitch + size_t(L / 2)) *
                             sizeof(float2);

// W_L^e from the LDS half table T[e] = W_L^e, e < L/2 (W_L^{e+L/2} = -W_L^e).
template <int L>
__device__ __forceinline__ float2 tw_half(const float2* twl, int e) {
  const float2 w = twl[e & (L / 2 - 1)];
  return e < L / 2 ? w : make_float2(-w.x, -w.y);
}

// Butterfly of a Stockham stage with P > 1: twiddle W_{PR}^{jk} = W_L^{jk L/(PR)},
// then the R-point DFT in registers.
template <int R, int P, int L>
__device__ __forceinline__ void twiddle_dft(float2 (&v)[R], int k, const float2* twl) {
  if constexpr (P > 1) {
    constexpr int TWS = L / (P * R);
#pragma unroll
    for (int j = 1; j < R; ++j) v[j] = cmul(v[j], tw_half<L>(twl, j * k * TWS));
  }
  dft<R>(v);
}

// A middle Stockham stage (LDS to LDS) over NL lines.  Butterfly b covers
// index i = b mod (L/R) of line b div (L/R); reads finish (barrier) before
// the in-place writes, which finish (barrier) before the next stage.
template <int LOGL, int NL, int NT, int S, int MLR, class Lay>
__device__ __forceinline__ void fft_stage(float2* buf, const float2* twl, int tid) {
  constexpr int LOGR = stage_logr(LOGL, S, MLR), R = 1 << LOGR;
  constexpr int P = 1 << stage_logp(LOGL, S, MLR);
  constexpr int L = 1 << LOGL;
  constexpr int NBL = L / R;
  constexpr int NB = NL * NBL;
  constexpr int PER = (NB + NT - 1) / NT;
  float2 v[PER][R];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if (NB % NT == 0 || b < NB) {
      const int i = b % NBL, line = b / NBL;
#pragma unroll
      for (int j = 0; j < R; ++j) v[s][j] = buf[Lay::template at_step<NBL>(i, j, line)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if (NB % NT == 0 || b < NB) {
      const int i = b % NBL, line = b / NBL;
      const int k = i & (P - 1);
      twiddle_dft<R, P, L>(v[s], k, twl);
      const int base = (i - k) * R + k;
#pragma unroll
      for (int m = 0; m < R; ++m) buf[Lay::template at_step<P>(base, m, line)] = v[s][m];
    }
  }
  __syncthreads();
}

// Middle stages 1 .. last-1.
template <int LOGL, int NL, int NT, int S, int MLR, class Lay>
__device__ __forceinline__ void fft_middle(float2* buf, const float2* twl, int tid) {
  if constexpr (S < stage_count(LOGL, MLR) - 1) {
    fft_stage<LOGL, NL, NT, S, MLR, Lay>(buf, twl, tid);
    fft_middle<LOGL, NL, NT, S + 1, MLR, Lay>(buf, twl, tid);
  }
}

// FP32 stage twiddle table W_4096^e from FP64, written at the start of every
// call; each FFT workgroup copies the W_L^e, e < L/2, it needs into LDS.
// It also clears the call's flagged-template counter.
__global__ void k_twiddles(void* ws) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) *flag_counter(ws) = 0ull;
  if (e >= kTwLen) return;
  double s, c;
  sincospi(-2.0 * double(e) / double(kTwLen), &s, &c);
  tw_stage(ws)[e] = make_float2(float(c), float(s));
}

// W_N^e for 0 <= e < N <= 2^24.
__device__ __forceinline__ float2 tw_n(int64_t e, int64_t n_fft) {
  return cis_neg_frac(e, __builtin_ctzll(uint64_t(n_fft)));
}

template <int LOGL, int MLR>
constexpr int kR0 = 1 << stage_logr(LOGL, 0, MLR);
template <int LOGL, int NL, int NT, int MLR>
constexpr int kPer0 = (NL * ((1 << LOGL) / kR0<LOGL, MLR>) + NT - 1) / NT;

// Work items: one workgroup per item, line groups fastest within a
// template, and the block index remapped so that the workgroups an XCD runs
// together take neighbouring line groups (the row pass writes 2F in runs of
// RQ floats per row group; neighbouring groups complete each other's cache
// lines in that XCD's L2 before write-back).

struct ColItem {
  int live, g, arr;
  int64_t cg;  // column group: columns cg * NL .. cg * NL + NL - 1
  double sd[4];
};

// Column pass: lines are NL consecutive columns [c0, c0 + NL) of one array of
// one template slot; line length Rr = 2^LOGL.  Rows at or beyond rows_act
// are zero padding and are not read.  The first Stockham stage reads its
// inputs straight from HBM and the last one writes its outputs, times the
// four-step twiddle W_N^{q c}, straight back (both with columns fastest
// across threads: NL-element contiguous runs); only the middle stages go
// through LDS.  Items: (C / NL column groups) x 2 arrays x template slots.
// GROUPED: the input is the unphased series of the slot's sky/orbit group;
// stage 0 applies the template's spin-down phase while loading and the
// output goes to the slot's own buffer.
//
// Item description (status, columns, array, spin-down coefficients).
template <bool GROUPED>
__device__ __forceinline__ ColItem cols_item(const PlanConst& P, void* ws, const ChunkMap& map,
                                             int slots, int n_gx, int item) {
  ColItem it;
  it.live = 0;
  it.cg = int64_t(item % n_gx);
  const int rest = item / n_gx;
  it.arr = rest & 1;
  it.g = rest >> 1;
  TmplParams* tpp = tmpl_params(ws, P, map, it.g);
  int32_t status = tpp->status;
  if (GROUPED) {
    const int32_t gs = *group_status(ws, P, slots, map.tmpl_buf[it.g]);
    if (gs != 0 && threadIdx.x == 0) atomicOr(&tpp->status, gs);
    status |= gs;
  }
  if (status != 0) return it;
  it.live = 1;
#pragma unroll
  for (int q = 0; q < 4; ++q) it.sd[q] = tpp->sd[q];
  return it;
}

// The item's first-stage inputs into registers (buffer loads; rows at or
// beyond rows_act lie past the descriptor's end and read as zero).
template <int LOGL, int NL, int NT, bool GROUPED, int MLR>
__device__ __forceinline__ void cols_load(const PlanConst& P, void* ws, const ChunkMap& map,
                                          int slots, int arr_base, int64_t C, int64_t rows_act,
                                          const ColItem& it,
                                          float2 (&v)[kPer0<LOGL, NL, NT, MLR>]
                                                     [kR0<LOGL, MLR>]) {
  constexpr int L = 1 << LOGL;
  constexpr int R0 = kR0<LOGL, MLR>, NB0 = NL * (L / R0);
  constexpr int PER = kPer0<LOGL, NL, NT, MLR>;
  const float2* src = GROUPED ? group_buf(ws, P, slots, map.tmpl_buf[it.g], it.arr)
                              : slot_buf(ws, P, it.g, arr_base + it.arr);
  const auto rs = buf_rsrc(src, uint32_t(rows_act * C * int64_t(sizeof(float2))));
  const int tid = threadIdx.x;
  const int64_t c0 = it.cg * NL;
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if (NB0 % NT == 0 || b < NB0) {
      const int line = b % NL, i = b / NL;
      const uint32_t voff = uint32_t((int64_t(i) * C + c0 + line) * int64_t(sizeof(float2)));
#pragma unroll
      for (int j = 0; j < R0; ++j)
        v[s][j] = buf_load2(rs, voff, uint32_t(int64_t(j) * (L / R0) * C * int64_t(sizeof(float2))));
    }
  }
}

// Stage 0: registers -> (spin-down phase-in) -> DFT -> LDS.
template <int LOGL, int NL, int NT, bool GROUPED, int MLR>
__device__ __forceinline__ void cols_stage0(const ColItem& it, int64_t C, int64_t rows_act,
                                            float2 (&v)[kPer0<LOGL, NL, NT, MLR>]
                                                       [kR0<LOGL, MLR>],
                                            float2* lds, int tid) {
  constexpr int L = 1 << LOGL;
  constexpr int R0 = kR0<LOGL, MLR>, NB0 = NL * (L / R0);
  constexpr int PER0 = kPer0<LOGL, NL, NT, MLR>;
  using Lay = LdsLayout<L, R0, NL>;
  const int64_t c0 = it.cg * NL;
#pragma unroll
  for (int s = 0; s < PER0; ++s) {
    const int b = tid + s * NT;
    if (NB0 % NT == 0 || b < NB0) {
      const int line = b % NL, i = b / NL;
      if (GROUPED) {
#pragma unroll
        for (int j = 0; j < R0; ++j) {
          const int r = i + j * (L / R0);
          if (r < rows_act)
            v[s][j] = cmul_exact(v[s][j], spindown_rotation(it.sd, int64_t(r) * C + c0 + line));
        }
      }
      dft<R0>(v[s]);
#pragma unroll
      for (int m = 0; m < R0; ++m) lds[Lay::at_block(i, m, line)] = v[s][m];
    }
  }
}

// Middle stages in LDS, then the last stage: LDS -> DFT -> x W_N^{q c} -> HBM.
// The line's outputs k go to rows q = QS k + h (QS = 2: one half of a column
// split in two, see k_fft_cols_half).
template <int LOGL, int NL, int NT, int MLR, int QS = 1>
__device__ __forceinline__ void cols_finish(const PlanConst& P, void* ws, int arr_base,
                                            int64_t C, const ColItem& it, float2* lds,
                                            const float2* twl, int tid, int h = 0) {
  constexpr int L = 1 << LOGL;
  constexpr int NS = stage_count(LOGL, MLR);
  constexpr int R0 = kR0<LOGL, MLR>;
  constexpr int RL = 1 << stage_logr(LOGL, NS - 1, MLR), PL = L / RL, NBL = NL * PL;
  using Lay = LdsLayout<L, R0, NL>;
  fft_middle<LOGL, NL, NT, 1, MLR, Lay>(lds, twl, tid);
  const int64_t nmask = P.n_fft - 1;
  const int64_t c0 = it.cg * NL;
  const auto wr = buf_rsrc(slot_buf(ws, P, it.g, arr_base + it.arr),
                           uint32_t(P.n_fft * int64_t(sizeof(float2))));
  constexpr int PER = (NBL + NT - 1) / NT;
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if (NBL % NT == 0 || b < NBL) {
      const int line = b % NL, i = b / NL;
      float2 u[RL];
#pragma unroll
      for (int j = 0; j < RL; ++j) u[j] = lds[Lay::template at_step<PL>(i, j, line)];
      twiddle_dft<RL, PL, L>(u, i, twl);
      const int64_t c = c0 + line;
      // row q = QS (i + m PL) + h: W_N^{c q} = W_N^{c q0} (W_N^{c QS PL})^m
      const int64_t q0 = int64_t(QS) * i + h;
      float2 w = tw_n((q0 * c) & nmask, P.n_fft);
      const float2 step = tw_n((int64_t(QS) * PL * c) & nmask, P.n_fft);
      const uint32_t voff = uint32_t((q0 * C + c) * int64_t(sizeof(float2)));
#pragma unroll
      for (int m = 0; m < RL; ++m) {
        buf_store2(cmul(u[m], w), wr, voff,
                   uint32_t(int64_t(m) * QS * PL * C * int64_t(sizeof(float2))));
        w = cmul(w, step);
      }
    }
  }
}

template <int LOGL, int NL, int NT, bool GROUPED, int MLR>
__global__ __launch_bounds__(NT) void k_fft_cols(PlanConst P, void* ws, ChunkMap map, int slots,
                                                 int arr_base, int log_c, int64_t rows_act) {
  extern __shared__ float2 lds[];
  constexpr int L = 1 << LOGL;
  constexpr int R0 = kR0<LOGL, MLR>;
  constexpr int PER0 = kPer0<LOGL, NL, NT, MLR>;
  using Lay = LdsLayout<L, R0, NL>;
  float2* twl = lds + NL * Lay::pitch;
  const int tid = threadIdx.x;
  const int64_t C = int64_t(1) << log_c;
  {
    const float2* __restrict__ tws = tw_stage(ws);
    for (int e = tid; e < L / 2; e += NT) twl[e] = tws[e * (kTwLen / L)];
  }
  float2 v[PER0][R0];
  const ColItem it = cols_item<GROUPED>(P, ws, map, slots, int(C / NL),
                                        int(xcd_remap(blockIdx.x, gridDim.x)));
  if (!it.live) return;
  cols_load<LOGL, NL, NT, GROUPED, MLR>(P, ws, map, slots, arr_base, C, rows_act, it, v);
  cols_stage0<LOGL, NL, NT, GROUPED, MLR>(it, C, rows_act, v, lds, tid);
  __syncthreads();
  cols_finish<LOGL, NL, NT, MLR>(P, ws, arr_base, C, it, lds, twl, tid);
}

// The column pass for long columns in half the LDS.  With H = L/2 and
// y_h[r] = (x[r] + (-1)^h x[r + H]) W_L^{r h}, r < H, rows 2k + h of the
// column's transform are the H-point transform of y_h (one radix-2 step of
// decimation in frequency).  Each thread loads x[r] and x[r + H] of its
// first-stage butterflies and combines them in registers; y_0 goes through
// the LDS stages while y_1 waits in registers, then y_1 follows.  Half the
// LDS lets two workgroups share a compute unit, so that one's loads and
// stores overlap the other's transform.
template <int LOGL, int NL, int NT, bool GROUPED, int MLR>
__global__ __launch_bounds__(NT, NT / 128) void k_fft_cols_half(PlanConst P, void* ws, ChunkMap map,
                                                         int slots, int arr_base, int log_c,
                                                         int64_t rows_act) {
  extern __shared__ float2 lds[];
  constexpr int LH = LOGL - 1;
  constexpr int L = 1 << LOGL, H = L / 2;
  constexpr int R0 = kR0<LH, MLR>, S0 = H / R0, NB0 = NL * S0;
  constexpr int PER0 = kPer0<LH, NL, NT, MLR>;
  using Lay = LdsLayout<H, R0, NL>;
  float2* twl = lds + NL * Lay::pitch;
  const int tid = threadIdx.x;
  const int64_t C = int64_t(1) << log_c;
  const float2* __restrict__ tws = tw_stage(ws);
  for (int e = tid; e < H / 2; e += NT) twl[e] = tws[e * (kTwLen / H)];
  const ColItem it = cols_item<GROUPED>(P, ws, map, slots, int(C / NL),
                                        int(xcd_remap(blockIdx.x, gridDim.x)));
  if (!it.live) return;
  const int64_t c0 = it.cg * NL;
  float2 a[PER0][R0], b[PER0][R0];
  {
    const float2* src = GROUPED ? group_buf(ws, P, slots, map.tmpl_buf[it.g], it.arr)
                                : slot_buf(ws, P, it.g, arr_base + it.arr);
    const auto rs = buf_rsrc(src, uint32_t(rows_act * C * int64_t(sizeof(float2))));
#pragma unroll
    for (int s = 0; s < PER0; ++s) {
      const int bb = tid + s * NT;
      if (NB0 % NT == 0 || bb < NB0) {
        const int line = bb % NL, i = bb / NL;
        const uint32_t voff = uint32_t((int64_t(i) * C + c0 + line) * int64_t(sizeof(float2)));
#pragma unroll
        for (int j = 0; j < R0; ++j) {
          a[s][j] = buf_load2(rs, voff, uint32_t(int64_t(j) * S0 * C * int64_t(sizeof(float2))));
          b[s][j] = buf_load2(rs, voff,
                              uint32_t((int64_t(j) * S0 + H) * C * int64_t(sizeof(float2))));
        }
      }
    }
  }
  // spin-down phase (search path), the radix-2 step and y_1's twiddle W_L^r
#pragma unroll
  for (int s = 0; s < PER0; ++s) {
    const int bb = tid + s * NT;
    if (NB0 % NT == 0 || bb < NB0) {
      const int line = bb % NL, i = bb / NL;
#pragma unroll
      for (int j = 0; j < R0; ++j) {
        const int r = i + j * S0;
        if (GROUPED) {
          if (r < rows_act)
            a[s][j] = cmul_exact(a[s][j], spindown_rotation(it.sd, int64_t(r) * C + c0 + line));
          if (r + H < rows_act)
            b[s][j] = cmul_exact(b[s][j],
                                 spindown_rotation(it.sd, int64_t(r + H) * C + c0 + line));
        }
        const float2 d = csub(a[s][j], b[s][j]);
        a[s][j] = cadd(a[s][j], b[s][j]);
        b[s][j] = cmul(d, tws[r * (kTwLen / L)]);
      }
    }
  }
  // y_0: first stage into LDS, the other stages, rows 2k; then y_1, rows 2k + 1
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int s = 0; s < PER0; ++s) {
      const int bb = tid + s * NT;
      if (NB0 % NT == 0 || bb < NB0) {
        const int line = bb % NL, i = bb / NL;
        float2(&v)[R0] = h ? b[s] : a[s];
        dft<R0>(v);
#pragma unroll
        for (int m = 0; m < R0; ++m) lds[Lay::at_block(i, m, line)] = v[m];
      }
    }
    __syncthreads();
    cols_finish<LH, NL, NT, MLR, 2>(P, ws, arr_base, C, it, lds, twl, tid, h);
    // the last stage has read the lines before y_1's first stage writes them
    if (h == 0) __syncthreads();
  }
}

// Row pass with the 2F epilogue (eq. Fstat, normalised as 2F = 2 F^T M^-1 F,
// which is 2 (|Fa'|^2 + |Fb'|^2) for the whitened antenna patterns).  An item
// is RQ rows q0..q0+RQ-1 of both y_a' and y_b' (line length C = 2^LOGL); the
// first stage reads the rows straight from HBM (contiguous across threads),
// the last stage leaves the a and b values of the same bins in one thread,
// which writes 2F (rows fastest across threads: RQ-element runs of the
// output).  Items: (Rr / RQ) row groups x template slots.
// Row-pass epilogues: 2F (forward); the adjoint spectrum H = g conj(F') of
// both arrays at every natural FFT index m (zero outside the band), written to
// arrays 2 and 3 of the slot, with 2F if twoF is not null; or the complex
// transform itself, conjugated, written to arrays 0 and 1 at the natural
// index for indices below k_pad (the inverse transform of the adjoint).
// kRow2F stores 2F only (the plain full-band output); kRow2FExt is the same
// transform with every optional output of RowOutput (Fa/Fb, accumulation,
// candidates, loudest bin).
// Row epilogues: plain 2F stores; the adjoint's two; the extended forward one
// (Fa/Fb, accumulation, candidates, loudest bin); candidates and loudest bin
// only (no 2F array).
enum RowMode { kRow2F = 0, kRowAdjoint = 1, kRowConj = 2, kRow2FExt = 3, kRowCand = 4 };

// 2F = 2 (|Fa'|^2 + |Fb'|^2) with explicit FMA, so that every epilogue gives
// the same bits.
__device__ __forceinline__ float two_f(float2 fa, float2 fb) {
  return 2.0f * (fmaf(fa.x, fa.x, fa.y * fa.y) + fmaf(fb.x, fb.x, fb.y * fb.y));
}

struct RowItem {
  int live, flagged, g;
  int64_t q0, tmpl;
  float l11, l21, l22;
};

// A bin above the threshold joins the candidate list (slots past the
// capacity are counted, not stored).
__device__ __forceinline__ void keep_candidate(const RowOutput& out, int64_t tmpl, int64_t o,
                                               float v2) {
  if (out.cand && v2 > out.threshold) {
    const unsigned long long idx = atomicAdd(out.count, 1ull);
    if (idx < (unsigned long long)out.cap)
      out.cand[idx] = fstat_candidate{int32_t(tmpl), int32_t(o), v2, 0};
  }
}
// Loudest-bin key: 2F's bits (2F >= 0, so unsigned order is float order)
// above the band offset, so the largest key is the loudest bin and equal 2F
// resolve to the highest bin.
__device__ __forceinline__ unsigned long long best_key(float v2, int64_t o) {
  return (static_cast<unsigned long long>(__float_as_uint(v2)) << 32) |
         static_cast<unsigned long long>(o);
}
// The workgroup's keys into the template's entry: wavefront maximum, one
// atomic per wave, and none where the entry already holds as much (it only
// grows, so a smaller key can never be the maximum; every row item of a
// template would otherwise contend for the one address).
__device__ __forceinline__ void best_to_global(const RowOutput& out, int64_t tmpl,
                                               unsigned long long key) {
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_down(key, off, 64);
    key = o > key ? o : key;
  }
  if ((threadIdx.x & 63) == 0 && key != 0ull) {
    const unsigned long long cur =
        __hip_atomic_load(out.best + tmpl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (key > cur) atomicMax(out.best + tmpl, key);
  }
}

template <int MODE>
__device__ __forceinline__ RowItem rows_item(const PlanConst& P, void* ws, const ChunkMap& map,
                                             int item, int n_gx, int RQ) {
  RowItem it;
  it.live = it.flagged = 0;
  it.q0 = int64_t(item % n_gx) * RQ;
  it.g = item / n_gx;
  it.tmpl = map.tmpl[it.g];
  const TmplParams& tp = *tmpl_params(ws, P, map, it.g);
  if (tp.status != 0) {
    it.flagged = 1;
    return it;
  }
  it.live = 1;
  it.l11 = tp.l11;
  it.l21 = tp.l21;
  it.l22 = tp.l22;
  return it;
}

// First-stage inputs of butterflies s = S0 .. S0 + NSB - 1 (b = tid + s NT;
// line b / (L / R0): lines 0..RQ-1 are the a rows, RQ..2RQ-1 the b rows).
template <int LOGL, int RQ, int NT, int MODE, int MLR, int S0, int NSB>
__device__ __forceinline__ void rows_load(const PlanConst& P, void* ws, const RowItem& it,
                                          float2 (&v)[NSB][kR0<LOGL, MLR>]) {
  constexpr int L = 1 << LOGL;
  constexpr int NL = 2 * RQ;
  constexpr int R0 = kR0<LOGL, MLR>, NBL0 = L / R0, NB0 = NL * NBL0;
  // arrays a and b of the slot are adjacent: one descriptor covers both
  const auto rs = buf_rsrc(slot_buf(ws, P, it.g, MODE == kRowConj ? 2 : 0),
                           uint32_t(2 * P.n_fft * int64_t(sizeof(float2))));
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < NSB; ++s) {
    const int b = tid + (S0 + s) * NT;
    if (NB0 % NT == 0 || b < NB0) {
      const int i = b % NBL0, line = b / NBL0;
      const int64_t e0 = (line < RQ ? 0 : P.n_fft) + (it.q0 + line % RQ) * L + i;
      const uint32_t voff = uint32_t(e0 * int64_t(sizeof(float2)));
      // streaming reads pay off with the plain 2F epilogue (its partial 2F
      // lines stay in L2); with the extended epilogue they cost 2 % (measured)
#pragma unroll
      for (int j = 0; j < R0; ++j) {
        const uint32_t soff = uint32_t(j * NBL0 * int(sizeof(float2)));
        v[s][j] = MODE == kRow2F ? buf_load2_stream(rs, voff, soff) : buf_load2(rs, voff, soff);
      }
    }
  }
}

// The row epilogue for one output element: natural index nat, a and b
// values.  Returns 2F of an in-band bin (-1 otherwise) for the caller's
// running maximum.
template <int MODE>
__device__ __forceinline__ float rows_out(const PlanConst& P, void* ws, const RowItem& it,
                                          int64_t nat, float2 fa, float2 fb,
                                          const RowOutput& out) {
  const int64_t N = P.n_fft;
  if (MODE == kRowConj) {
    if (nat < P.k_pad) {
      slot_buf(ws, P, it.g, 0)[nat] = make_float2(fa.x, -fa.y);
      slot_buf(ws, P, it.g, 1)[nat] = make_float2(fb.x, -fb.y);
    }
    return -1.0f;
  }
  const int64_t ib = (nat + N / 2) & (N - 1);
  const bool in_band = ib >= P.bin_lo && ib < P.bin_lo + P.n_bins;
  const int64_t o = ib - P.bin_lo;
  if (MODE == kRowAdjoint) {
    const float gv = in_band ? out.gin[it.tmpl * P.n_bins + o] : 0.0f;
    slot_buf(ws, P, it.g, 2)[nat] = make_float2(gv * fa.x, -gv * fa.y);
    slot_buf(ws, P, it.g, 3)[nat] = make_float2(gv * fb.x, -gv * fb.y);
  }
  if (!in_band) return -1.0f;
  const float v2 = two_f(fa, fb);
  if (out.twoF) {
    float* dst = out.twoF + it.tmpl * P.n_bins + o;
    *dst = out.acc ? *dst + v2 : v2;
  }
  if (out.fafb) {
    // undo the whitening: Fa = l11 Fa', Fb = l21 Fa' + l22 Fb'
    out.fafb[(it.tmpl * 2 + 0) * P.n_bins + o] = cscale(fa, it.l11);
    out.fafb[(it.tmpl * 2 + 1) * P.n_bins + o] =
        make_float2(it.l21 * fa.x + it.l22 * fb.x, it.l21 * fa.y + it.l22 * fb.y);
  }
  keep_candidate(out, it.tmpl, o, v2);
  return v2;
}

// A flagged template: NaN in every bin the item owns (and the all-ones
// marker in its best entry); the template's first row group counts it.
template <int LOGL, int RQ, int NT>
__device__ __forceinline__ void rows_flagged(const PlanConst& P, void* ws, const RowItem& it,
                                             int64_t Rr, const RowOutput& out) {
  constexpr int L = 1 << LOGL;
  const int64_t N = P.n_fft;
  const float qnan = __builtin_nanf("");
  if (it.q0 == 0 && threadIdx.x == 0) atomicAdd(flag_counter(ws), 1ull);
  if (out.best && threadIdx.x == 0) atomicMax(out.best + it.tmpl, ~0ull);
  for (int e = threadIdx.x; e < L * RQ; e += NT) {
    const int ql = e % RQ, p = e / RQ;
    const int64_t i = (it.q0 + ql + Rr * p + N / 2) & (N - 1);
    if (i < P.bin_lo || i >= P.bin_lo + P.n_bins) continue;
    const int64_t o = i - P.bin_lo;
    if (out.twoF) out.twoF[it.tmpl * P.n_bins + o] = qnan;
    if (out.fafb) {
      out.fafb[(it.tmpl * 2 + 0) * P.n_bins + o] = make_float2(qnan, qnan);
      out.fafb[(it.tmpl * 2 + 1) * P.n_bins + o] = make_float2(qnan, qnan);
    }
  }
}

// Stage 0 of both arrays (registers -> DFT -> LDS).
template <int LOGL, int RQ, int NT, int MLR, int NL>
__device__ __forceinline__ void rows_stage0(float2* lds, int tid,
                                            float2 (&v)[kPer0<LOGL, NL, NT, MLR>]
                                                       [kR0<LOGL, MLR>]) {
  constexpr int L = 1 << LOGL;
  constexpr int R0 = kR0<LOGL, MLR>, NBL0 = L / R0;
  constexpr int PER0 = kPer0<LOGL, NL, NT, MLR>;
  using Lay = LdsLayout<L, R0, RQ>;
#pragma unroll
  for (int s = 0; s < PER0; ++s) {
    const int b = tid + s * NT;
    if ((NL * NBL0) % NT == 0 || b < NL * NBL0) {
      const int i = b % NBL0, line = b / NBL0;
      dft<R0>(v[s]);
#pragma unroll
      for (int m = 0; m < R0; ++m) lds[Lay::at_block(i, m, line)] = v[s][m];
    }
  }
}

// Middle stages, then the last stage of both arrays and the epilogue.  The
// line's outputs k are the row transform's entries p = QS k + h (QS = 2: one
// half of a row split in two, see k_fft_rows_half).
template <int LOGL, int RQ, int NT, int MODE, int MLR, int QS = 1>
__device__ __forceinline__ void rows_finish(const PlanConst& P, void* ws, const RowItem& it,
                                            const RowOutput& out, int64_t Rr, float2* lds,
                                            const float2* twl, int tid, int h = 0) {
  constexpr int L = 1 << LOGL;
  constexpr int NL = 2 * RQ;
  constexpr int NS = stage_count(LOGL, MLR);
  constexpr int R0 = kR0<LOGL, MLR>;
  constexpr int RL = 1 << stage_logr(LOGL, NS - 1, MLR), PL = L / RL, NBL = RQ * PL;
  constexpr int PER = (NBL + NT - 1) / NT;
  using Lay = LdsLayout<L, R0, RQ>;
  fft_middle<LOGL, NL, NT, 1, MLR, Lay>(lds, twl, tid);
  unsigned long long bkey = 0ull;
  float pa[MODE == kRowCand ? PER : 1][MODE == kRowCand ? RL : 1];
  // plain 2F: band offsets o = ((nat + N/2) mod N) - bin_lo in 32 bits; the
  // descriptor spans this template's n_bins floats, so the store of a bin
  // outside the band (o >= n_bins, also when the subtraction wraps) is dropped
  const auto tf = buf_rsrc(MODE == kRow2F ? out.twoF + it.tmpl * P.n_bins : nullptr,
                           MODE == kRow2F ? uint32_t(P.n_bins * int64_t(sizeof(float))) : 0u);
  const uint32_t nmask = uint32_t(P.n_fft - 1), lo = uint32_t(P.bin_lo);
  const uint32_t ostep = uint32_t(Rr * QS * PL);
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if (NBL % NT == 0 || b < NBL) {
      const int ql = b % RQ, i = b / RQ;
      float2 va[RL], vb[RL];
#pragma unroll
      for (int j = 0; j < RL; ++j) {
        va[j] = lds[Lay::template at_step<PL>(i, j, ql)];
        vb[j] = lds[Lay::template at_step<PL>(i, j, RQ + ql)];
      }
      twiddle_dft<RL, PL, L>(va, i, twl);
      twiddle_dft<RL, PL, L>(vb, i, twl);
      if (MODE == kRow2F) {
        const uint32_t o0 = uint32_t(it.q0 + ql + Rr * (QS * i + h)) + uint32_t(P.n_fft / 2);
#pragma unroll
        for (int m = 0; m < RL; ++m) {
          const uint32_t o = ((o0 + uint32_t(m) * ostep) & nmask) - lo;
          buf_store1(two_f(va[m], vb[m]), tf, o * uint32_t(sizeof(float)));
        }
        continue;
      }
      if (MODE == kRowCand) {
        // 2F now (the plain pass's bits), candidates after the transforms
#pragma unroll
        for (int m = 0; m < RL; ++m) pa[s][m] = two_f(va[m], vb[m]);
        continue;
      }
#pragma unroll
      for (int m = 0; m < RL; ++m) {
        const int64_t nat = it.q0 + ql + Rr * (int64_t(QS) * (i + m * PL) + h);
        const float v2 = rows_out<MODE>(P, ws, it, nat, va[m], vb[m], out);
        if (v2 >= 0.0f) {
          const unsigned long long key =
              best_key(v2, ((nat + P.n_fft / 2) & (P.n_fft - 1)) - P.bin_lo);
          bkey = key > bkey ? key : bkey;
        }
      }
    }
  }
  if constexpr (MODE == kRowCand) {
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int b = tid + s * NT;
      if (NBL % NT == 0 || b < NBL) {
        const int ql = b % RQ, i = b / RQ;
        const uint32_t o0 = uint32_t(it.q0 + ql + Rr * (QS * i + h)) + uint32_t(P.n_fft / 2);
#pragma unroll
        for (int m = 0; m < RL; ++m) {
          const uint32_t o = ((o0 + uint32_t(m) * ostep) & nmask) - lo;
          if (o < uint32_t(P.n_bins)) {
            keep_candidate(out, it.tmpl, o, pa[s][m]);
            const unsigned long long key = best_key(pa[s][m], o);
            bkey = key > bkey ? key : bkey;
          }
        }
      }
    }
  }
  if ((MODE == kRow2FExt || MODE == kRowCand) && out.best) best_to_global(out, it.tmpl, bkey);
}

template <int LOGL, int RQ, int NT, int MODE, int MLR>
__global__ __launch_bounds__(NT) void k_fft_rows(PlanConst P, void* ws, ChunkMap map, int slots,
                                                 int log_rr, RowOutput out) {
  extern __shared__ float2 lds[];
  constexpr int L = 1 << LOGL;
  constexpr int NL = 2 * RQ;  // lines: the a rows then the b rows
  constexpr int R0 = kR0<LOGL, MLR>;
  constexpr int PER0 = kPer0<LOGL, NL, NT, MLR>;
  using Lay = LdsLayout<L, R0, RQ>;
  float2* twl = lds + NL * Lay::pitch;
  const int64_t Rr = int64_t(1) << log_rr;
  const int tid = threadIdx.x;
  // grouped path: every reader of the group buffers the next chunk resamples
  // has finished (column pass of this chunk), so their status words restart
  if (blockIdx.x == 0 && tid < map.n_reset) *group_status(ws, P, slots, map.reset_buf[tid]) = 0;
  {
    const float2* __restrict__ tws = tw_stage(ws);
    for (int e = tid; e < L / 2; e += NT) twl[e] = tws[e * (kTwLen / L)];
  }
  const RowItem it =
      rows_item<MODE>(P, ws, map, int(xcd_remap(blockIdx.x, gridDim.x)), int(Rr / RQ), RQ);
  if (it.flagged && MODE != kRowConj) rows_flagged<LOGL, RQ, NT>(P, ws, it, Rr, out);
  if (!it.live) return;
  float2 v[PER0][R0];
  rows_load<LOGL, RQ, NT, MODE, MLR, 0, PER0>(P, ws, it, v);
  rows_stage0<LOGL, RQ, NT, MLR, NL>(lds, tid, v);
  __syncthreads();
  rows_finish<LOGL, RQ, NT, MODE, MLR>(P, ws, it, out, Rr, lds, twl, tid);
}

// The row pass for long rows in half the LDS: the radix-2 step of
// k_fft_cols_half applied to the RQ rows of both arrays (y_h[c] = (x[c] +
// (-1)^h x[c + L/2]) W_L^{c h}; entries 2k + h of the row transform are the
// (L/2)-point transform of y_h), y_1 waiting in registers while y_0 goes
// through LDS and the epilogue, so two workgroups share a compute unit
// (plain 2F; the other epilogues need more registers and run one: the
// candidate epilogue at two would spill the waiting half).
template <int LOGL, int RQ, int NT, int MODE, int MLR>
__global__ __launch_bounds__(NT, MODE == kRow2F ? NT / 128 : NT / 256) void
k_fft_rows_half(
    PlanConst P, void* ws, ChunkMap map, int slots, int log_rr, RowOutput out) {
  extern __shared__ float2 lds[];
  constexpr int LH = LOGL - 1;
  constexpr int L = 1 << LOGL, H = L / 2;
  constexpr int NL = 2 * RQ;
  constexpr int R0 = kR0<LH, MLR>, S0 = H / R0, NB0 = NL * S0;
  constexpr int PER0 = kPer0<LH, NL, NT, MLR>;
  using Lay = LdsLayout<H, R0, RQ>;
  float2* twl = lds + NL * Lay::pitch;
  const int64_t Rr = int64_t(1) << log_rr;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid < map.n_reset) *group_status(ws, P, slots, map.reset_buf[tid]) = 0;
  const float2* __restrict__ tws = tw_stage(ws);
  for (int e = tid; e < H / 2; e += NT) twl[e] = tws[e * (kTwLen / H)];
  const RowItem it =
      rows_item<MODE>(P, ws, map, int(xcd_remap(blockIdx.x, gridDim.x)), int(Rr / RQ), RQ);
  if (it.flagged && MODE != kRowConj) rows_flagged<LOGL, RQ, NT>(P, ws, it, Rr, out);
  if (!it.live) return;
  float2 a[PER0][R0], b[PER0][R0];
  {
    const auto rs = buf_rsrc(slot_buf(ws, P, it.g, MODE == kRowConj ? 2 : 0),
                             uint32_t(2 * P.n_fft * int64_t(sizeof(float2))));
#pragma unroll
    for (int s = 0; s < PER0; ++s) {
      const int bb = tid + s * NT;
      if (NB0 % NT == 0 || bb < NB0) {
        const int i = bb % S0, line = bb / S0;
        const int64_t e0 = (line < RQ ? 0 : P.n_fft) + (it.q0 + line % RQ) * L + i;
        const uint32_t voff = uint32_t(e0 * int64_t(sizeof(float2)));
#pragma unroll
        for (int j = 0; j < R0; ++j) {
          const uint32_t soff = uint32_t(j * S0 * int(sizeof(float2)));
          const uint32_t soff2 = uint32_t((j * S0 + H) * int(sizeof(float2)));
          a[s][j] = MODE == kRow2F ? buf_load2_stream(rs, voff, soff) : buf_load2(rs, voff, soff);
          b[s][j] = MODE == kRow2F ? buf_load2_stream(rs, voff, soff2)
                                   : buf_load2(rs, voff, soff2);
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < PER0; ++s) {
    const int bb = tid + s * NT;
    if (NB0 % NT == 0 || bb < NB0) {
      const int i = bb % S0;
#pragma unroll
      for (int j = 0; j < R0; ++j) {
        const int c = i + j * S0;
        const float2 d = csub(a[s][j], b[s][j]);
        a[s][j] = cadd(a[s][j], b[s][j]);
        b[s][j] = cmul(d, tws[c * (kTwLen / L)]);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int s = 0; s < PER0; ++s) {
      const int bb = tid + s * NT;
      if (NB0 % NT == 0 || bb < NB0) {
        const int i = bb % S0, line = bb / S0;
        float2(&v)[R0] = h ? b[s] : a[s];
        dft<R0>(v);
#pragma unroll
        for (int m = 0; m < R0; ++m) lds[Lay::at_block(i, m, line)] = v[m];
      }
    }
    __syncthreads();
    rows_finish<LH, RQ, NT, MODE, MLR, 2>(P, ws, it, out, Rr, lds, twl, tid, h);
    if (h == 0) __syncthreads();
  }
}

// Plain 2F row pass holding one array at a time: the RQ rows of y_a' are
// transformed and |Fa'|^2 of every bin the thread owns is kept in registers,
// then the same rows of y_b' reuse the LDS lines and the thread writes
// 2F = 2 (|Fa'|^2 + |Fb'|^2) (the same arithmetic, so the same bits, as
// k_fft_rows), or, with MODE kRowCand, keeps the bins above the threshold and
// the loudest bin instead of writing 2F.  With RQ lines of LDS instead of 2 RQ, two workgroups share a
// compute unit (the launch bound asks for registers to match) while the 2F
// runs stay RQ floats long.  At lines of 2^11 the compiler keeps two LDS
// offsets in scratch; recomputing the offsets in each pass instead measured
// 3 % slower.
template <int LOGL, int RQ, int NT, int MLR, int MODE>
__global__ __launch_bounds__(NT, NT / 128) void k_fft_rows_split(PlanConst P, void* ws,
                                                                  ChunkMap map, int slots,
                                                                  int log_rr, RowOutput out) {
  extern __shared__ float2 lds[];
  constexpr int L = 1 << LOGL;
  constexpr int NS = stage_count(LOGL, MLR);
  constexpr int R0 = kR0<LOGL, MLR>, NBL0 = L / R0, NB0 = RQ * NBL0;
  constexpr int RL = 1 << stage_logr(LOGL, NS - 1, MLR), PL = L / RL, NBL = RQ * PL;
  constexpr int PER0 = (NB0 + NT - 1) / NT;
  constexpr int PER = (NBL + NT - 1) / NT;
  using Lay = LdsLayout<L, R0, RQ>;
  float2* twl = lds + RQ * Lay::pitch;
  const int64_t Rr = int64_t(1) << log_rr;
  const int tid = threadIdx.x;
  // grouped path: every reader of the group buffers the next chunk resamples
  // has finished (column pass of this chunk), so their status words restart
  if (blockIdx.x == 0 && tid < map.n_reset) *group_status(ws, P, slots, map.reset_buf[tid]) = 0;
  {
    const float2* __restrict__ tws = tw_stage(ws);
    for (int e = tid; e < L / 2; e += NT) twl[e] = tws[e * (kTwLen / L)];
  }
  const RowItem it =
      rows_item<MODE>(P, ws, map, int(xcd_remap(blockIdx.x, gridDim.x)), int(Rr / RQ), RQ);
  if (it.flagged) rows_flagged<LOGL, RQ, NT>(P, ws, it, Rr, out);
  if (!it.live) return;
  const auto tf = buf_rsrc(MODE == kRow2F ? out.twoF + it.tmpl * P.n_bins : nullptr,
                           MODE == kRow2F ? uint32_t(P.n_bins * int64_t(sizeof(float))) : 0u);
  const uint32_t nmask = uint32_t(P.n_fft - 1), lo = uint32_t(P.bin_lo);
  const uint32_t ostep = uint32_t(Rr * PL);
  float pa[PER][RL];
#pragma unroll
  for (int arr = 0; arr < 2; ++arr) {
    // the a pass's last stage has finished reading the lines
    if (arr == 1) __syncthreads();
    const auto rs = buf_rsrc(slot_buf(ws, P, it.g, arr),
                             uint32_t(P.n_fft * int64_t(sizeof(float2))));
    float2 v[PER0][R0];
#pragma unroll
    for (int s = 0; s < PER0; ++s) {
      const int b = tid + s * NT;
      if (NB0 % NT == 0 || b < NB0) {
        const int i = b % NBL0, line = b / NBL0;
        const uint32_t voff = uint32_t(((it.q0 + line) * L + i) * int64_t(sizeof(float2)));
#pragma unroll
        for (int j = 0; j < R0; ++j)
          v[s][j] = buf_load2_stream(rs, voff, uint32_t(j * NBL0 * int(sizeof(float2))));
      }
    }
#pragma unroll
    for (int s = 0; s < PER0; ++s) {
      const int b = tid + s * NT;
      if (NB0 % NT == 0 || b < NB0) {
        const int i = b % NBL0, line = b / NBL0;
        dft<R0>(v[s]);
#pragma unroll
        for (int m = 0; m < R0; ++m) lds[Lay::at_block(i, m, line)] = v[s][m];
      }
    }
    __syncthreads();
    fft_middle<LOGL, RQ, NT, 1, MLR, Lay>(lds, twl, tid);
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int b = tid + s * NT;
      if (NBL % NT == 0 || b < NBL) {
        const int ql = b % RQ, i = b / RQ;
        float2 u[RL];
#pragma unroll
        for (int j = 0; j < RL; ++j) u[j] = lds[Lay::template at_step<PL>(i, j, ql)];
        twiddle_dft<RL, PL, L>(u, i, twl);
        if (arr == 0) {
#pragma unroll
          for (int m = 0; m < RL; ++m) pa[s][m] = fmaf(u[m].x, u[m].x, u[m].y * u[m].y);
        } else {
          const uint32_t o0 = uint32_t(it.q0 + ql + Rr * i) + uint32_t(P.n_fft / 2);
#pragma unroll
          for (int m = 0; m < RL; ++m) {
            const uint32_t o = ((o0 + uint32_t(m) * ostep) & nmask) - lo;
            const float v2 = 2.0f * (pa[s][m] + fmaf(u[m].x, u[m].x, u[m].y * u[m].y));
            if constexpr (MODE == kRow2F) {
              buf_store1(v2, tf, o * uint32_t(sizeof(float)));
            } else {
              pa[s][m] = v2;
            }
          }
        }
      }
    }
  }
  if constexpr (MODE == kRowCand) {
    // after the transforms, so the candidate code does not compete with
    // them for registers
    unsigned long long bkey = 0ull;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int b = tid + s * NT;
      if (NBL % NT == 0 || b < NBL) {
        const int ql = b % RQ, i = b / RQ;
        const uint32_t o0 = uint32_t(it.q0 + ql + Rr * i) + uint32_t(P.n_fft / 2);
#pragma unroll
        for (int m = 0; m < RL; ++m) {
          const uint32_t o = ((o0 + uint32_t(m) * ostep) & nmask) - lo;
          if (o < uint32_t(P.n_bins)) {
            keep_candidate(out, it.tmpl, o, pa[s][m]);
            const unsigned long long key = best_key(pa[s][m], o);
            bkey = key > bkey ? key : bkey;
          }
        }
      }
    }
    if (out.best) best_to_global(out, it.tmpl, bkey);
  }
}

// Copy of the resampled series for the diagnostic entry point: y_a, y_b of
// slot g into out[t][2][n_fft], zero beyond the computed grid, with the
// whitening undone (y_a = l11 y_a', y_b = l21 y_a' + l22 y_b').
__global__ void k_copy_series(PlanConst P, void* ws, ChunkMap map, float2* out) {
  const int g = blockIdx.y;
  const TmplParams& tp = *tmpl_params(ws, P, map, g);
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
