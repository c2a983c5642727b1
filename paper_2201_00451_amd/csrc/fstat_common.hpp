// Shared device-side definitions of the gfx950 resampling F-statistic path:
// per-plan constants passed by value to every kernel, the per-template
// constant block written by the prologue kernel, the workspace layout, and
// the FP64 timing helpers of steps (iii) and (iv) of Sec. 3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fstat.h"

namespace fstat {

constexpr int kMaxDet = FSTAT_MAX_DET;
constexpr double kPi = 3.14159265358979323846;

// Resampling tile: outputs per workgroup, threads, and the staged-sample
// capacity (tile + 1/16 drift allowance + 2D taps for D <= 32 + slack).  Two
// outputs per thread keep the resampling kernel at 115 registers and the
// adjoint at 249, so four and two waves per SIMD fit without spills
// (measured against 1024-point tiles: single-bin gradients 1800 to 2370 per
// second, resampling 4 % faster on sky positions, 1 % slower on binary
// orbits).
constexpr int kResTile = 512;
constexpr int kResTileLog = 9;
static_assert(kResTile == 1 << kResTileLog, "tile size is 2^kResTileLog");
constexpr int kResThreads = 256;
constexpr int kResPerThread = kResTile / kResThreads;
// Waves per SIMD of the resampling kernel whose timing knots were solved
// ahead (its registers: 512 / waves).
constexpr int kResWavesAhead = 5;
constexpr int kResWcap = kResTile + kResTile / 16 + 64 + 8;
// Flags of the staged window's 32-sample blocks (any live sample).
constexpr int kResBlk = (kResWcap + kResThreads) / 32 + 2;

// Ephemeris nodes a resampling tile stages in LDS (projected on the sky), per
// detector: bounds the ephemeris spacing from below (a tile spans its
// kResTile points plus twice the plan's max_delay and the tap reach).
constexpr int kNodeCap = 128;

// Detectors a resampling tile processes together: their timing solves,
// staging and interpolation share the tile's phases (and barriers).
constexpr int kDetPass = 2;

// Knot interpolation of the timing in the resampling kernel: the grid delays
// and the heterodyne phases of the input samples are solved exactly every G
// points (G = 2^knot_log2, 4 <= G <= 64, chosen per template from an error
// bound) and interpolated in between by cubic Hermite in FP64; knot_log2 = 0
// solves every point.  Knot capacities of one tile: grid knots G apart over
// the tile and its end, sample knots G apart over the staged window.
constexpr int kKnotLogMin = 2;
constexpr int kKnotLogMax = 6;
constexpr int kGridKnots = kResTile / (1 << kKnotLogMin) + 1;
constexpr int kSampKnots = (kResWcap - 1) / (1 << kKnotLogMin) + 2;

// On the search and plain forward paths the knots of templates with
// G >= 2^kKnotLogGlobal are solved ahead of the resampling, all in parallel,
// into a knot area of the series' buffer.  Per detector, in 16-byte units:
//   [0, knot_gcap)   the grid intervals m = 0 .. k_pad / G (from k = m G):
//                    the source position u = k + off + q of the interval's
//                    points as I_m + theta(v), v = (k - m G) / G, with the
//                    cubic theta in FP32 (float4: theta(0), then the
//                    coefficients of v, v^2, v^3; the last interval holds
//                    theta(0) only)
//   [knot_ioff, ..)  the integers I_m (int32)
//   [knot_soff, ..)  the sample intervals m = 0 .. (n_X - 1) / G (from
//                    j = m G), two units each: the heterodyne phase of the
//                    interval's samples in quarter turns as a cubic in
//                    t = j - m G, in FP64 (constant term reduced modulo one
//                    turn)
//   [knot_toff, ..)  per resampling tile, kTileRecUnits: the antenna Taylor
//                    coefficients about the tile's middle point and that
//                    point's theta(0) and I (plans whose tiles take the Taylor
//                    form only)
// Capacities at the smallest such G.
constexpr int kKnotLogGlobal = 4;
constexpr int kTileRecUnits = 4;
// k_knots: blocks of kKnotThreads knots, each block's last knot the next
// block's first, so that every grid interval finds both its ends in one block.
constexpr int kKnotThreads = 256;
__host__ __device__ inline int64_t knot_grid_blocks(int64_t gcap) {
  return (gcap + kKnotThreads - 2) / (kKnotThreads - 1);
}
__host__ __device__ inline int64_t knot_samp_blocks(int64_t scap) {
  return (scap + kKnotThreads - 2) / (kKnotThreads - 1);
}
__host__ __device__ inline int64_t knot_tile_blocks(int64_t k_pad) {
  return ((k_pad >> kResTileLog) + kKnotThreads - 1) / kKnotThreads;
}
// The whitened antenna patterns over a tile are taken as quintic polynomials
// in the sidereal angle's offset from the tile's middle point while the tile
// spans at most this angle on either side (radians).
constexpr double kTaylorMaxAngle = 0.1;
__host__ __device__ inline int64_t knot_grid_cap(int64_t k_pad) {
  return (k_pad >> kKnotLogGlobal) + 1;
}
__host__ __device__ inline int64_t knot_samp_cap(int64_t n) {
  return ((n - 1) >> kKnotLogGlobal) + 2;
}

// Moment reduction: fixed block count per detector (deterministic order).
constexpr int kMomBlocks = 256;
constexpr int kMomThreads = 256;

// Per-detector constants of a plan.
struct DetConst {
  double t0;          // time of sample 0
  double off;         // (tau0 - t0)/dt: grid index offset
  double lst0_cyc;    // (lon + sidereal angle at t=0) / 2 pi
  double lat, gamma;  // latitude, arm-bisector azimuth (CCW from East)
  double sl, cl;      // sin, cos of the latitude
  double s2g, c2g;    // sin, cos of twice the arm-bisector azimuth
  double w;           // 1/noise_var
  int64_t n;
  const float2* x;
  const uint8_t* valid;
  const double* ephem;
};

// Everything a kernel needs about the plan and the inputs (passed by value).
struct PlanConst {
  int32_t ndet, D;
  int32_t tmpl_stride;  // doubles per template row (8, or 10 for Keplerian orbits)
  double dt, inv_dt, f_het, t_ref, tau0, max_delay;
  double sid_rate_cyc;  // sidereal rate / 2 pi (cycles per s)
  int64_t n_fft, bin_lo, n_bins;
  int64_t k_pad;        // grid points computed by the resampler (multiple of tile and row)
  int64_t slot_stride;  // bytes per template slot of the workspace (path dependent)
  int64_t part_offset;  // adjoint paths: bytes from a slot's start to its tile partials
  int64_t knot_stride;  // 16-byte units per detector of a knot area
  int64_t knot_gcap;    // grid intervals of a detector's area
  int64_t knot_ioff, knot_soff, knot_toff;  // units to the integers, sample intervals, tiles
  int32_t res_taylor;   // the tiles take the antenna patterns' Taylor form
  int64_t knot_bytes;   // bytes of a knot area (each group buffer holds one)
  int64_t knot_offset;  // plain path: bytes from a slot's start to its knot area;
                        // 0: the slots have none (the tiles solve their knots)
  char* params;         // search path: per-template parameter blocks (kParamBytes
                        // each, by template index); null: the slots' own blocks
  int64_t n_eph;
  double eph_t0, eph_dt, inv_eph_dt;
  const double* moments;
  DetConst det[kMaxDet];
};

// Per-template constants, one block per workspace slot.
struct TmplParams {
  double nhat[3];
  double df, f1dot, f2dot, asini, om_b, tp;
  double nu_b;  // orbital frequency 1 / porb (0 for an isolated source)
  // Keplerian orbit (kepler != 0): eccentricity, sin and cos of the argument
  // of periapsis, sqrt(1 - ecc^2)
  int32_t kepler;
  double ecc, sin_w, cos_w, sq_e;
  // spin-down and sub-bin phase in quarter turns (4 x cycles) as a cubic in
  // the grid index k: 4 Phi(k) = sd[0] + k (sd[1] + k (sd[2] + k sd[3]))
  double sd[4];
  double alpha_cyc[kMaxDet];  // (alpha - lon - sidereal angle at 0) / 2 pi
  // Whitened, weighted antenna patterns: with M = [[A, C], [C, B]] = L L^T
  // (Cholesky), (a', b') = L^-1 (a, b) so that 2F = 2 (|Fa'|^2 + |Fb'|^2).
  // w_X a'(x) = ca0 + ca1 cos x + ca2 sin x + ca3 cos 2x + ca4 sin 2x.
  float ca[kMaxDet][5];
  float cb[kMaxDet][5];
  float l11, l21, l22;        // L, to report Fa = l11 Fa', Fb = l21 Fa' + l22 Fb'
  int32_t status;             // nonzero: every output bin of the template is NaN
  int32_t knot_log2;          // knot spacing of the resampling's timing (0: none)
  // Adjoint only: derivatives of the sky direction and of the whitened
  // coefficients with respect to (alpha, delta) at fixed x, and 2 pi / porb.
  double dnhat[2][3];
  float dca[2][kMaxDet][5];
  float dcb[2][kMaxDet][5];
  double porb;
  // Adjoint: a constant subtracted from the input-side delay derivatives
  // d delta_j / d(alpha, delta) (their value for detector 0 at the middle of
  // the grid).  A constant c contributes -2 pi i f_h c y'_k to dy'_k, whose
  // share of the gradient, 8 pi f_h c Im sum_k X_k y'_k = 8 pi f_h c
  // Im sum_m g_m |F'_m|^2, is exactly zero; removing it before rounding to
  // FP32 keeps the ~3e5 rad/rad sky phase derivative from cancelling in FP32.
  double dshift[2];
  // Single-bin adjoint only: natural FFT index of the template's bin and the
  // adjoint spectrum there, conj(Fa'), conj(Fb') (re, im, re, im).
  int64_t bin_nat;
  double hbin[4];
};

// Status bits of a template (any bit: NaN in every output bin).
constexpr int32_t kStatusTiming = 1;    // non-finite or invalid sky / orbit parameters
constexpr int32_t kStatusCoverage = 2;  // delays exceed the plan's max_delay
constexpr int32_t kStatusWindow = 4;    // a tile's input window overflowed the staging
constexpr int32_t kStatusNodes = 8;     // a delay evaluation left the staged ephemeris
constexpr int32_t kStatusPhase = 16;    // non-finite spin-down or sub-bin parameters
constexpr int32_t kStatusBin = 32;      // single-bin path: bin outside the band
// Bits that concern the resampled series of a sky/orbit group.
constexpr int32_t kStatusGroupMask = kStatusTiming | kStatusCoverage | kStatusWindow | kStatusNodes;

// Where the row pass puts its results (passed by value).  twoF: full band
// (stored, or added when acc is set); fafb: Fa and Fb; gin: adjoint weights;
// cand/count/cap/threshold: bins with 2F above the threshold appended to a
// list (count is the total, which may exceed cap); best: per template the
// largest 2F and its bin packed as (float bits << 32) | bin.
struct RowOutput {
  float* twoF;
  float2* fafb;
  const float* gin;
  fstat_candidate* cand;
  unsigned long long* count;
  unsigned long long* best;
  int64_t cap;
  float threshold;
  int32_t acc;
};

// Template slots of one launch sequence and, for the grouped path, the
// sky/orbit groups it resamples.  Passed by value to every kernel.
constexpr int kMaxSlots = 32;
struct ChunkMap {
  int32_t n_tmpl;               // slots in use
  int32_t n_grp;                // groups resampled by this chunk (grouped path)
  int64_t tmpl[kMaxSlots];      // template (output row) of slot s
  int32_t tmpl_buf[kMaxSlots];  // group buffer slot s reads (grouped path)
  int32_t grp_slot[kMaxSlots];  // slot holding the parameters of resampled group i
  int32_t grp_buf[kMaxSlots];   // group buffer resampled group i writes
  int32_t n_reset;              // grouped path: group buffers whose status word the
  int32_t reset_buf[kMaxSlots]; //   row pass clears for the next chunk's resampling
};

constexpr size_t kParamBytes = 1024;
static_assert(sizeof(TmplParams) <= kParamBytes, "param block");
// Workspace header: moment partials, then the FP32 twiddle table W_4096^e
// (stage twiddles of every line length <= 4096) written from FP64 at the
// start of every call, and reserved space.
constexpr int kTwLen = 4096;
constexpr size_t kMomentBytes = size_t(kMaxDet) * kMomBlocks * 10 * sizeof(double);
constexpr size_t kTwOffset = kMomentBytes;
constexpr size_t kHeaderBytes = kTwOffset + 3 * kTwLen * sizeof(float2) + 4096;
__host__ __device__ inline float2* tw_stage(void* ws) {
  return reinterpret_cast<float2*>(static_cast<char*>(ws) + kTwOffset);
}
// In the reserved space: the number of templates of the current call whose
// outputs are NaN (cleared by the first kernel of every call, counted once
// per template by the row pass or the single-bin reduction).
constexpr size_t kFlagOffset = kTwOffset + 3 * kTwLen * sizeof(float2);
__host__ __device__ inline unsigned long long* flag_counter(void* ws) {
  return reinterpret_cast<unsigned long long*>(static_cast<char*>(ws) + kFlagOffset);
}

// Workspace: header (moment partials, twiddles), then template slots of
// [TmplParams | narr arrays of n_fft float2 | extra bytes], narr = 2 for the
// forward paths (y_a / Z_a, y_b / Z_b) and 4 plus per-tile gradient partials
// for the adjoint.
__host__ __device__ inline size_t slot_bytes(int64_t n_fft, int narr = 2, size_t extra = 0) {
  return kParamBytes + size_t(n_fft) * narr * sizeof(float2) + extra;
}
__host__ __device__ inline char* slot_base(void* ws, const PlanConst& P, int g) {
  return static_cast<char*>(ws) + kHeaderBytes + size_t(g) * size_t(P.slot_stride);
}
__host__ __device__ inline TmplParams* slot_params(void* ws, const PlanConst& P, int g) {
  return reinterpret_cast<TmplParams*>(slot_base(ws, P, g));
}
// Parameter block of the template in slot g: the slot's own, or on the search
// path the template's block of the per-template array.
__host__ __device__ inline TmplParams* tmpl_params(void* ws, const PlanConst& P,
                                                  const ChunkMap& map, int g) {
  return P.params ? reinterpret_cast<TmplParams*>(P.params + size_t(map.tmpl[g]) * kParamBytes)
                  : slot_params(ws, P, g);
}
__host__ __device__ inline float2* slot_buf(void* ws, const PlanConst& P, int g, int arr) {
  return reinterpret_cast<float2*>(slot_base(ws, P, g) + kParamBytes) + size_t(arr) * P.n_fft;
}
// Adjoint paths: per-tile partial sums (8 doubles per tile) at part_offset
// from the slot's start (after the four arrays of the general adjoint, right
// after the parameter block on the single-bin path).
__host__ __device__ inline double* slot_partials(void* ws, const PlanConst& P, int g) {
  return reinterpret_cast<double*>(slot_base(ws, P, g) + P.part_offset);
}

// Grouped path: after `slots` template slots come group buffers of
// [status (256 B) | y_a : k_pad float2 | y_b : k_pad float2 | knot area], the
// resampled series of one sky/orbit group before its spin-down phase.
constexpr size_t kGroupHeader = 256;
__host__ __device__ inline size_t group_bytes(int64_t k_pad, int64_t knot_bytes) {
  return kGroupHeader + size_t(k_pad) * 2 * sizeof(float2) + size_t(knot_bytes);
}
__host__ __device__ inline char* group_base(void* ws, const PlanConst& P, int slots, int b) {
  return slot_base(ws, P, slots) + size_t(b) * group_bytes(P.k_pad, P.knot_bytes);
}
__host__ __device__ inline double2* group_knots(void* ws, const PlanConst& P, int slots, int b) {
  return reinterpret_cast<double2*>(group_base(ws, P, slots, b) + kGroupHeader +
                                    size_t(P.k_pad) * 2 * sizeof(float2));
}
__host__ __device__ inline double2* slot_knots(void* ws, const PlanConst& P, int g) {
  return P.knot_offset ? reinterpret_cast<double2*>(slot_base(ws, P, g) + P.knot_offset)
                       : nullptr;
}
__host__ __device__ inline int32_t* group_status(void* ws, const PlanConst& P, int slots, int b) {
  return reinterpret_cast<int32_t*>(group_base(ws, P, slots, b));
}
__host__ __device__ inline float2* group_buf(void* ws, const PlanConst& P, int slots, int b,
                                             int arr) {
  return reinterpret_cast<float2*>(group_base(ws, P, slots, b) + kGroupHeader) +
         size_t(arr) * P.k_pad;
}

// Raw buffer access (gfx9 buffer descriptor): a 32-bit per-lane byte offset
// plus a uniform one, so a run of loads shares one address register; a load
// at or past num_bytes returns zero without touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t num_bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(num_bytes), 0x00020000);
}
__device__ __forceinline__ float2 buf_load2(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                            uint32_t soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// Streaming read (non-temporal cache policy): for data read exactly once, so
// that it does not evict lines other loads and stores still use from L2 (the
// row passes read the intermediate once; meanwhile their partial 2F lines
// wait in L2 for their neighbours).
__device__ __forceinline__ float2 buf_load2_stream(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                   uint32_t soff) {
  constexpr int kNonTemporal = 2;
  return __builtin_bit_cast(float2,
                            __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kNonTemporal));
}
__device__ __forceinline__ void buf_store2(float2 x, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                           uint32_t soff) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, x), r, voff, soff, 0);
}
// One float; an offset at or past the descriptor's end drops the store.
__device__ __forceinline__ void buf_store1(float x, __amdgpu_buffer_rsrc_t r, uint32_t voff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, voff, 0, 0);
}

// ---------------------------------------------------------------------------
// FP64 timing (Sec. 2: t_b = t + t_m; binary: t_b = t_src + R(t_src)).
// ---------------------------------------------------------------------------

// Cubic Hermite interpolation on one interval: positions p0, p1 and slopes
// v0, v1 (per second) at its ends, u in [0, 1] the fraction of the interval h.
__device__ inline void hermite(double p0, double v0, double p1, double v1, double u, double h,
                               double inv_h, double& d, double& dd) {
  double u2 = u * u, u3 = u2 * u;
  d = (2.0 * u3 - 3.0 * u2 + 1.0) * p0 + (u3 - 2.0 * u2 + u) * h * v0 +
      (-2.0 * u3 + 3.0 * u2) * p1 + (u3 - u2) * h * v1;
  dd = (6.0 * u2 - 6.0 * u) * (p0 - p1) * inv_h + (3.0 * u2 - 4.0 * u + 1.0) * v0 +
       (3.0 * u2 - 2.0 * u) * v1;
}

// Roemer delay n.r(t) and its time derivative read from the tabulated
// detector trajectory in global memory (node index clamped to the table).
struct GlobalRoemer {
  const double* tab;
  const double* nh;
  int64_t n_eph;
  double t0, h, inv_h;
  __device__ void operator()(double t, double& d, double& dd) const {
    double s = (t - t0) * inv_h;
    int64_t i = static_cast<int64_t>(floor(s));
    i = i < 0 ? 0 : (i > n_eph - 2 ? n_eph - 2 : i);
    const double* e0 = tab + 6 * i;
    const double* e1 = e0 + 6;
    double p0 = nh[0] * e0[0] + nh[1] * e0[1] + nh[2] * e0[2];
    double v0 = nh[0] * e0[3] + nh[1] * e0[4] + nh[2] * e0[5];
    double p1 = nh[0] * e1[0] + nh[1] * e1[1] + nh[2] * e1[2];
    double v1 = nh[0] * e1[3] + nh[1] * e1[4] + nh[2] * e1[5];
    hermite(p0, v0, p1, v1, s - static_cast<double>(i), h, inv_h, d, dd);
  }
};

// GlobalRoemer that keeps the interval it read last in registers: the
// successive evaluations of one fixed-point or Newton solve fall in the same
// interval (they differ by far less than its length), so a solve reads the
// trajectory about once.  Same arithmetic, so the same values.
struct CachedRoemer {
  const double* tab;
  const double* nh;
  int64_t n_eph;
  double t0, h, inv_h;
  mutable int64_t i_cached = -1;
  mutable double p0 = 0.0, v0 = 0.0, p1 = 0.0, v1 = 0.0;
  __device__ void operator()(double t, double& d, double& dd) const {
    double s = (t - t0) * inv_h;
    int64_t i = static_cast<int64_t>(floor(s));
    i = i < 0 ? 0 : (i > n_eph - 2 ? n_eph - 2 : i);
    if (i != i_cached) {
      const double* e0 = tab + 6 * i;
      const double* e1 = e0 + 6;
      p0 = nh[0] * e0[0] + nh[1] * e0[1] + nh[2] * e0[2];
      v0 = nh[0] * e0[3] + nh[1] * e0[4] + nh[2] * e0[5];
      p1 = nh[0] * e1[0] + nh[1] * e1[1] + nh[2] * e1[2];
      v1 = nh[0] * e1[3] + nh[1] * e1[4] + nh[2] * e1[5];
      i_cached = i;
    }
    hermite(p0, v0, p1, v1, s - static_cast<double>(i), h, inv_h, d, dd);
  }
};

// The same cubic per interval, staged in LDS as its power-series
// coefficients in u = (t - t_i) / h: interval i holds (c0, c1), (c2, c3) with
// c0 = p0, c1 = h v0, c2 = 3 (p1 - p0) - h (2 v0 + v1),
// c3 = 2 (p0 - p1) + h (v0 + v1) of the projected nodes i, i + 1, so an
// evaluation is three FMAs for the delay and three for its slope.  count is
// the number of nodes (intervals + 1); an evaluation outside them is clamped
// (memory-safe) and raises `oob`.
struct CubicRoemer {
  const double2* coef;
  int count;
  double t0, inv_h;
  __device__ void operator()(double t, double& d, double& dd, bool& oob) const {
    const double s = (t - t0) * inv_h;
    int i = static_cast<int>(fmin(fmax(floor(s), -1.0), double(count)));
    if (i < 0 || i > count - 2) {
      oob = true;
      i = i < 0 ? 0 : count - 2;
    }
    const double u = s - static_cast<double>(i);
    const double2 a = coef[2 * i], b = coef[2 * i + 1];
    d = fma(fma(fma(b.y, u, b.x), u, a.y), u, a.x);
    dd = fma(fma(3.0 * b.y, u, 2.0 * b.x), u, a.y) * inv_h;
  }
};
// Interval coefficients of CubicRoemer from projected positions p and
// velocities v of two neighbouring nodes h apart.
__device__ inline void cubic_interval(double p0, double v0, double p1, double v1, double h,
                                      double2& lo, double2& hi) {
  lo = make_double2(p0, h * v0);
  hi = make_double2(3.0 * (p1 - p0) - h * (2.0 * v0 + v1), 2.0 * (p0 - p1) + h * (v0 + v1));
}

// The Hermite form from nodes already projected on the sky (n.r, n.v) and
// staged in LDS: node i sits at t0 + i h.  An evaluation outside the staged
// nodes is clamped (memory-safe) and raises `oob`.
struct NodeRoemer {
  const double2* nodes;
  int count;
  double t0, h, inv_h;
  __device__ void operator()(double t, double& d, double& dd, bool& oob) const {
    double s = (t - t0) * inv_h;
    double fl = floor(s);
    int i = static_cast<int>(fmin(fmax(fl, -1.0), double(count)));
    if (i < 0 || i > count - 2) {
      oob = true;
      i = i < 0 ? 0 : count - 2;
    }
    double2 a = nodes[i], b = nodes[i + 1];
    hermite(a.x, a.y, b.x, b.y, s - static_cast<double>(i), h, inv_h, d, dd);
  }
};

// sin and cos of 2 pi c for a phase c in FP64 cycles (|c| < 2^28): the
// quarter-turn count and remainder are split exactly in FP64, then the
// Taylor polynomials of sin and cos in x = (pi/2) r, |x| <= pi/4, through x^13
// and x^14 (truncation below 3e-14), and a quadrant swap.
__device__ inline void sincos_cycles(double c, double& sn, double& cs) {
  const double c4 = 4.0 * c;
  const double q = rint(c4);
  const double x = (c4 - q) * 1.57079632679489661923;
  const double u = x * x;
  double ps = fma(u, -1.0 / 6227020800.0, 1.0 / 39916800.0);
  ps = fma(u, ps, -1.0 / 362880.0);
  ps = fma(u, ps, 1.0 / 5040.0);
  ps = fma(u, ps, -1.0 / 120.0);
  ps = fma(u, ps, 1.0 / 6.0);
  const double s0 = fma(-x * u, ps, x);
  double pc = fma(u, 1.0 / 87178291200.0, -1.0 / 479001600.0);
  pc = fma(u, pc, 1.0 / 3628800.0);
  pc = fma(u, pc, -1.0 / 40320.0);
  pc = fma(u, pc, 1.0 / 720.0);
  pc = fma(u, pc, -1.0 / 24.0);
  pc = fma(u, pc, 0.5);
  const double c0 = fma(-u, pc, 1.0);
  const int n = int(q) & 3;
  const double x1 = (n & 1) ? s0 : c0, y1 = (n & 1) ? c0 : s0;
  cs = (n == 1 || n == 2) ? -x1 : x1;
  sn = (n & 2) ? -y1 : y1;
}

// Keplerian orbit: R(t') and R'(t') from the eccentric anomaly E of Kepler's
// equation E - ecc sin E = M, M = 2 pi (t' - tp) / porb reduced to half a
// turn in FP64 cycles; Newton's iteration from E = M + ecc sin M until the
// update is at the rounding level (at most 12 steps; quadratic convergence
// from this start for ecc < 0.95).
__device__ inline void kepler_delay(const TmplParams& tp, double t, double& r, double& rp) {
  double mc = (t - tp.tp) * tp.nu_b;
  mc -= rint(mc);
  const double M = 2.0 * kPi * mc;
  double sm, cm;
  sincos_cycles(mc, sm, cm);
  double E = M + tp.ecc * sm, sE = 0.0, cE = 1.0;
  for (int it = 0; it < 12; ++it) {
    sincos_cycles(E * (0.5 / kPi), sE, cE);
    const double step = (E - tp.ecc * sE - M) / (1.0 - tp.ecc * cE);
    E -= step;
    if (fabs(step) < 1e-15) break;
  }
  sincos_cycles(E * (0.5 / kPi), sE, cE);
  r = tp.asini * (tp.sin_w * (cE - tp.ecc) + tp.cos_w * tp.sq_e * sE);
  const double dr_de = tp.asini * (tp.cos_w * tp.sq_e * cE - tp.sin_w * sE);
  rp = dr_de * tp.om_b / (1.0 - tp.ecc * cE);
}

// The source's orbital Roemer delay R(t') and its rate R'(t') (both 0 for
// an isolated source): circular asini sin(2 pi (t' - tp) / porb), or the
// Keplerian orbit.  KEP = false compiles the circular orbit only (plans
// without Keplerian rows), so those kernels carry no Kepler solver.
template <bool KEP>
__device__ inline void orbit_delay(const TmplParams& tp, double t, double& r, double& rp) {
  if (tp.asini == 0.0) {
    r = rp = 0.0;
  } else if (KEP && tp.kepler) {
    kepler_delay(tp, t, r, rp);
  } else {
    double s, c;
    sincos_cycles((t - tp.tp) * tp.nu_b, s, c);
    r = tp.asini * s;
    rp = tp.asini * tp.om_b * c;
  }
}

// Binary Roemer delay R(tau) of the source (0 for an isolated source).
template <bool KEP>
__device__ inline double binary_delay(const TmplParams& tp, double tau) {
  if (tp.asini == 0.0) return 0.0;
  if (KEP && tp.kepler) {
    double r, rp;
    kepler_delay(tp, tau, r, rp);
    return r;
  }
  double s, c;
  sincos_cycles((tau - tp.tp) * tp.nu_b, s, c);
  return tp.asini * s;
}

// Step (iv): for the source-frame time tau return T - tau, where the detector
// time T satisfies T + roemer(T) = tau + R(tau).  One fixed-point step from
// T = t_b then one Newton step; 1/(1 + roemer') by its series to third order
// (|roemer'| < 1e-3 for any Earth-bound detector: residual < 1e-12 s).
// grid_delay_rb takes the binary delay rb = R(tau) already evaluated.
template <class RoemerFn, class... Flag>
__device__ inline double grid_delay_rb(const RoemerFn& roemer, double rb, double tau,
                                       Flag&... oob) {
  double d0, dd0;
  roemer(tau + rb, d0, dd0, oob...);
  double dl = rb - d0;
  double d1, x;
  roemer(tau + dl, d1, x, oob...);
  double g = dl + d1 - rb;
  return dl - g * (1.0 - x * (1.0 - x * (1.0 - x)));
}
template <bool KEP, class RoemerFn, class... Flag>
__device__ inline double grid_delay(const RoemerFn& roemer, const TmplParams& tp, double tau,
                                    Flag&... oob) {
  return grid_delay_rb(roemer, binary_delay<KEP>(tp, tau), tau, oob...);
}


// Step (iv) from a prediction: one Newton step on T + roemer(T) = tau + rb
// (rb = R(tau)) started at T = tau + guess.  The caller predicts from a
// solved neighbour by linearising the Roemer delay only (the binary delay is
// exact), so the guess is off by |roemer''| dT^2 / 2 < 2e-3 s within a tile and
// the step leaves < 1e-15 s.  Returns T - tau; x receives roemer'(T).
template <class RoemerFn, class... Flag>
__device__ inline double grid_delay_newton(const RoemerFn& roemer, double tau, double rb,
                                           double guess, double& x, Flag&... oob) {
  double d1;
  roemer(tau + guess, d1, x, oob...);
  return guess - (guess + d1 - rb) * (1.0 - x * (1.0 - x * (1.0 - x)));
}

// The source-frame delay R(t_src) of the emission that reaches the
// barycentre at tb (t_src + R(t_src) = tb): one Newton step from R(tb).  The
// phase at t_src is the phase at tb minus om_b r0, an angle below
// asini om_b < 1e-2 rad, so its sine and cosine follow from the ones at tb by
// angle addition with short series (truncation below 1e-17), and the Newton
// denominator 1 / (1 + asini om_b cos) is its series to third order
// (residual < 1e-12 s).  s and c receive the sine and cosine of the orbital
// phase at tb - R(tb), the first iterate of t_src.
__device__ inline double binary_inverse(const TmplParams& tp, double tb, double& s, double& c) {
  double s0, c0;
  sincos_cycles((tb - tp.tp) * tp.nu_b, s0, c0);
  const double r0 = tp.asini * s0;
  const double e = tp.om_b * r0, e2 = e * e;
  const double ce = fma(e2, fma(e2, 1.0 / 24.0, -0.5), 1.0);
  const double se = e * fma(e2, -1.0 / 6.0, 1.0);
  s = fma(s0, ce, -c0 * se);
  c = fma(c0, ce, s0 * se);
  const double h = r0 - tp.asini * s;
  const double g = tp.asini * tp.om_b * c;
  return r0 - h * fma(g, fma(g, 1.0 - g, -1.0), 1.0);
}

// R(t_src) for a Keplerian orbit, t_src + R(t_src) = tb: Newton's iteration
// from t_src = tb - R(tb), three steps (contraction max|R'| < 1e-2: residual
// below 1e-12 s).
__device__ inline double kepler_inverse(const TmplParams& tp, double tb) {
  double r, rp;
  kepler_delay(tp, tb, r, rp);
  double ts = tb - r;
  for (int it = 0; it < 3; ++it) {
    kepler_delay(tp, ts, r, rp);
    ts -= (ts + r - tb) / (1.0 + rp);
  }
  return tb - ts;
}

// R(t_src) for the emission that reaches the barycentre at tb, either orbit.
template <bool KEP>
__device__ inline double orbit_inverse(const TmplParams& tp, double tb) {
  if (KEP && tp.kepler) return kepler_inverse(tp, tb);
  double s, c;
  return binary_inverse(tp, tb, s, c);
}

// Step (iii): for the detector sample time t return t_src - t, where
// t_src + R(t_src) = t + roemer(t).  R is found by one Newton step from
// R(t_b) (contraction asini * om_b < 1e-2: residual < 1e-12 s), or for a
// Keplerian orbit by kepler_inverse.
template <bool KEP, class RoemerFn, class... Flag>
__device__ inline double sample_delay(const RoemerFn& roemer, const TmplParams& tp, double t,
                                      Flag&... oob) {
  double dr, ddr;
  roemer(t, dr, ddr, oob...);
  double r = 0.0;
  if (tp.asini != 0.0) r = orbit_inverse<KEP>(tp, t + dr);
  return dr - r;
}

// Step (iii) at a knot: the heterodyne phase f_h (t_src - t) in cycles at
// the detector sample time t and its rate per second,
//   d(t_src - t)/dt = roemer'(t) - R'(t_src) (1 + roemer'(t)) / (1 + R'(t_src)),
// with the orbital phase at t_src taken again after the inverse (its first
// iterate is 1e-3 s off, too far for the rate).
// sample_phase_d also returns the delay t_src - t itself.
template <bool KEP, class RoemerFn, class... Flag>
__device__ inline void sample_phase_d(const RoemerFn& roemer, const TmplParams& tp, double t,
                                      double f_het, double& ph, double& dph, double& delay,
                                      Flag&... oob) {
  double dr, ddr;
  roemer(t, dr, ddr, oob...);
  double r = 0.0, rate = 0.0;
  if (tp.asini != 0.0) {
    r = orbit_inverse<KEP>(tp, t + dr);
    double r2, rp;
    orbit_delay<KEP>(tp, t + dr - r, r2, rp);
    rate = rp * (1.0 + ddr) / (1.0 + rp);
  }
  delay = dr - r;
  ph = f_het * delay;
  dph = f_het * (ddr - rate);
}
template <bool KEP, class RoemerFn, class... Flag>
__device__ inline void sample_phase(const RoemerFn& roemer, const TmplParams& tp, double t,
                                    double f_het, double& ph, double& dph, Flag&... oob) {
  double delay;
  sample_phase_d<KEP>(roemer, tp, t, f_het, ph, dph, delay, oob...);
}

// Cubic Hermite coefficients in u in [0, 1] of one knot interval from the
// values and the derivatives per unit step at its ends, the ends g steps
// apart: p(u) = c0 + u (c1 + u (c2 + u c3)).
__device__ inline void hermite_interval(double2 a, double2 b, double g, double2& lo,
                                        double2& hi) {
  lo = make_double2(a.x, g * a.y);
  hi = make_double2(3.0 * (b.x - a.x) - g * (2.0 * a.y + b.y),
                    2.0 * (a.x - b.x) + g * (a.y + b.y));
}
__device__ __forceinline__ double hermite_eval(const double2* c, int seg, double u) {
  const double2 lo = c[2 * seg], hi = c[2 * seg + 1];
  return fma(fma(fma(hi.y, u, hi.x), u, lo.y), u, lo.x);
}

// Split a fractional sample position into floor and fraction, keeping the
// fraction below one after rounding to float.
__device__ inline void split_u(double u, int64_t& j0, float& f) {
  double fl = floor(u);
  j0 = static_cast<int64_t>(fl);
  f = static_cast<float>(u - fl);
  if (f >= 1.0f) {
    j0 += 1;
    f = 0.0f;
  }
}

// (cos, sin) of (pi/2)(n + r) for an integer quarter-turn count n and a
// remainder |r| <= 1/2.  sin((pi/2) r) = r P(r^2), cos((pi/2) r) = 1 + r^2 Q(r^2)
// with P cubic and Q cubic, fitted for this file to the functions on
// [0, 1/4] in r^2 (least squares on Chebyshev nodes, reweighted towards
// equal ripple); evaluated with FMA in FP32 the results are within 9e-8 (sin)
// and 6e-8 (cos) of the exact values.  The quadrant then swaps and negates.
__device__ __forceinline__ float2 cis_quarter(int n, float r) {
  const float u = r * r;
  float ps = fmaf(u, -4.602177069e-03f, 7.968022674e-02f);
  ps = fmaf(u, ps, -6.459634900e-01f);
  ps = fmaf(u, ps, 1.570796371e+00f);
  const float sn = r * ps;
  float pc = fmaf(u, 9.040216682e-04f, -2.086028829e-02f);
  pc = fmaf(u, pc, 2.536692321e-01f);
  pc = fmaf(u, pc, -1.233700514e+00f);
  const float cs = fmaf(u, pc, 1.0f);
  const bool odd = (n & 1) != 0;
  const float x = odd ? sn : cs, y = odd ? cs : sn;
  // cos is negative in quadrants 1 and 2, sin in quadrants 2 and 3
  const uint32_t sx = uint32_t((n + 1) & 2) << 30, sy = uint32_t(n & 2) << 30;
  return make_float2(__uint_as_float(__float_as_uint(x) ^ sx),
                     __uint_as_float(__float_as_uint(y) ^ sy));
}

// (cos 2 pi c, sin 2 pi c) for a phase c in FP64 cycles (|c| < 2^28): the
// quarter-turn count and remainder are taken exactly in FP64, so only the
// remainder is rounded to FP32.
__device__ __forceinline__ float2 cis_cycles(double c) {
  const double c4 = 4.0 * c;
  const double q = rint(c4);
  return cis_quarter(int(q), static_cast<float>(c4 - q));
}

// The same for a phase already in FP32 cycles (exact quarter-turn split).
__device__ __forceinline__ float2 cis_cycles_f32(float c) {
  const float c4 = 4.0f * c;
  const float q = rintf(c4);
  return cis_quarter(int(q), c4 - q);
}

// exp(-2 pi i e / n) for 0 <= e < n = 2^log_n <= 2^24: the quarter-turn
// count and remainder of 4 e / n are split exactly in integers.
__device__ __forceinline__ float2 cis_neg_frac(int64_t e, int log_n) {
  const int64_t t = e << 2;
  const int64_t q = (t + (int64_t(1) << (log_n - 1))) >> log_n;
  const float r = ldexpf(float(int32_t(t - (q << log_n))), -log_n);
  const float2 v = cis_quarter(int(q), r);
  return make_float2(v.x, -v.y);
}

// exp(-i Phi_s(tau_k)) exp(-2 pi i df (tau_k - tau0)): the spin-down phase of
// Sec. 2 about t_ref and the sub-bin frequency offset.  The template carries
// the phase as a cubic in the grid index k in quarter turns
// (spindown_coefficients); it is evaluated in FP64 with FMA, split into a
// quarter-turn count and an FP32 remainder, and rotated with cis_quarter.
// One definition for every kernel that applies it, so the per-template and
// grouped paths agree bit for bit.
__host__ __device__ inline void spindown_coefficients(const PlanConst& P, double f1dot,
                                                      double f2dot, double df, double sd[4]) {
  // with d0 = tau0 - t_ref and s = dt k, in cycles:
  //   f1dot (d0 + s)^2 / 2 + f2dot (d0 + s)^3 / 6 + df s
  // stored times 4 (quarter turns; the scaling by 4 is exact)
  // The constant term is reduced modulo one turn (exactly: fmod rounds
  // nothing), so that the quarter-turn count of the evaluated cubic stays far
  // inside 32 bits even for a reference time years away from the grid.
  const double d0 = P.tau0 - P.t_ref, dt = P.dt;
  sd[0] = fmod(4.0 * (f1dot * d0 * d0 * 0.5 + f2dot * d0 * d0 * d0 * (1.0 / 6.0)), 4.0);
  sd[1] = 4.0 * (dt * (f1dot * d0 + f2dot * d0 * d0 * 0.5 + df));
  sd[2] = 4.0 * (dt * dt * (f1dot * 0.5 + f2dot * d0 * 0.5));
  sd[3] = 4.0 * (dt * dt * dt * f2dot * (1.0 / 6.0));
}
// k < n_fft <= 2^24
__device__ __forceinline__ float2 spindown_rotation(const double sd[4], int64_t k) {
  const double x = double(int32_t(k));
  const double c4 = fma(x, fma(x, fma(x, sd[3], sd[2]), sd[1]), sd[0]);
  const double q = rint(c4);
  const float2 e = cis_quarter(int(q), static_cast<float>(c4 - q));
  return make_float2(e.x, -e.y);
}

__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// Complex product with explicit FMA: applying the spin-down rotation in
// different kernels must give the same bits whatever the compiler contracts.
__device__ inline float2 cmul_exact(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

}  // namespace fstat
