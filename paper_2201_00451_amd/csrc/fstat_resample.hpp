// Steps (iii)-(v) of Sec. 3 and the weighting of step (vi), fused.
//
// One workgroup owns kResTile consecutive points of the regular source-frame
// grid tau_k = tau0 + k dt of one template.  For each detector it
//   1. stages the ephemeris intervals the tile can touch in LDS: the cubic
//      Hermite of each interval, from its two nodes projected on the sky
//      direction (n.r, n.v), as power-series coefficients, so every later
//      delay evaluation is three FMAs on LDS data;
//   2. solves the detector epochs T_k of step (iv) for the thread's own grid
//      points (FP64): the tile's first point by a fixed-point and a Newton
//      step, every other point by one Newton step from the first point's
//      solution extrapolated along dT/dtau; T_k is monotonic in k, so the
//      tile's first and last points bound the input samples it touches;
//   3. stages those samples in LDS after the step (iii) heterodyne correction
//      z_j = x_j exp(-2 pi i f_h (t_src,j - t_j)) (FP64 delay, split
//      exactly into quarter turns and an FP32 remainder, polynomial
//      rotation): each input sample is read from HBM
//      and corrected once per tile;
//   4. interpolates z at T_k with the 2D-tap Hann-windowed sinc
//      h(s) = sinc(s) (1 + cos(pi s / D)) / 2 (the paper leaves the kernel of
//      step (v) unnamed) and accumulates w_X a'(T_k) zhat_k, w_X b'(T_k) zhat_k
//      with the whitened antenna patterns of the template.
// Finally it removes the spin-down phase Phi_s(tau_k) and the sub-bin offset
// df (FP64 phase, FP32 rotation) and writes y_a', y_b' (float2) with
// coalesced stores.  FP64 is used only for times and phases.
//
// The half-width D is a template parameter: with s = f + c_t, c_t = D-1-t,
//   h_t = sin(pi f) * [A_t cos(pi f/D) + B_t sin(pi f/D) + C_t] / s,
//   A_t = (-1)^{c_t} cos(pi c_t/D) / (2 pi), B_t = -(-1)^{c_t} sin(pi c_t/D) / (2 pi),
//   C_t = (-1)^{c_t} / (2 pi),
// so each tap costs one reciprocal, two FMAs for the window and two for the
// accumulation; sin(pi f) multiplies the finished sum.
#pragma once

#include <utility>

#include "fstat_common.hpp"

namespace fstat {

// Compile-time cos and sin of pi * n / d (Taylor series after reduction to
// [-pi/4, pi/4]); used only to build tap constants.
__host__ __device__ constexpr double ct_poly_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
__host__ __device__ constexpr double ct_poly_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// cos(pi q / 4) and sin(pi q / 4) for integer q, then angle addition
__host__ __device__ constexpr double ct_cospi(int n, int d) {
  // pi n/d = pi (q/4) + r with |r| <= pi/8
  const double x = double(n) / double(d);
  const int q = int(x * 4.0 + (x >= 0 ? 0.5 : -0.5));
  const double r = kPi * (x - q / 4.0);
  const int qm = ((q % 8) + 8) % 8;
  const double h = 0.70710678118654752440;
  const double cq = qm == 0 ? 1.0 : qm == 1 ? h : qm == 2 ? 0.0 : qm == 3 ? -h
                  : qm == 4 ? -1.0 : qm == 5 ? -h : qm == 6 ? 0.0 : h;
  const double sq = qm == 0 ? 0.0 : qm == 1 ? h : qm == 2 ? 1.0 : qm == 3 ? h
                  : qm == 4 ? 0.0 : qm == 5 ? -h : qm == 6 ? -1.0 : -h;
  return cq * ct_poly_cos(r) - sq * ct_poly_sin(r);
}
__host__ __device__ constexpr double ct_sinpi(int n, int d) {
  const double x = double(n) / double(d);
  const int q = int(x * 4.0 + (x >= 0 ? 0.5 : -0.5));
  const double r = kPi * (x - q / 4.0);
  const int qm = ((q % 8) + 8) % 8;
  const double h = 0.70710678118654752440;
  const double cq = qm == 0 ? 1.0 : qm == 1 ? h : qm == 2 ? 0.0 : qm == 3 ? -h
                  : qm == 4 ? -1.0 : qm == 5 ? -h : qm == 6 ? 0.0 : h;
  const double sq = qm == 0 ? 0.0 : qm == 1 ? h : qm == 2 ? 1.0 : qm == 3 ? h
                  : qm == 4 ? 0.0 : qm == 5 ? -h : qm == 6 ? -1.0 : -h;
  return sq * ct_poly_cos(r) + cq * ct_poly_sin(r);
}

// Tap constants of half-width D, built at compile time into constant memory
// (read with uniform indices, whether or not the tap loop is unrolled):
//   A_t, B_t, C_t as above; Ct_t = cos(pi c_t / D), St_t = sin(pi c_t / D).
struct TapConst {
  float A[64], B[64], C[64], Ct[64], St[64];
};
template <int D>
__host__ __device__ constexpr TapConst make_taps() {
  TapConst k{};
  for (int t = 0; t < 2 * D; ++t) {
    const int c = D - 1 - t;
    const double sgn = (c & 1) ? -1.0 : 1.0;
    const double cc = ct_cospi(c, D), ss = ct_sinpi(c, D);
    k.A[t] = float(sgn * cc / (2.0 * kPi));
    k.B[t] = float(-sgn * ss / (2.0 * kPi));
    k.C[t] = float(sgn / (2.0 * kPi));
    k.Ct[t] = float(cc);
    k.St[t] = float(ss);
  }
  return k;
}
template <int D>
__constant__ TapConst kTaps = make_taps<D>();

// One tap of the forward interpolation with its constants as compile-time
// literals: with c = D - 1 - T the tap's integer offset,
//   h_T (up to the common factor sin(pi f) / (2 pi)) =
//     (-1)^c (1 + cos(pi c/D) cos(pi f/D) - sin(pi c/D) sin(pi f/D)) / (f + c),
// the Hann window by angle addition and the sinc's alternating sign folded
// into the accumulation.  Two literal FMAs for the window, one reciprocal,
// one multiply and two FMAs per tap; no constant reaches a register.
template <int D, int T>
__device__ __forceinline__ void interp_tap(float f, float wc, float ws, const float2* zp,
                                           float& sx, float& sy) {
  constexpr int c = D - 1 - T;
  constexpr float cs = float(ct_cospi(c, D));
  constexpr float sn = float(ct_sinpi(c, D));
  const float w = fmaf(wc, cs, fmaf(ws, -sn, 1.0f));
  float h = w * __builtin_amdgcn_rcpf(f + float(c));
  if constexpr ((c & 1) != 0) h = -h;
  const float2 zv = zp[T];
  sx = fmaf(h, zv.x, sx);
  sy = fmaf(h, zv.y, sy);
}
template <int D, int... T>
__device__ __forceinline__ void interp_taps(std::integer_sequence<int, T...>, float f, float wc,
                                            float ws, const float2* zp, float& sx, float& sy) {
  (interp_tap<D, T>(f, wc, ws, zp, sx, sy), ...);
}

// sin(pi f) / (2 pi) for 0 <= f < 1 from h = min(f, 1 - f) (exact for f >=
// 1/2): the odd Taylor series of sin(pi h) / (2 pi) through h^13, whose first
// omitted term is below 7e-10 of the value at h = 1/2, so the result keeps
// its relative precision at both ends of the interval, where the sinc's
// numerator meets the vanishing denominator of the nearest tap.
struct SinPiCoef {
  float c[7];
};
__host__ __device__ constexpr SinPiCoef make_sinpi_coef() {
  SinPiCoef k{};
  double t = 0.5;  // pi / (2 pi)
  for (int n = 0; n < 7; ++n) {
    k.c[n] = float(t);
    t *= -(kPi * kPi) / double((2 * n + 2) * (2 * n + 3));
  }
  return k;
}
__device__ __forceinline__ float sinpi_over_2pi(float f) {
  constexpr SinPiCoef k = make_sinpi_coef();
  const float h = fminf(f, 1.0f - f);
  const float u = h * h;
  float p = k.c[6];
#pragma unroll
  for (int n = 5; n >= 0; --n) p = fmaf(p, u, k.c[n]);
  return h * p;
}

// Step (v): the 2D-tap interpolation of the samples zp[0 .. 2D) at the
// fraction f of the point between zp[D - 1] and zp[D].
template <int D>
__device__ __forceinline__ float2 sinc_interp(float f, const float2* zp) {
  static_assert(D >= 4, "the window phase stays within one eighth turn");
  if (f == 0.0f) return zp[D - 1];
  // window phase pi f / D: 2 f / D <= 1/2 quarter turns, no reduction
  const float2 wcs = cis_quarter(0, 4.0f * (f * (0.5f / float(D))));
  float sx = 0.f, sy = 0.f;
  interp_taps<D>(std::make_integer_sequence<int, 2 * D>{}, f, wcs.x, wcs.y, zp, sx, sy);
  const float sp = sinpi_over_2pi(f);
  return make_float2(sx * sp, sy * sp);
}

// The weighting of step (vi): the whitened antenna patterns of detector X
// at T = tau + q dt times the interpolated value, added to acc_a, acc_b.
__device__ __forceinline__ void weight_add(const PlanConst& P, const TmplParams& tp, int X,
                                           double tau, double q, float2 zh, float2& acc_a,
                                           float2& acc_b) {
  // x = alpha - phi(T), in cycles
  const float2 ex = cis_cycles(tp.alpha_cyc[X] - P.sid_rate_cyc * (tau + q * P.dt));
  const float cx = ex.x, sx = ex.y;
  const float c2 = cx * cx - sx * sx, s2 = 2.0f * sx * cx;
  const float a = tp.ca[X][0] + tp.ca[X][1] * cx + tp.ca[X][2] * sx + tp.ca[X][3] * c2 +
                  tp.ca[X][4] * s2;
  const float b = tp.cb[X][0] + tp.cb[X][1] * cx + tp.cb[X][2] * sx + tp.cb[X][3] * c2 +
                  tp.cb[X][4] * s2;
  acc_a.x = fmaf(a, zh.x, acc_a.x);
  acc_a.y = fmaf(a, zh.y, acc_a.y);
  acc_b.x = fmaf(b, zh.x, acc_b.x);
  acc_b.y = fmaf(b, zh.y, acc_b.y);
}

// The first tap of grid point k_s + kk in the staged window (start lo, W
// samples): u = k + off + q = j0 + f, taps j0-D+1 .. j0+D; monotonic T_k keeps
// them inside the window, the clamp only guards memory.
template <int D>
__device__ __forceinline__ int tap_base(const PlanConst& P, int X, int64_t lo, int W,
                                        int64_t k_s, int kk, double q, float& f) {
  int64_t j0;
  split_u(double(k_s + kk) + P.det[X].off + q, j0, f);
  const int base = int(j0 - lo) - (D - 1);
  return base < 0 ? 0 : (base > W - 2 * D ? W - 2 * D : base);
}
// Whether any tap from base on falls on a live sample (block flags blk).
template <int D>
__device__ __forceinline__ bool taps_live(const int32_t* blk, int base) {
  return (blk[base >> 5] | blk[(base + 2 * D - 1) >> 5]) != 0;
}

// Steps (v) and the weighting of (vi) at one grid point k_s + kk of detector
// X, whose epoch is T_k = tau_k + q dt, from the staged window zs.  A point
// whose taps all fall on zero samples adds nothing.
template <int D>
__device__ __forceinline__ void interp_point(const PlanConst& P, const TmplParams& tp, int X,
                                             const float2* zs, const int32_t* blk, int64_t lo,
                                             int W, int64_t k_s, int kk, double q, double tau_s,
                                             float2& acc_a, float2& acc_b) {
  float f;
  const int base = tap_base<D>(P, X, lo, W, k_s, kk, q, f);
  if (!taps_live<D>(blk, base)) return;
  weight_add(P, tp, X, tau_s + P.dt * double(kk), q, sinc_interp<D>(f, zs + base), acc_a, acc_b);
}

// The whitened antenna patterns of detector X over one tile as quintic
// polynomials in the sidereal angle's offset d from the tile's middle point:
// with x = alpha - phi(T), a(x) = ca0 + ca1 cos x + ca2 sin x + ca3 cos 2x
// + ca4 sin 2x has the Taylor coefficients a_n = a^(n)(x_r) / n! at x_r
// (and b likewise).  The remainder is below (2|d|)^6 / 6! of the coefficients'
// scale, 1e-7 at |d| = 0.1 rad, the bound kTaylorMaxAngle under which the
// tile takes this form.  c[0..5]: a_0..a_5, c[6..11]: b_0..b_5.
constexpr int kTaylorCoef = 12;
static_assert(kTaylorCoef + 2 <= kTileRecUnits * 4, "a tile record holds the coefficients");
__device__ inline void antenna_taylor(const TmplParams& tp, int X, double x_cyc,
                                      float (&c)[kTaylorCoef]) {
  const float2 e = cis_cycles(x_cyc);
  const float c1 = e.x, s1 = e.y;
  const float c2 = c1 * c1 - s1 * s1, s2 = 2.0f * s1 * c1;
#pragma unroll
  for (int ab = 0; ab < 2; ++ab) {
    const float* k = ab ? tp.cb[X] : tp.ca[X];
    // value p and derivative q of the first and second harmonic at x_r
    const float p1 = k[1] * c1 + k[2] * s1, q1 = k[2] * c1 - k[1] * s1;
    const float p2 = k[3] * c2 + k[4] * s2, q2 = k[4] * c2 - k[3] * s2;
    float* o = c + 6 * ab;
    o[0] = k[0] + p1 + p2;
    o[1] = q1 + 2.0f * q2;
    o[2] = -(p1 + 4.0f * p2) * (1.0f / 2.0f);
    o[3] = -(q1 + 8.0f * q2) * (1.0f / 6.0f);
    o[4] = (p1 + 16.0f * p2) * (1.0f / 24.0f);
    o[5] = (q1 + 32.0f * q2) * (1.0f / 120.0f);
  }
}

// Steps (v) and (vi) at one grid point whose taps start at base in the staged
// window zs (fraction f), with the antenna patterns from the tile's Taylor
// coefficients c (uniform across the tile) at the angle offset d (radians).
template <int D>
__device__ __forceinline__ void interp_point_taylor(const float2* zs, const int32_t* blk, int W,
                                                    int base, float f, float d,
                                                    const float (&c)[kTaylorCoef], float2& acc_a,
                                                    float2& acc_b) {
  base = base < 0 ? 0 : (base > W - 2 * D ? W - 2 * D : base);
  if (!taps_live<D>(blk, base)) return;
  const float2 zh = sinc_interp<D>(f, zs + base);
  float a = c[5], b = c[11];
#pragma unroll
  for (int n = 4; n >= 0; --n) {
    a = fmaf(a, d, c[n]);
    b = fmaf(b, d, c[6 + n]);
  }
  acc_a.x = fmaf(a, zh.x, acc_a.x);
  acc_a.y = fmaf(a, zh.y, acc_a.y);
  acc_b.x = fmaf(b, zh.x, acc_b.x);
  acc_b.y = fmaf(b, zh.y, acc_b.y);
}

// q = (T_k - tau_k)/dt at grid offset k within its knot interval from the
// interval's two knots (value, derivative per grid step) G steps apart.
__device__ __forceinline__ double knot_hermite(const double2* kn, int G, double u) {
  double2 c[2];
  hermite_interval(kn[0], kn[1], double(G), c[0], c[1]);
  return hermite_eval(c, 0, u);
}

// A value every lane of the wave holds, moved to scalar registers.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint64_t u = uint64_t(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(u));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(u >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}

// Steps (iii)-(v) and the antenna weighting for the kResTile grid points of
// the tile starting at k_s: acc_a[i], acc_b[i] receive sum_X a'_X(T_k)
// zhat_X(u_k) (and b'), k = k_s + tid + i kResThreads, before the spin-down
// phase.  Returns false, after flagging the template's status word, when the
// template must report NaN (the return is uniform across the block).
//
// Detectors are taken kDetPass at a time, each pass in five phases separated
// by barriers: (1) the pass's ephemeris intervals, and the binary delay at
// the grid knots; (2) the detector epochs at the grid knots; (3) each
// detector's staged window from them, the loads of its input samples, and the
// heterodyne phase at the sample knots while those loads are in flight;
// (4) the corrected samples into LDS; (5) interpolation and weighting.
//
// Timing (tp.knot_log2 = log2 G > 0): the grid delays q_k = (T_k - tau_k)/dt
// are solved exactly at every G-th grid point of the tile and its end, the
// heterodyne phases f_h (t_src,j - t_j) at every G-th staged sample, each
// with its derivative, and every point in between takes the cubic Hermite of
// its interval (FP64).  G is chosen per template so that the interpolation
// error stays below 2e-7 cycles of phase and 1e-7 samples of grid position.
// knot_log2 = 0: every grid point and sample is solved.
// Zero samples (gaps, and outside the data) are staged as zeros without any
// timing; a wave whose outputs' taps all fall on zero samples skips the
// interpolation (it would add zeros).
template <int D, bool KEP>
__device__ inline bool resample_tile(const PlanConst& P, const TmplParams& tp,
                                     int32_t* status_word, int64_t k_s, float2* zsa,
                                     int32_t* blka, float2 (&acc_a)[kResPerThread],
                                     float2 (&acc_b)[kResPerThread]) {
  constexpr int kRounds = (kResWcap + kResThreads - 1) / kResThreads;
  const int tid = threadIdx.x;
  __shared__ double2 coef[kDetPass][2 * kNodeCap];
  __shared__ double2 orb[kGridKnots];  // binary delay and rate at the grid knots
  // knot path: grid knots (q, dq/dk) of each detector, then its sample knots
  // (phase, dphase/dj); exact path: q of every grid point of each detector
  __shared__ double2 kbuf[kDetPass * (kGridKnots + kSampKnots)];
  __shared__ int bad;
  static_assert(kDetPass * (kGridKnots + kSampKnots) * 2 >= kDetPass * kResTile,
                "exact-path delays must fit the knot buffer");
  double2* const gk = kbuf;                          // [kDetPass][kGridKnots]
  double2* const sk = kbuf + kDetPass * kGridKnots;  // [kDetPass][kSampKnots]
  double* const qx = reinterpret_cast<double*>(kbuf);  // [kDetPass][kResTile]

  if (tid == 0) bad = 0;
  bool oob = false;
#pragma unroll
  for (int i = 0; i < kResPerThread; ++i) {
    acc_a[i] = make_float2(0.f, 0.f);
    acc_b[i] = make_float2(0.f, 0.f);
  }
  const int kl = tp.knot_log2;
  const bool knots = kl != 0;
  const int G = 1 << kl;
  const double inv_g = 1.0 / double(G);
  const int nkg = kResTile / G + 1;
  // time span any delay evaluation of this tile can reach (sample knots run
  // up to G samples past the staged window)
  const double pad = P.max_delay + double(D + 2 + (1 << kKnotLogMax)) * P.dt;
  const double t_first = P.tau0 + P.dt * double(k_s) - pad;
  const double t_last = P.tau0 + P.dt * double(k_s + kResTile - 1) + pad;
  int64_t n_lo = int64_t(floor((t_first - P.eph_t0) * P.inv_eph_dt)) - 1;
  n_lo = n_lo < 0 ? 0 : (n_lo > P.n_eph - 2 ? P.n_eph - 2 : n_lo);
  int64_t n_hi = int64_t(floor((t_last - P.eph_t0) * P.inv_eph_dt)) + 2;
  n_hi = n_hi > P.n_eph - 1 ? P.n_eph - 1 : n_hi;
  int n_count = int(n_hi - n_lo + 1);
  n_count = n_count > kNodeCap ? kNodeCap : (n_count < 2 ? 2 : n_count);
  const double node_t0 = P.eph_t0 + double(n_lo) * P.eph_dt;
  const double tau_s = P.tau0 + P.dt * double(k_s);
  // exact path: the binary delay at the own grid points (all detectors)
  double rbk[kResPerThread];
  double rb0 = 0.0;
  if (!knots) {
    rb0 = binary_delay<KEP>(tp, tau_s);
#pragma unroll
    for (int i = 0; i < kResPerThread; ++i)
      rbk[i] = binary_delay<KEP>(tp, tau_s + P.dt * double(tid + i * kResThreads));
  }

  for (int X0 = 0; X0 < P.ndet; X0 += kDetPass) {
    const int np = P.ndet - X0 < kDetPass ? P.ndet - X0 : kDetPass;
    // 1. interval coefficients from the projected nodes i and i + 1 of each
    // detector of the pass; the binary delay and its rate at the grid knots
    {
      const int ni = n_count - 1;
      for (int e = tid; e < np * ni; e += kResThreads) {
        const int xp = e >= ni ? 1 : 0;
        const int i = e - xp * ni;
        const double* n = P.det[X0 + xp].ephem + 6 * (n_lo + i);
        const double p0 = tp.nhat[0] * n[0] + tp.nhat[1] * n[1] + tp.nhat[2] * n[2];
        const double v0 = tp.nhat[0] * n[3] + tp.nhat[1] * n[4] + tp.nhat[2] * n[5];
        const double p1 = tp.nhat[0] * n[6] + tp.nhat[1] * n[7] + tp.nhat[2] * n[8];
        const double v1 = tp.nhat[0] * n[9] + tp.nhat[1] * n[10] + tp.nhat[2] * n[11];
        cubic_interval(p0, v0, p1, v1, P.eph_dt, coef[xp][2 * i], coef[xp][2 * i + 1]);
      }
      if (knots && X0 == 0 && tid < nkg) {
        double r, rp;
        orbit_delay<KEP>(tp, tau_s + P.dt * double(tid * G), r, rp);
        orb[tid] = make_double2(r, rp);
      }
    }
    __syncthreads();
    // 2. detector epochs as q = (T - tau)/dt: at the grid knots (fixed point
    // and three Newton steps, with dq/dk = (R'(tau) - roemer'(T)) /
    // (1 + roemer'(T))), or at every own grid point (the tile's first point
    // in full, the rest by one Newton step from a prediction that carries the
    // exact binary delay and linearises the Roemer delay about the first
    // point: T ~ T_s + (t_b - t_b,s) / (1 + roemer'(T_s)))
    if (knots) {
      for (int e = tid; e < np * nkg; e += kResThreads) {
        const int xp = e >= nkg ? 1 : 0;
        const int t = e - xp * nkg;
        const CubicRoemer re{coef[xp], n_count, node_t0, P.inv_eph_dt};
        const double tau = tau_s + P.dt * double(t * G);
        const double2 o = orb[t];
        double x;
        double dl = grid_delay_rb(re, o.x, tau, oob);
        dl = grid_delay_newton(re, tau, o.x, dl, x, oob);
        dl = grid_delay_newton(re, tau, o.x, dl, x, oob);
        gk[xp * kGridKnots + t] = make_double2(dl * P.inv_dt, (o.y - x) / (1.0 + x));
      }
    } else {
      for (int xp = 0; xp < np; ++xp) {
        const CubicRoemer re{coef[xp], n_count, node_t0, P.inv_eph_dt};
        double x0;
        double d0 = grid_delay_rb(re, rb0, tau_s, oob);
        d0 = grid_delay_newton(re, tau_s, rb0, d0, x0, oob);
        d0 = grid_delay_newton(re, tau_s, rb0, d0, x0, oob);
        const double inv0 = 1.0 - x0 * (1.0 - x0 * (1.0 - x0));
#pragma unroll
        for (int i = 0; i < kResPerThread; ++i) {
          const int kk = tid + i * kResThreads;
          const double dtau = P.dt * double(kk);
          const double guess = d0 + (dtau + rbk[i] - rb0) * inv0 - dtau;
          double x;
          qx[xp * kResTile + kk] =
              grid_delay_newton(re, tau_s + dtau, rbk[i], guess, x, oob) * P.inv_dt;
        }
      }
    }
    __syncthreads();
    // 3. each detector's staged window from its first and last epochs (T_k
    // is monotonic in k; the knot path bounds the last point by the knot
    // just past the tile), the loads of its samples, and the heterodyne
    // phase at its sample knots while they are in flight
    int64_t lo[kDetPass];
    int W[kDetPass];
    bool wbad = false;
#pragma unroll
    for (int xp = 0; xp < kDetPass; ++xp) {
      lo[xp] = 0;
      W[xp] = 0;
      if (xp >= np) continue;
      const double q0 = knots ? gk[xp * kGridKnots].x : qx[xp * kResTile];
      const double q1 = knots ? gk[xp * kGridKnots + nkg - 1].x : qx[xp * kResTile + kResTile - 1];
      const int64_t k1 = knots ? k_s + kResTile : k_s + kResTile - 1;
      int64_t j_first, j_last;
      float f;
      split_u(double(k_s) + P.det[X0 + xp].off + q0, j_first, f);
      split_u(double(k1) + P.det[X0 + xp].off + q1, j_last, f);
      // every thread computes the same window from LDS: keep it in scalar
      // registers
      lo[xp] = uniform_i64(j_first - D + 1);
      const int64_t nwin = j_last + D - lo[xp] + 1;
      // delay drift beyond 1/16 per tile: flag the template (NaN output)
      if (nwin > kResWcap || nwin < 2 * D) wbad = true;
      W[xp] = __builtin_amdgcn_readfirstlane(int(nwin));
    }
    if (wbad) {
      if (tid == 0) atomicOr(status_word, kStatusWindow);
      return false;
    }
    float2 xv[kDetPass][kRounds];
#pragma unroll
    for (int xp = 0; xp < kDetPass; ++xp) {
      const DetConst& d = P.det[X0 + (xp < np ? xp : 0)];
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        const int w = r * kResThreads + tid;
        const int64_t j = lo[xp] + w;
        xv[xp][r] = (xp < np && w < W[xp] && j >= 0 && j < d.n) ? d.x[j] : make_float2(0.f, 0.f);
      }
    }
    if (knots) {
      const int nks0 = ((W[0] - 1) >> kl) + 2;
      const int nks1 = np > 1 ? ((W[1] - 1) >> kl) + 2 : 0;
      for (int e = tid; e < nks0 + nks1; e += kResThreads) {
        const int xp = e >= nks0 ? 1 : 0;
        const int t = e - xp * nks0;
        const CubicRoemer re{coef[xp], n_count, node_t0, P.inv_eph_dt};
        double ph, dph;
        const int64_t lox = xp ? lo[1] : lo[0];
        sample_phase<KEP>(re, tp, P.det[X0 + xp].t0 + P.dt * double(lox + int64_t(t) * G),
                          P.f_het, ph, dph, oob);
        sk[xp * kSampKnots + t] = make_double2(ph, dph * P.dt);
      }
    }
    __syncthreads();
    // 4. corrected input samples z_j = x_j exp(-2 pi i f_h (t_src,j - t_j));
    // a zero sample (outside the data, or in a gap) stays zero, untimed
#pragma unroll 1
    for (int xp = 0; xp < np; ++xp) {
      const CubicRoemer re{coef[xp], n_count, node_t0, P.inv_eph_dt};
      const int64_t lox = xp ? lo[1] : lo[0];
      const int Wx = xp ? W[1] : W[0];
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        const int w = r * kResThreads + tid;
        if (r * kResThreads >= Wx) break;
        const float2 x = xp ? xv[1][r] : xv[0][r];
        const bool live = x.x != 0.f || x.y != 0.f;
        float2 z = make_float2(0.f, 0.f);
        if (live) {
          double ph;
          if (knots) {
            ph = knot_hermite(sk + xp * kSampKnots + (w >> kl), G, double(w & (G - 1)) * inv_g);
          } else {
            ph = P.f_het * sample_delay<KEP>(re, tp, P.det[X0 + xp].t0 + P.dt * double(lox + w),
                                             oob);
          }
          const float2 e = cis_cycles(ph);
          // x * exp(-2 pi i f_h dl)
          z = make_float2(x.x * e.x + x.y * e.y, x.y * e.x - x.x * e.y);
        }
        if (w < Wx) zsa[xp * kResWcap + w] = z;
        // which 32-sample blocks of the window hold a live sample
        const unsigned long long m = __ballot(live);
        if ((tid & 63) == 0) {
          const int b = w >> 5;
          blka[xp * kResBlk + b] = uint32_t(m) != 0u;
          blka[xp * kResBlk + b + 1] = uint32_t(m >> 32) != 0u;
        }
      }
    }
    __syncthreads();
    // 5. interpolation and antenna weighting (each accumulator takes the
    // detectors in order)
#pragma unroll 1
    for (int xp = 0; xp < np; ++xp) {
      const int X = X0 + xp;
      const int64_t lox = xp ? lo[1] : lo[0];
      const int Wx = xp ? W[1] : W[0];
#pragma unroll
      for (int i = 0; i < kResPerThread; ++i) {
        const int kk = tid + i * kResThreads;
        const double q = knots ? knot_hermite(gk + xp * kGridKnots + (kk >> kl), G,
                                              double(kk & (G - 1)) * inv_g)
                               : qx[xp * kResTile + kk];
        interp_point<D>(P, tp, X, zsa + xp * kResWcap, blka + xp * kResBlk, lox, Wx, k_s, kk, q,
                        tau_s, acc_a[i], acc_b[i]);
      }
    }
    if (X0 + kDetPass < P.ndet) __syncthreads();
  }
  if (oob) bad = 1;
  __syncthreads();
  if (bad) {
    // a delay evaluation left the staged ephemeris nodes: the delay exceeds
    // the plan's max_delay; flag the template (NaN output)
    if (tid == 0) atomicOr(status_word, kStatusNodes);
    return false;
  }
  return true;
}

// The tile for a template whose timing knots k_knots solved ahead (knot
// area kn): each thread reads the knot records of its own samples and grid
// points, so a pass of kDetPass detectors has two phases, the corrected
// samples into LDS and then interpolation and weighting, with one barrier
// between them.  The window of a detector runs from the tile's first source
// position to the one of the interval just past the tile (T_k is monotonic in
// k).  The grid points take their source positions from the FP32 interval
// cubics relative to the intervals' integers, and (plans with res_taylor) the
// antenna patterns from the tile's Taylor record, so the interpolation phase
// runs without FP64 arithmetic.
template <int D>
__device__ inline bool resample_tile_gk(const PlanConst& P, const TmplParams& tp,
                                        const double2* __restrict__ kn, int32_t* status_word,
                                        int64_t k_s, float2* zsa, int32_t* blka,
                                        float2 (&acc_a)[kResPerThread],
                                        float2 (&acc_b)[kResPerThread]) {
  constexpr int kRounds = (kResWcap + kResThreads - 1) / kResThreads;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < kResPerThread; ++i) {
    acc_a[i] = make_float2(0.f, 0.f);
    acc_b[i] = make_float2(0.f, 0.f);
  }
  const int kl = tp.knot_log2;
  const int G = 1 << kl;
  const float inv_gf = 1.0f / float(G);
  const double tau_s = P.tau0 + P.dt * double(k_s);
  const int64_t e_s = k_s >> kl;  // the tile's first interval
  // d(angle)/d(grid step) of the sidereal angle x, radians
  const float dstep = float(-2.0 * kPi * P.sid_rate_cyc * P.dt);
  for (int X0 = 0; X0 < P.ndet; X0 += kDetPass) {
    const int np = P.ndet - X0 < kDetPass ? P.ndet - X0 : kDetPass;
    int64_t lo[kDetPass];
    int W[kDetPass];
    bool wbad = false;
#pragma unroll
    for (int xp = 0; xp < kDetPass; ++xp) {
      lo[xp] = 0;
      W[xp] = 0;
      if (xp >= np) continue;
      const double2* ka = kn + (X0 + xp) * P.knot_stride;
      const float4* gr = reinterpret_cast<const float4*>(ka);
      const int32_t* gi = reinterpret_cast<const int32_t*>(ka + P.knot_ioff);
      const int64_t e_e = (k_s + kResTile) >> kl;
      // floor of the source position at the tile's first point and at the
      // point just past it (theta(0) in [0, 1], 1 after rounding)
      const int64_t j_first = k_s + gi[e_s] + (gr[e_s].x >= 1.0f ? 1 : 0);
      const int64_t j_last = k_s + kResTile + gi[e_e] + (gr[e_e].x >= 1.0f ? 1 : 0);
      lo[xp] = uniform_i64(j_first - D + 1);
      const int64_t nwin = j_last + D - lo[xp] + 1;
      // delay drift beyond 1/16 per tile: flag the template (NaN output)
      if (nwin > kResWcap || nwin < 2 * D) wbad = true;
      W[xp] = __builtin_amdgcn_readfirstlane(int(nwin));
    }
    if (wbad) {
      if (tid == 0) atomicOr(status_word, kStatusWindow);
      return false;
    }
    // corrected input samples z_j = x_j exp(-2 pi i f_h (t_src,j - t_j)) from
    // the sample knots; a zero sample (outside the data, or in a gap) stays
    // zero
#pragma unroll 1
    for (int xp = 0; xp < np; ++xp) {
      const DetConst& d = P.det[X0 + xp];
      const int64_t lox = xp ? lo[1] : lo[0];
      const int Wx = xp ? W[1] : W[0];
      // window offsets w in [wlo, whi) hold data samples j = lox + w; the
      // interval records from the one of sample lox on (floor division)
      const int32_t wlo = lox < 0 ? int32_t(-lox) : 0;
      const int32_t whi = d.n - lox < int64_t(Wx) ? int32_t(d.n - lox) : Wx;
      const int32_t jph = int32_t(lox & (G - 1));
      const double2* sr = kn + (X0 + xp) * P.knot_stride + P.knot_soff + 2 * (lox >> kl);
      const float2* xs = d.x + lox;
      float2 xv[kRounds];
      double2 k0[kRounds], k1[kRounds];
      // a wave whose lanes all lie past the window skips the round (its
      // 32-sample blocks lie past the last one a tap reads)
      const int w0 = __builtin_amdgcn_readfirstlane(tid) & ~63;
      const bool any = wlo < whi;
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        const int w = r * kResThreads + tid;
        const bool in = w >= wlo && w < whi;
        xv[r] = in ? xs[w] : make_float2(0.f, 0.f);
        // record of the sample's interval (of the nearest data sample); none
        // for a wave past the window
        const bool rec = any && r * kResThreads + w0 < Wx;
        const int32_t wc = rec ? (w < wlo ? wlo : (w >= whi ? whi - 1 : w)) : wlo;
        const double2* rc = sr + 2 * ((jph + wc) >> kl);
        k0[r] = rec ? rc[0] : make_double2(0.0, 0.0);
        k1[r] = rec ? rc[1] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        if (r * kResThreads + w0 >= Wx) break;
        const int w = r * kResThreads + tid;
        const float2 x = xv[r];
        const bool live = x.x != 0.f || x.y != 0.f;
        float2 z = make_float2(0.f, 0.f);
        if (live) {
          // heterodyne phase in quarter turns
          const double t = double((jph + w) & (G - 1));
          const double c4 = fma(fma(fma(k1[r].y, t, k1[r].x), t, k0[r].y), t, k0[r].x);
          const double q = rint(c4);
          const float2 e = cis_quarter(int(q), static_cast<float>(c4 - q));
          // x * exp(-2 pi i f_h dl)
          z = make_float2(x.x * e.x + x.y * e.y, x.y * e.x - x.x * e.y);
        }
        if (w < Wx) zsa[xp * kResWcap + w] = z;
        // which 32-sample blocks of the window hold a live sample
        const unsigned long long mb = __ballot(live);
        if ((tid & 63) == 0) {
          const int b = w >> 5;
          blka[xp * kResBlk + b] = uint32_t(mb) != 0u;
          blka[xp * kResBlk + b + 1] = uint32_t(mb >> 32) != 0u;
        }
      }
    }
    __syncthreads();
    // interpolation and antenna weighting (each accumulator takes the
    // detectors in order)
#pragma unroll 1
    for (int xp = 0; xp < np; ++xp) {
      const int X = X0 + xp;
      const double2* ka = kn + X * P.knot_stride;
      const float4* gr = reinterpret_cast<const float4*>(ka) + e_s;
      const int32_t* gi = reinterpret_cast<const int32_t*>(ka + P.knot_ioff) + e_s;
      const int64_t lox = xp ? lo[1] : lo[0];
      const int Wx = xp ? W[1] : W[0];
      const int32_t sb = int32_t(k_s - lox) - (D - 1);
      if (P.res_taylor) {
        // the tile's record: uniform, scalar registers
        const float* tr = reinterpret_cast<const float*>(ka + P.knot_toff +
                                                         (k_s >> kResTileLog) * kTileRecUnits);
        float c[kTaylorCoef];
#pragma unroll
        for (int n = 0; n < kTaylorCoef; ++n) c[n] = tr[n];
        const float th_r = tr[kTaylorCoef];
        const int32_t i_r = __float_as_int(tr[kTaylorCoef + 1]);
#pragma unroll
        for (int i = 0; i < kResPerThread; ++i) {
          const int kk = tid + i * kResThreads;
          const float4 cq = gr[kk >> kl];
          const int32_t im = gi[kk >> kl];
          const float v = float(kk & (G - 1)) * inv_gf;
          const float th = fmaf(fmaf(fmaf(cq.w, v, cq.z), v, cq.y), v, cq.x);
          const float fl = floorf(th);
          float f = th - fl;
          int base = sb + im + kk + int(fl);
          if (f >= 1.0f) {
            f = 0.0f;
            base += 1;
          }
          // sidereal angle offset from the tile's middle point
          const float d = (float(kk - kResTile / 2 + (im - i_r)) + (th - th_r)) * dstep;
          interp_point_taylor<D>(zsa + xp * kResWcap, blka + xp * kResBlk, Wx, base, f, d, c,
                                 acc_a[i], acc_b[i]);
        }
      } else {
#pragma unroll
        for (int i = 0; i < kResPerThread; ++i) {
          const int kk = tid + i * kResThreads;
          const float4 cq = gr[kk >> kl];
          const int32_t im = gi[kk >> kl];
          const float v = float(kk & (G - 1)) * inv_gf;
          const float th = fmaf(fmaf(fmaf(cq.w, v, cq.z), v, cq.y), v, cq.x);
          const float fl = floorf(th);
          float f = th - fl;
          int base = sb + im + kk + int(fl);
          if (f >= 1.0f) {
            f = 0.0f;
            base += 1;
          }
          base = base < 0 ? 0 : (base > Wx - 2 * D ? Wx - 2 * D : base);
          if (!taps_live<D>(blka + xp * kResBlk, base)) continue;
          const float2 zh = sinc_interp<D>(f, zsa + xp * kResWcap + base);
          // q = u - k - off
          const double q = (double(im) - P.det[X].off) + double(th);
          weight_add(P, tp, X, tau_s + P.dt * double(kk), q, zh, acc_a[i], acc_b[i]);
        }
      }
    }
    if (X0 + kDetPass < P.ndet) __syncthreads();
  }
  return true;
}

// Grid knot at k: q = (T_k - tau_k)/dt from the detector epoch of tau = tau0 +
// k dt (fixed point and two Newton steps) and dq/dk = (R'(tau) - roemer'(T)) /
// (1 + roemer'(T)); far: the delay exceeds the plan's max_delay.
template <bool KEP>
__device__ __forceinline__ double2 grid_knot(const PlanConst& P, const TmplParams& tp,
                                             const CachedRoemer& re, int64_t k, bool& far) {
  const double tau = P.tau0 + P.dt * double(k);
  double rb, rbd, x;
  orbit_delay<KEP>(tp, tau, rb, rbd);
  double dl = grid_delay_rb(re, rb, tau);
  dl = grid_delay_newton(re, tau, rb, dl, x);
  dl = grid_delay_newton(re, tau, rb, dl, x);
  far = !(fabs(dl) <= P.max_delay);
  return make_double2(dl * P.inv_dt, (rbd - x) / (1.0 + x));
}

// Timing knots of one template (slot) or sky/orbit group whose knot spacing
// G = 2^tp.knot_log2 is at least 2^kKnotLogGlobal, for the detector
// blockIdx.z: the same FP64 solves as the tiles' own knots (steps (iv) and
// (iii) of Sec. 3), one knot per thread, with the Roemer delay from the
// detector's tabulated trajectory (the interval read last kept in
// registers).  Three ranges of blocks:
//  - the first blocks solve the grid knots and turn each interval's two
//    end knots into its record (the cubic Hermite form of q between them,
//    relative to the integer part of the interval's first source position);
//  - knot_tile_blocks blocks (plans with res_taylor) solve the knot at each
//    tile's middle point again and write the tile's antenna Taylor record;
//  - the rest solve the sample knots.
// A delay beyond the plan's max_delay flags the template (as a tile whose
// delay leaves its staged nodes does).
template <bool GROUPED, bool KEP>
__global__ __launch_bounds__(kKnotThreads) void k_knots(PlanConst P, void* ws, ChunkMap map,
                                                        int slots) {
  const int gi = blockIdx.y;
  const int slot = GROUPED ? map.grp_slot[gi] : gi;
  const TmplParams& tp = *tmpl_params(ws, P, map, slot);
  if (GROUPED ? (tp.status & kStatusGroupMask) != 0 : tp.status != 0) return;
  const int kl = tp.knot_log2;
  if (kl < kKnotLogGlobal) return;
  int32_t* status_word = GROUPED ? group_status(ws, P, slots, map.grp_buf[gi])
                                 : &tmpl_params(ws, P, map, slot)->status;
  const int X = blockIdx.z;
  const DetConst& d = P.det[X];
  double2* kn = (GROUPED ? group_knots(ws, P, slots, map.grp_buf[gi]) : slot_knots(ws, P, slot)) +
                X * P.knot_stride;
  const int G = 1 << kl;
  const CachedRoemer re{d.ephem, tp.nhat, P.n_eph, P.eph_t0, P.eph_dt, P.inv_eph_dt};
  // blocks launched per range: enough for the coarsest spacing; a template
  // with a finer one walks its chunks of kKnotThreads - 1 knots in steps of
  // the range's block count
  int64_t scap = 0;
  for (int Y = 0; Y < P.ndet; ++Y) scap = max(scap, ((P.det[Y].n - 1) >> kKnotLogMax) + 2);
  const int64_t gblocks = knot_grid_blocks((P.k_pad >> kKnotLogMax) + 1);
  const int64_t tblocks = knot_tile_blocks(P.k_pad);
  const int64_t sblocks = knot_samp_blocks(scap);
  const int64_t b = blockIdx.x;
  __shared__ double2 nb[kKnotThreads];
  bool far = false;
  if (b < gblocks) {
    const int64_t last = P.k_pad >> kl;
    const int64_t chunks = knot_grid_blocks(last + 1);
    for (int64_t c = b; c < chunks; c += gblocks) {
      const int64_t e = c * (kKnotThreads - 1) + threadIdx.x;
      double2 kv = make_double2(0.0, 0.0);
      if (e <= last) {
        bool f;
        kv = grid_knot<KEP>(P, tp, re, e * G, f);
        far |= f;
      }
      nb[threadIdx.x] = kv;
      __syncthreads();
      if (threadIdx.x < kKnotThreads - 1 && e <= last) {
        double2 c0, c1;
        if (e < last) {
          hermite_interval(kv, nb[threadIdx.x + 1], double(G), c0, c1);
        } else {
          c0 = make_double2(kv.x, 0.0);
          c1 = make_double2(0.0, 0.0);
        }
        const double a = d.off + c0.x;
        const double fa = floor(a);
        reinterpret_cast<float4*>(kn)[e] =
            make_float4(float(a - fa), float(c0.y), float(c1.x), float(c1.y));
        reinterpret_cast<int32_t*>(kn + P.knot_ioff)[e] = int32_t(fa);
      }
      __syncthreads();
    }
  } else if (b < gblocks + tblocks) {
    const int64_t t = (b - gblocks) * kKnotThreads + threadIdx.x;
    if (P.res_taylor && t < (P.k_pad >> kResTileLog)) {
      // the tile's middle point is a knot (G divides half a tile)
      const int64_t k = (t << kResTileLog) + kResTile / 2;
      bool far_t;
      const double2 kv = grid_knot<KEP>(P, tp, re, k, far_t);
      float c[kTaylorCoef];
      antenna_taylor(tp, X, tp.alpha_cyc[X] - P.sid_rate_cyc * (P.tau0 + P.dt * double(k) +
                                                                kv.x * P.dt), c);
      const double a = d.off + kv.x;
      const double fa = floor(a);
      float* tr = reinterpret_cast<float*>(kn + P.knot_toff + t * kTileRecUnits);
#pragma unroll
      for (int n = 0; n < kTaylorCoef; ++n) tr[n] = c[n];
      tr[kTaylorCoef] = float(a - fa);
      tr[kTaylorCoef + 1] = __int_as_float(int32_t(fa));
    }
  } else {
    // sample knot m: heterodyne phase at t = t0 + m G dt and its change per
    // sample; the record of interval m from knots m and m + 1
    const int64_t last = ((d.n - 1) >> kl) + 1;
    const int64_t chunks = knot_samp_blocks(last + 1);
    for (int64_t c = b - gblocks - tblocks; c < chunks; c += sblocks) {
      const int64_t m = c * (kKnotThreads - 1) + threadIdx.x;
      double2 kv = make_double2(0.0, 0.0);
      if (m <= last) {
        double ph, dph, delay;
        sample_phase_d<KEP>(re, tp, d.t0 + P.dt * double(m * G), P.f_het, ph, dph, delay);
        kv = make_double2(ph, dph * P.dt);
        far |= !(fabs(delay) <= P.max_delay);
      }
      nb[threadIdx.x] = kv;
      __syncthreads();
      if (threadIdx.x < kKnotThreads - 1 && m < last) {
        double2 c0, c1;
        hermite_interval(kv, nb[threadIdx.x + 1], double(G), c0, c1);
        // in quarter turns and in t = u G (scalings by powers of two: exact)
        const double ig = 1.0 / double(G);
        double2* rec = kn + P.knot_soff + 2 * m;
        rec[0] = make_double2(fmod(4.0 * c0.x, 4.0), 4.0 * c0.y * ig);
        rec[1] = make_double2(4.0 * c1.x * ig * ig, 4.0 * c1.y * ig * ig * ig);
      }
      __syncthreads();
    }
  }
  if (far) atomicOr(status_word, kStatusNodes);
}

// Resampling kernels.  GROUPED = false: blockIdx.y is a template slot; the
// spin-down phase is applied and y_a', y_b' go to the slot's arrays 0 and 1.
// GROUPED = true: blockIdx.y is a sky/orbit group of the chunk; the series is
// written without the spin-down phase to the group's buffer, which every
// template of the group reads (the reuse of the sky-dependent barycentring
// across spin-down templates that Sec. 4.1 measures).
//
// Where a resampling block writes, and whether the template (group) is
// live: a leader whose sky or orbit is invalid invalidates the whole group
// (its status word tells every member's column pass not to read the buffer).
struct ResTarget {
  const TmplParams* tp;
  int32_t* status;
  float2* ya;
  float2* yb;
  const double2* kn;  // knot area (null: none)
  bool live;
};
template <bool GROUPED>
__device__ __forceinline__ ResTarget res_target(const PlanConst& P, void* ws, const ChunkMap& map,
                                                int slots) {
  const int gi = blockIdx.y;
  const int slot = GROUPED ? map.grp_slot[gi] : gi;
  ResTarget r;
  r.tp = tmpl_params(ws, P, map, slot);
  r.status = GROUPED ? group_status(ws, P, slots, map.grp_buf[gi])
                     : &tmpl_params(ws, P, map, slot)->status;
  r.ya = GROUPED ? group_buf(ws, P, slots, map.grp_buf[gi], 0) : slot_buf(ws, P, slot, 0);
  r.yb = GROUPED ? group_buf(ws, P, slots, map.grp_buf[gi], 1) : slot_buf(ws, P, slot, 1);
  r.kn = P.knot_bytes == 0 ? nullptr
         : GROUPED         ? group_knots(ws, P, slots, map.grp_buf[gi])
                           : slot_knots(ws, P, slot);
  r.live = true;
  if (GROUPED) {
    const int32_t gflag = r.tp->status & kStatusGroupMask;
    if (gflag != 0) {
      if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr(r.status, gflag);
      r.live = false;
    }
  } else if (r.tp->status != 0) {
    r.live = false;
  }
  return r;
}
// Whether a template's timing knots were solved ahead (k_knots).
__device__ __forceinline__ bool knots_ahead(const ResTarget& r) {
  return r.kn != nullptr && r.tp->knot_log2 >= kKnotLogGlobal;
}
template <bool GROUPED>
__device__ __forceinline__ void res_store(const ResTarget& r, int64_t k_s,
                                          const float2 (&acc_a)[kResPerThread],
                                          const float2 (&acc_b)[kResPerThread]) {
#pragma unroll
  for (int i = 0; i < kResPerThread; ++i) {
    const int64_t k = k_s + threadIdx.x + i * kResThreads;
    if (GROUPED) {
      r.ya[k] = acc_a[i];
      r.yb[k] = acc_b[i];
    } else {
      // spin-down phase and sub-bin offset: y = acc * exp(-2 pi i cyc)
      const float2 e = spindown_rotation(r.tp->sd, k);
      r.ya[k] = cmul_exact(acc_a[i], e);
      r.yb[k] = cmul_exact(acc_b[i], e);
    }
  }
}

// Templates whose knots were solved ahead: one tile per block.  Without the
// in-tile timing the kernel fits 96 registers without spills, five waves per
// SIMD, which covers the tile's memory latencies better (binary workload, per
// template: 102 us at four waves, 89 at five, 96 at six with 48 bytes
// spilled, 153 at eight).
template <int D, bool GROUPED>
__global__ __launch_bounds__(kResThreads, kResWavesAhead) void k_resample(PlanConst P, void* ws,
                                                                       ChunkMap map, int slots) {
  const ResTarget r = res_target<GROUPED>(P, ws, map, slots);
  if (!r.live || !knots_ahead(r)) return;
  __shared__ float2 zs[kDetPass * kResWcap];
  __shared__ int32_t blk[kDetPass * kResBlk];
  const int64_t k_s = int64_t(blockIdx.x) * kResTile;
  float2 acc_a[kResPerThread], acc_b[kResPerThread];
  if (!resample_tile_gk<D>(P, *r.tp, r.kn, r.status, k_s, zs, blk, acc_a, acc_b)) return;
  res_store<GROUPED>(r, k_s, acc_a, acc_b);
}

// The other templates (knot spacing below 16 points, or no knot area): the
// tile solves its own timing (four waves per SIMD, 128 registers: its FP64
// and LDS latency chains hide better with more waves).  A block walks tiles
// blockIdx.x, + gridDim.x, ..., so that a launch over templates that all had
// their knots solved ahead is a few thousand blocks that return at once.
template <int D, bool GROUPED, bool KEP>
__global__ __launch_bounds__(kResThreads, 4) void k_resample_own(PlanConst P, void* ws,
                                                               ChunkMap map, int slots) {
  const ResTarget r = res_target<GROUPED>(P, ws, map, slots);
  if (!r.live || knots_ahead(r)) return;
  __shared__ float2 zs[kDetPass * kResWcap];
  __shared__ int32_t blk[kDetPass * kResBlk];
  const int64_t tiles = P.k_pad / kResTile;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t k_s = t * kResTile;
    float2 acc_a[kResPerThread], acc_b[kResPerThread];
    if (!resample_tile<D, KEP>(P, *r.tp, r.status, k_s, zs, blk, acc_a, acc_b)) return;
    res_store<GROUPED>(r, k_s, acc_a, acc_b);
    // the next tile's first phase rewrites what this one's last read
    __syncthreads();
  }
}

// exp(-2 pi i nat k / N) with the product reduced exactly in integers.
__device__ inline float2 bin_twiddle(int64_t nat, int64_t k, int64_t n_fft) {
  return cis_neg_frac((nat * k) & (n_fft - 1), __builtin_ctzll(uint64_t(n_fft)));
}

// Natural FFT index of band bin i (bins ascend in frequency from bin_lo of
// the centred spectrum).
__host__ __device__ inline int64_t band_bin_nat(const PlanConst& P, int64_t i) {
  return (P.bin_lo + i + P.n_fft / 2) & (P.n_fft - 1);
}

// Single-bin forward path: the whitened transforms Fa'(m), Fb'(m) at one bin
// m per template as a direct sum over the grid, sum_k y'_k exp(-2 pi i m k/N)
// (step (vi) restricted to one output bin), reduced per tile into the slot's
// partials (Fa'.re, Fa'.im, Fb'.re, Fb'.im in FP64).
template <int D, bool KEP>
__global__ __launch_bounds__(kResThreads, 4) void k_resample_bin(PlanConst P, void* ws, ChunkMap map,
                                                             const int64_t* __restrict__ bins) {
  const int slot = blockIdx.y;
  TmplParams* tpp = slot_params(ws, P, slot);
  const TmplParams& tp = *tpp;
  double* partial = slot_partials(ws, P, slot) + size_t(blockIdx.x) * 8;
  const int64_t k_s = int64_t(blockIdx.x) * kResTile;
  const int tid = threadIdx.x;
  if (tp.status != 0) return;
  __shared__ float2 zs[kDetPass * kResWcap];
  __shared__ int32_t blk[kDetPass * kResBlk];
  float2 acc_a[kResPerThread], acc_b[kResPerThread];
  if (!resample_tile<D, KEP>(P, tp, &tpp->status, k_s, zs, blk, acc_a, acc_b)) return;
  const int64_t bin = bins[map.tmpl[slot]];
  const int64_t nat = band_bin_nat(P, bin);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < kResPerThread; ++i) {
    const int64_t k = k_s + tid + i * kResThreads;
    const float2 e = cmul(spindown_rotation(tp.sd, k),
                          bin_twiddle(nat, k, P.n_fft));
    const float2 ya = cmul(acc_a[i], e), yb = cmul(acc_b[i], e);
    s[0] += double(ya.x);
    s[1] += double(ya.y);
    s[2] += double(yb.x);
    s[3] += double(yb.y);
  }
  __shared__ double red[kResThreads / 64][4];
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double v = s[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  if (tid < 4) {
    double v = 0.0;
    for (int w = 0; w < kResThreads / 64; ++w) v += red[w][tid];
    partial[tid] = v;
  }
}

// Per-template totals of per-tile partials (8 doubles per tile, the first
// NQ used) by one workgroup: each thread sums a fixed stripe of tiles, then a
// fixed tree combines the threads, so a template's totals come out the same
// on every run.  The totals land in s of thread 0.
constexpr int kFinalThreads = 256;
template <int NQ>
__device__ inline void tile_sums(const double* __restrict__ part, int64_t ntiles, double (&s)[NQ]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NQ; ++q) s[q] = 0.0;
  for (int64_t b = tid; b < ntiles; b += kFinalThreads)
#pragma unroll
    for (int q = 0; q < NQ; ++q) s[q] += part[b * 8 + q];
  __shared__ double red[NQ][kFinalThreads];
#pragma unroll
  for (int q = 0; q < NQ; ++q) red[q][tid] = s[q];
  __syncthreads();
  for (int off = kFinalThreads / 2; off > 0; off >>= 1) {
    if (tid < off)
#pragma unroll
      for (int q = 0; q < NQ; ++q) red[q][tid] += red[q][tid + off];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) s[q] = red[q][0];
}

// Per template: Fa'(m), Fb'(m) from the tile partials (tile order), 2F at the
// bin, and the adjoint spectrum of L = 2F(m) at that bin, H = conj(F'(m))
// (kept in the parameter block for the gradient kernel).  A bin outside the
// band flags the template.
__global__ __launch_bounds__(kFinalThreads) void k_bin_final(PlanConst P, void* ws, ChunkMap map,
                                                             int64_t ntiles,
                                                             const int64_t* __restrict__ bins,
                                                             float* __restrict__ twoF) {
  const int slot = blockIdx.x;
  double f[4];
  tile_sums<4>(slot_partials(ws, P, slot), ntiles, f);
  if (threadIdx.x != 0) return;
  TmplParams& tp = *slot_params(ws, P, slot);
  const int64_t bin = bins[map.tmpl[slot]];
  if (bin < 0 || bin >= P.n_bins) tp.status |= kStatusBin;
  if (tp.status != 0) atomicAdd(flag_counter(ws), 1ull);
  tp.bin_nat = band_bin_nat(P, bin);
  tp.hbin[0] = f[0];
  tp.hbin[1] = -f[1];
  tp.hbin[2] = f[2];
  tp.hbin[3] = -f[3];
  const double v = 2.0 * (f[0] * f[0] + f[1] * f[1] + f[2] * f[2] + f[3] * f[3]);
  if (twoF) twoF[map.tmpl[slot]] = tp.status != 0 ? __builtin_nanf("") : float(v);
}

}  // namespace fstat
