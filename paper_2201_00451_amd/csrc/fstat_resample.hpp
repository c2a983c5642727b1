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

// Steps (iii)-(v) and the antenna weighting for the kResTile grid points of
// the tile starting at k_s: acc_a[i], acc_b[i] receive sum_X a'_X(T_k)
// zhat_X(u_k) (and b'), k = k_s + tid + i kResThreads, before the spin-down
// phase.  Returns false, after flagging the template's status word, when the
// template must report NaN (the return is uniform across the block).
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
                                     int32_t* status_word, int64_t k_s,
                                     float2 (&acc_a)[kResPerThread],
                                     float2 (&acc_b)[kResPerThread]) {
  const int tid = threadIdx.x;
  __shared__ float2 zs[kResWcap];
  __shared__ double2 coef[2 * kNodeCap];
  __shared__ double2 knot[kSampKnots];           // knot values and derivatives
  __shared__ double2 gc[2 * (kGridKnots - 1)];   // grid-delay intervals
  __shared__ double2 sc[2 * (kSampKnots - 1)];   // sample-phase intervals
  __shared__ int32_t blk[(kResWcap + kResThreads) / 32 + 2];
  __shared__ int64_t win_lo, win_hi;
  __shared__ int bad;

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
  const CubicRoemer re{coef, n_count, P.eph_t0 + double(n_lo) * P.eph_dt, P.inv_eph_dt};
  const double tau_s = P.tau0 + P.dt * double(k_s);
  // the binary delay depends on the grid point only: once for all detectors
  // (at the own grid knot, with its rate, or at the own grid points)
  double rb0 = 0.0, rbd0 = 0.0;
  double rbk[kResPerThread];
  if (knots) {
    if (tid < nkg) orbit_delay<KEP>(tp, tau_s + P.dt * double(tid * G), rb0, rbd0);
  } else {
    rb0 = binary_delay<KEP>(tp, tau_s);
#pragma unroll
    for (int i = 0; i < kResPerThread; ++i)
      rbk[i] = binary_delay<KEP>(tp, tau_s + P.dt * double(tid + i * kResThreads));
  }

  for (int X = 0; X < P.ndet; ++X) {
    const DetConst& d = P.det[X];
    // 1. interval coefficients from the projected nodes i and i + 1
    for (int i = tid; i < n_count - 1; i += kResThreads) {
      const double* e = d.ephem + 6 * (n_lo + i);
      const double p0 = tp.nhat[0] * e[0] + tp.nhat[1] * e[1] + tp.nhat[2] * e[2];
      const double v0 = tp.nhat[0] * e[3] + tp.nhat[1] * e[4] + tp.nhat[2] * e[5];
      const double p1 = tp.nhat[0] * e[6] + tp.nhat[1] * e[7] + tp.nhat[2] * e[8];
      const double v1 = tp.nhat[0] * e[9] + tp.nhat[1] * e[10] + tp.nhat[2] * e[11];
      cubic_interval(p0, v0, p1, v1, P.eph_dt, coef[2 * i], coef[2 * i + 1]);
    }
    __syncthreads();
    // 2. detector epochs of the own grid points as q = (T - tau)/dt and
    // u = (T - t0)/dt = k + off + q
    double q[kResPerThread];
    int64_t j0[kResPerThread];
    float fr[kResPerThread];
    if (knots) {
      // exact solves at the grid knots (fixed point and three Newton steps),
      // with dq/dk = d(T - tau)/dtau = (R'(tau) - roemer'(T)) / (1 + roemer'(T))
      if (tid < nkg) {
        const double tau = tau_s + P.dt * double(tid * G);
        double x;
        double dl = grid_delay<KEP>(re, tp, tau, oob);
        dl = grid_delay_newton(re, tau, rb0, dl, x, oob);
        dl = grid_delay_newton(re, tau, rb0, dl, x, oob);
        knot[tid] = make_double2(dl * P.inv_dt, (rbd0 - x) / (1.0 + x));
      }
      __syncthreads();
      if (tid < nkg - 1) hermite_interval(knot[tid], knot[tid + 1], double(G), gc[2 * tid],
                                          gc[2 * tid + 1]);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kResPerThread; ++i) {
        const int kk = tid + i * kResThreads;
        q[i] = hermite_eval(gc, kk >> kl, double(kk & (G - 1)) * inv_g);
        split_u(double(k_s + kk) + d.off + q[i], j0[i], fr[i]);
      }
    } else {
      // the tile's first point in full (fixed point, two Newton steps), the
      // rest by one Newton step from a prediction that carries the exact
      // binary delay and linearises the Roemer delay about the first point:
      // T ~ T_s + (t_b - t_b,s) / (1 + roemer'(T_s))
      double x0;
      double d0 = grid_delay<KEP>(re, tp, tau_s, oob);
      d0 = grid_delay_newton(re, tau_s, rb0, d0, x0, oob);
      d0 = grid_delay_newton(re, tau_s, rb0, d0, x0, oob);
      const double inv0 = 1.0 - x0 * (1.0 - x0 * (1.0 - x0));
#pragma unroll
      for (int i = 0; i < kResPerThread; ++i) {
        const int64_t kk = tid + i * kResThreads;
        const double dtau = P.dt * double(kk);
        const double tau = tau_s + dtau;
        const double rb = rbk[i];
        const double guess = d0 + (dtau + rb - rb0) * inv0 - dtau;
        double x;
        q[i] = grid_delay_newton(re, tau, rb, guess, x, oob) * P.inv_dt;
        split_u(double(k_s + kk) + d.off + q[i], j0[i], fr[i]);
      }
    }
    if (tid == 0) win_lo = j0[0] - D + 1;
    if (tid == kResThreads - 1) win_hi = j0[kResPerThread - 1] + D;
    __syncthreads();
    const int64_t lo = win_lo;
    const int64_t nwin = win_hi - lo + 1;
    if (nwin > kResWcap || nwin < 2 * D) {
      // delay drift beyond 1/16 per tile: flag the template (NaN output)
      if (tid == 0) atomicOr(status_word, kStatusWindow);
      return false;
    }
    const int W = int(nwin);
    // 3. corrected input samples: knots of the heterodyne phase first
    if (knots) {
      const int nks = ((W - 1) >> kl) + 2;
      if (tid < nks) {
        double ph, dph;
        sample_phase<KEP>(re, tp, d.t0 + P.dt * double(lo + int64_t(tid) * G), P.f_het, ph, dph,
                     oob);
        knot[tid] = make_double2(ph, dph * P.dt);
      }
      __syncthreads();
      if (tid < nks - 1) hermite_interval(knot[tid], knot[tid + 1], double(G), sc[2 * tid],
                                          sc[2 * tid + 1]);
      __syncthreads();
    }
    for (int w0 = 0; w0 < W; w0 += kResThreads) {
      const int w = w0 + tid;
      const int64_t j = lo + w;
      const float2 xv = (w < W && j >= 0 && j < d.n) ? d.x[j] : make_float2(0.f, 0.f);
      // a zero sample (outside the data, or in a gap) stays zero: no timing
      const bool live = xv.x != 0.f || xv.y != 0.f;
      float2 z = make_float2(0.f, 0.f);
      if (live) {
        const double ph = knots ? hermite_eval(sc, w >> kl, double(w & (G - 1)) * inv_g)
                                : P.f_het * sample_delay<KEP>(re, tp, d.t0 + P.dt * double(j), oob);
        const float2 e = cis_cycles(ph);
        // x * exp(-2 pi i f_h dl)
        z = make_float2(xv.x * e.x + xv.y * e.y, xv.y * e.x - xv.x * e.y);
      }
      if (w < W) zs[w] = z;
      // which 32-sample blocks of the window hold a live sample
      const unsigned long long m = __ballot(live);
      if ((tid & 63) == 0) {
        const int b = (w0 + tid) >> 5;
        blk[b] = uint32_t(m) != 0u;
        blk[b + 1] = uint32_t(m >> 32) != 0u;
      }
    }
    __syncthreads();
    // 4. interpolation and antenna weighting
#pragma unroll
    for (int i = 0; i < kResPerThread; ++i) {
      const float f = fr[i];
      // taps j0-D+1 .. j0+D; monotonic T_k keeps them inside the window,
      // the clamp only guards memory
      int base = int(j0[i] - lo) - (D - 1);
      base = base < 0 ? 0 : (base > W - 2 * D ? W - 2 * D : base);
      if (!(blk[base >> 5] | blk[(base + 2 * D - 1) >> 5])) continue;
      const float2* zp = zs + base;
      float2 zh;
      if (f == 0.0f) {
        zh = zp[D - 1];
      } else {
        // window phase pi f / D and sinc numerator sin(pi f), in cycles
        const float2 wcs = cis_cycles_f32(f * (0.5f / float(D)));
        float sx = 0.f, sy = 0.f;
        interp_taps<D>(std::make_integer_sequence<int, 2 * D>{}, f, wcs.x, wcs.y, zp, sx, sy);
        const float sp = cis_cycles_f32(0.5f * f).y * float(0.5 / kPi);
        zh = make_float2(sx * sp, sy * sp);
      }
      // antenna patterns at T_k: x = alpha - phi(T_k), in cycles
      const double tau = tau_s + P.dt * double(tid + i * kResThreads);
      const float2 ex = cis_cycles(tp.alpha_cyc[X] - P.sid_rate_cyc * (tau + q[i] * P.dt));
      const float cx = ex.x, sx = ex.y;
      const float c2 = cx * cx - sx * sx, s2 = 2.0f * sx * cx;
      const float a = tp.ca[X][0] + tp.ca[X][1] * cx + tp.ca[X][2] * sx + tp.ca[X][3] * c2 +
                      tp.ca[X][4] * s2;
      const float b = tp.cb[X][0] + tp.cb[X][1] * cx + tp.cb[X][2] * sx + tp.cb[X][3] * c2 +
                      tp.cb[X][4] * s2;
      acc_a[i].x = fmaf(a, zh.x, acc_a[i].x);
      acc_a[i].y = fmaf(a, zh.y, acc_a[i].y);
      acc_b[i].x = fmaf(b, zh.x, acc_b[i].x);
      acc_b[i].y = fmaf(b, zh.y, acc_b[i].y);
    }
    __syncthreads();
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

// GROUPED = false: blockIdx.y is a template slot; the spin-down phase is
// applied and y_a', y_b' go to the slot's arrays 0 and 1.  GROUPED = true:
// blockIdx.y is a sky/orbit group of the chunk; the series is written without
// the spin-down phase to the group's buffer, which every template of the
// group reads (the reuse of the sky-dependent barycentring across spin-down
// templates that Sec. 4.1 measures).
// Four waves per SIMD (at most 128 registers, no spills at two outputs per
// thread): the timing's FP64 and LDS latency chains hide better with more
// waves (measured at 1024-point tiles: three waves against two, 11 % on sky
// positions and 17 % on binary orbits).
template <int D, bool GROUPED, bool KEP>
__global__ __launch_bounds__(kResThreads, 4) void k_resample(PlanConst P, void* ws, ChunkMap map,
                                                         int slots) {
  const int gi = blockIdx.y;
  const int slot = GROUPED ? map.grp_slot[gi] : gi;
  const TmplParams& tp = *tmpl_params(ws, P, map, slot);
  int32_t* status_word = GROUPED ? group_status(ws, P, slots, map.grp_buf[gi])
                                 : &tmpl_params(ws, P, map, slot)->status;
  float2* ya = GROUPED ? group_buf(ws, P, slots, map.grp_buf[gi], 0)
                       : slot_buf(ws, P, slot, 0);
  float2* yb = GROUPED ? group_buf(ws, P, slots, map.grp_buf[gi], 1)
                       : slot_buf(ws, P, slot, 1);
  const int64_t k_s = int64_t(blockIdx.x) * kResTile;
  if (GROUPED) {
    // a leader whose sky or orbit is invalid invalidates the whole group:
    // its status word tells every member's column pass not to read the buffer
    const int32_t gflag = tp.status & kStatusGroupMask;
    if (gflag != 0) {
      if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr(status_word, gflag);
      return;
    }
  } else if (tp.status != 0) {
    return;
  }
  float2 acc_a[kResPerThread], acc_b[kResPerThread];
  if (!resample_tile<D, KEP>(P, tp, status_word, k_s, acc_a, acc_b)) return;
#pragma unroll
  for (int i = 0; i < kResPerThread; ++i) {
    const int64_t k = k_s + threadIdx.x + i * kResThreads;
    if (GROUPED) {
      ya[k] = acc_a[i];
      yb[k] = acc_b[i];
    } else {
      // spin-down phase and sub-bin offset: y = acc * exp(-2 pi i cyc)
      const float2 e = spindown_rotation(tp.sd, k);
      ya[k] = cmul_exact(acc_a[i], e);
      yb[k] = cmul_exact(acc_b[i], e);
    }
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
  float2 acc_a[kResPerThread], acc_b[kResPerThread];
  if (!resample_tile<D, KEP>(P, tp, &tpp->status, k_s, acc_a, acc_b)) return;
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

// Per template: Fa'(m), Fb'(m) from the tile partials (tile order), 2F at the
// bin, and the adjoint spectrum of L = 2F(m) at that bin, H = conj(F'(m))
// (kept in the parameter block for the gradient kernel).  A bin outside the
// band flags the template.
__global__ void k_bin_final(PlanConst P, void* ws, ChunkMap map, int64_t ntiles,
                            const int64_t* __restrict__ bins, float* __restrict__ twoF) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= map.n_tmpl) return;
  TmplParams& tp = *slot_params(ws, P, slot);
  const double* part = slot_partials(ws, P, slot);
  const int64_t bin = bins[map.tmpl[slot]];
  if (bin < 0 || bin >= P.n_bins) tp.status |= kStatusBin;
  if (tp.status != 0) atomicAdd(flag_counter(ws), 1ull);
  double f[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t b = 0; b < ntiles; ++b)
    for (int q = 0; q < 4; ++q) f[q] += part[b * 8 + q];
  tp.bin_nat = band_bin_nat(P, bin);
  tp.hbin[0] = f[0];
  tp.hbin[1] = -f[1];
  tp.hbin[2] = f[2];
  tp.hbin[3] = -f[3];
  const double v = 2.0 * (f[0] * f[0] + f[1] * f[1] + f[2] * f[2] + f[3] * f[3]);
  if (twoF) twoF[map.tmpl[slot]] = tp.status != 0 ? __builtin_nanf("") : float(v);
}

}  // namespace fstat
