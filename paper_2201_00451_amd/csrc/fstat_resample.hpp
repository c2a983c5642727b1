// Steps (iii)-(v) of Sec. 3 and the weighting of step (vi), fused.
//
// One workgroup owns kResTile consecutive points of the regular source-frame
// grid tau_k = tau0 + k dt of one template.  For each detector it
//   1. stages the ephemeris nodes the tile can touch in LDS, projected on the
//      sky direction once per node (n.r, n.v), so every later delay
//      evaluation is a cubic Hermite on LDS data;
//   2. solves the detector epochs T_k of step (iv) for the thread's own grid
//      points (FP64); T_k is monotonic in k, so the first and last points of
//      the tile bound the input samples its interpolation windows touch;
//   3. stages those samples in LDS after the step (iii) heterodyne correction
//      z_j = x_j exp(-2 pi i f_h (t_src,j - t_j)) (FP64 delay, reduced to
//      [-1/2, 1/2] cycles, FP32 rotation): each input sample is read from HBM
//      and corrected once per tile;
//   4. interpolates z at T_k with the 2D-tap Hann-windowed sinc
//      h(s) = sinc(s) (1 + cos(pi s / D)) / 2 (the paper leaves the kernel of
//      step (v) unnamed) and accumulates w_X a'(T_k) zhat_k, w_X b'(T_k) zhat_k
//      with the whitened antenna patterns of the template.
// Finally it removes the spin-down phase Phi_s(tau_k) and the sub-bin offset
// df (FP64 phase, FP32 rotation) and writes y_a', y_b' (float2) with
// coalesced stores.  FP64 is used only for times and phases.
#pragma once

#include "fstat_common.hpp"

namespace fstat {

__global__ __launch_bounds__(kResThreads) void k_resample(PlanConst P, void* ws) {
  const int g = blockIdx.y;
  TmplParams* tpp = slot_params(ws, P.n_fft, g);
  const TmplParams& tp = *tpp;
  float2* ya = slot_buf(ws, P.n_fft, g, 0);
  float2* yb = slot_buf(ws, P.n_fft, g, 1);
  const int64_t k_s = int64_t(blockIdx.x) * kResTile;
  const int tid = threadIdx.x;

  __shared__ float2 zs[kResWcap];
  __shared__ double2 nodes[kNodeCap];
  __shared__ float tap_c[64], tap_s[64];
  __shared__ int64_t win_lo, win_hi;
  __shared__ int bad;

  const int D = P.D;
  if (tp.status != 0) {
    for (int i = 0; i < kResPerThread; ++i) {
      int64_t k = k_s + tid + i * kResThreads;
      ya[k] = make_float2(0.f, 0.f);
      yb[k] = make_float2(0.f, 0.f);
    }
    return;
  }
  // cos, sin of pi (D - 1 - t) / D for the window's angle addition
  if (tid < 2 * D) {
    float s, c;
    sincospif(float(D - 1 - tid) / float(D), &s, &c);
    tap_c[tid] = c;
    tap_s[tid] = s;
  }
  if (tid == 0) bad = 0;
  bool oob = false;
  float2 acc_a[kResPerThread], acc_b[kResPerThread];
  for (int i = 0; i < kResPerThread; ++i) {
    acc_a[i] = make_float2(0.f, 0.f);
    acc_b[i] = make_float2(0.f, 0.f);
  }
  // time span any delay evaluation of this tile can reach
  const double pad = P.max_delay + double(D + 2) * P.dt;
  const double t_first = P.tau0 + P.dt * double(k_s) - pad;
  const double t_last = P.tau0 + P.dt * double(k_s + kResTile - 1) + pad;
  int64_t n_lo = int64_t(floor((t_first - P.eph_t0) * P.inv_eph_dt)) - 1;
  n_lo = n_lo < 0 ? 0 : (n_lo > P.n_eph - 2 ? P.n_eph - 2 : n_lo);
  int64_t n_hi = int64_t(floor((t_last - P.eph_t0) * P.inv_eph_dt)) + 2;
  n_hi = n_hi > P.n_eph - 1 ? P.n_eph - 1 : n_hi;
  int n_count = int(n_hi - n_lo + 1);
  n_count = n_count > kNodeCap ? kNodeCap : (n_count < 2 ? 2 : n_count);
  const NodeRoemer re{nodes, n_count, P.eph_t0 + double(n_lo) * P.eph_dt, P.eph_dt, P.inv_eph_dt};

  for (int X = 0; X < P.ndet; ++X) {
    const DetConst& d = P.det[X];
    // 1. projected ephemeris nodes
    for (int i = tid; i < n_count; i += kResThreads) {
      const double* e = d.ephem + 6 * (n_lo + i);
      nodes[i] = make_double2(tp.nhat[0] * e[0] + tp.nhat[1] * e[1] + tp.nhat[2] * e[2],
                              tp.nhat[0] * e[3] + tp.nhat[1] * e[4] + tp.nhat[2] * e[5]);
    }
    __syncthreads();
    // 2. detector epochs of this thread's grid points
    double dly[kResPerThread];
    int64_t j0[kResPerThread];
    float fr[kResPerThread];
    for (int i = 0; i < kResPerThread; ++i) {
      const int64_t k = k_s + tid + i * kResThreads;
      dly[i] = grid_delay(re, tp, P.tau0 + P.dt * double(k), oob);
      split_u(double(k) + d.off + dly[i] * P.inv_dt, j0[i], fr[i]);
    }
    if (tid == 0) win_lo = j0[0] - D + 1;
    if (tid == kResThreads - 1) win_hi = j0[kResPerThread - 1] + D;
    __syncthreads();
    const int64_t lo = win_lo;
    const int64_t nwin = win_hi - lo + 1;
    if (nwin > kResWcap || nwin < 1) {
      // delay drift beyond 1/16 per tile: flag the template (NaN output)
      if (tid == 0) atomicOr(&tpp->status, 4);
      return;
    }
    const int W = int(nwin);
    // 3. corrected input samples
    for (int w = tid; w < W; w += kResThreads) {
      int64_t j = lo + w;
      float2 z = make_float2(0.f, 0.f);
      if (j >= 0 && j < d.n) {
        float2 xv = d.x[j];
        double dl = sample_delay(re, tp, d.t0 + P.dt * double(j), oob);
        float c = reduce_cycles(P.f_het * dl);
        float sn, cs;
        sincospif(2.0f * c, &sn, &cs);
        // x * exp(-2 pi i c)
        z = make_float2(xv.x * cs + xv.y * sn, xv.y * cs - xv.x * sn);
      }
      zs[w] = z;
    }
    __syncthreads();
    // 4. interpolation and antenna weighting
    const float inv_pi = 0.318309886183790671f;
    for (int i = 0; i < kResPerThread; ++i) {
      const int64_t k = k_s + tid + i * kResThreads;
      const float f = fr[i];
      float2 zh = make_float2(0.f, 0.f);
      const int64_t base = j0[i] - D + 1 - lo;
      if (f == 0.0f) {
        int64_t idx = j0[i] - lo;
        idx = idx < 0 ? 0 : (idx >= W ? W - 1 : idx);
        zh = zs[idx];
      } else {
        const float sp = sinpif(f) * inv_pi;
        float ws_, wc_;
        sincospif(f / float(D), &ws_, &wc_);
        for (int t = 0; t < 2 * D; ++t) {
          const float s = f + float(D - 1 - t);
          const float win = 0.5f + 0.5f * (wc_ * tap_c[t] - ws_ * tap_s[t]);
          const float h = (((D - 1 - t) & 1) ? -sp : sp) * __builtin_amdgcn_rcpf(s) * win;
          int64_t idx = base + t;
          idx = idx < 0 ? 0 : (idx >= W ? W - 1 : idx);
          const float2 zv = zs[idx];
          zh.x += h * zv.x;
          zh.y += h * zv.y;
        }
      }
      // antenna patterns at T_k: x = alpha - phi(T_k), in cycles
      const double tau = P.tau0 + P.dt * double(k);
      const float xc = reduce_cycles(tp.alpha_cyc[X] - P.sid_rate_cyc * (tau + dly[i]));
      float sx, cx;
      sincospif(2.0f * xc, &sx, &cx);
      const float c2 = cx * cx - sx * sx, s2 = 2.0f * sx * cx;
      const float a = tp.ca[X][0] + tp.ca[X][1] * cx + tp.ca[X][2] * sx + tp.ca[X][3] * c2 +
                      tp.ca[X][4] * s2;
      const float b = tp.cb[X][0] + tp.cb[X][1] * cx + tp.cb[X][2] * sx + tp.cb[X][3] * c2 +
                      tp.cb[X][4] * s2;
      acc_a[i].x += a * zh.x;
      acc_a[i].y += a * zh.y;
      acc_b[i].x += b * zh.x;
      acc_b[i].y += b * zh.y;
    }
    __syncthreads();
  }
  if (oob) bad = 1;
  __syncthreads();
  if (bad) {
    // a delay evaluation left the staged ephemeris nodes: the delay exceeds
    // the plan's max_delay; flag the template (NaN output)
    if (tid == 0) atomicOr(&tpp->status, 8);
    return;
  }
  // spin-down phase and sub-bin offset: y = acc * exp(-2 pi i cyc)
  for (int i = 0; i < kResPerThread; ++i) {
    const int64_t k = k_s + tid + i * kResThreads;
    const double tau = P.tau0 + P.dt * double(k);
    const double dtr = tau - P.t_ref;
    double cyc = tp.f1dot * dtr * dtr * 0.5 + tp.f2dot * dtr * dtr * dtr * (1.0 / 6.0);
    cyc = cyc - rint(cyc) + tp.df * (P.dt * double(k));
    const float c = reduce_cycles(cyc);
    float sn, cs;
    sincospif(2.0f * c, &sn, &cs);
    const float2 e = make_float2(cs, -sn);
    ya[k] = cmul(acc_a[i], e);
    yb[k] = cmul(acc_b[i], e);
  }
}

}  // namespace fstat
