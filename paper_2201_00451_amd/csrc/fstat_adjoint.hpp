// Adjoint of the resampling F-statistic: the gradient of L = sum_m g_m 2F_m
// with respect to theta = (df, f1dot, alpha, delta, asini, porb, tp).
//
// With y' the whitened weighted series and F' = FFT(y') (2F = 2 |F'|^2),
//   dL/dtheta = 4 Re sum_k X_k dy'_k/dtheta,  X = FFT(g conj(F')),
// so the adjoint runs the forward path again (nothing is stored between the
// forward and the backward call), forms g conj(F') in the row pass, runs the
// two FFT passes on it, and then one kernel recomputes y'_k together with its
// derivatives at every grid point and reduces 4 Re(X_k dy'_k) per template.
//
// y'_k = E_k sum_X [a'_X(T_k) zhat_X(u_k)] (same for b'), E_k the spin-down
// and sub-bin rotation, zhat(u) = sum_j h(u - j) z_j, z_j = x_j
// exp(-2 pi i f_h delta_j), delta_j = t_src,j - t_j, u_k = (T_k - t0)/dt.
// For the sky and orbit parameters:
//   dT_k    = (dR(tau_k) - d roemer(T_k)) / (1 + roemer'(T_k))       (step iv)
//   ddelta_j = (d roemer(t_j) - dR(t_src,j)) / (1 + R'(t_src,j))     (step iii)
//   d zhat  = sum_j h'(u - j) z_j du + sum_j h(u - j) (-2 pi i f_h ddelta_j) z_j
//   d a'    = (d a'/d theta at fixed x) + (d a'/dx) (d alpha - Omega dT)
// where d roemer = r . d nhat, dR the explicit orbit derivatives; for df and
// f1dot only E_k depends on theta.  Isolated templates (asini = 0) report zero
// orbit derivatives.  For alpha and delta a constant (the parameter block's
// dshift) is taken off d delta_j: its contribution to the gradient is exactly
// zero, and without it the large constant sky phase derivative would cancel
// in FP32 arithmetic.
#pragma once

#include "fstat_common.hpp"
#include "fstat_resample.hpp"

namespace fstat {

// Three sky projections of the staged ephemeris nodes: nhat (value and time
// derivative) and d nhat / d alpha, d nhat / d delta (values).
struct NodeRoemer3 {
  const double2* n0;
  const double2* na;
  const double2* nd;
  int count;
  double t0, h, inv_h;
  __device__ void operator()(double t, double& d, double& dd, double& da, double& ddel,
                             bool& oob) const {
    double s = (t - t0) * inv_h;
    double fl = floor(s);
    int i = static_cast<int>(fmin(fmax(fl, -1.0), double(count)));
    if (i < 0 || i > count - 2) {
      oob = true;
      i = i < 0 ? 0 : count - 2;
    }
    const double u = s - double(i), u2 = u * u, u3 = u2 * u;
    const double h00 = 2.0 * u3 - 3.0 * u2 + 1.0, h10 = (u3 - 2.0 * u2 + u) * h;
    const double h01 = -2.0 * u3 + 3.0 * u2, h11 = (u3 - u2) * h;
    const double g0 = (6.0 * u2 - 6.0 * u) * inv_h, g1 = 3.0 * u2 - 4.0 * u + 1.0,
                 g3 = 3.0 * u2 - 2.0 * u;
    const double2 a = n0[i], b = n0[i + 1];
    d = h00 * a.x + h10 * a.y + h01 * b.x + h11 * b.y;
    dd = g0 * (a.x - b.x) + g1 * a.y + g3 * b.y;
    const double2 pa = na[i], pb = na[i + 1];
    da = h00 * pa.x + h10 * pa.y + h01 * pb.x + h11 * pb.y;
    const double2 qa = nd[i], qb = nd[i + 1];
    ddel = h00 * qa.x + h10 * qa.y + h01 * qb.x + h11 * qb.y;
  }
};

constexpr int kGradParams = 7;  // df, f1dot, alpha, delta, asini, porb, tp

// ONEHOT = false: X comes from the transformed adjoint spectrum (arrays 0
// and 1 hold conj(X)).  ONEHOT = true (single-bin path): L = 2F(m) at one bin
// m, so H is non-zero only at m and X_k = H_m exp(-2 pi i m k / N) in closed
// form; the slot holds no arrays.
// Two waves per SIMD (249 registers at two outputs per thread, no spills).
template <int D, bool ONEHOT, bool KEP>
__global__ __launch_bounds__(kResThreads, 2) void k_grad(PlanConst P, void* ws) {
  const int slot = blockIdx.y;
  const TmplParams& tp = *slot_params(ws, P, slot);
  double* partial = slot_partials(ws, P, slot) + size_t(blockIdx.x) * 8;
  const int64_t k_s = int64_t(blockIdx.x) * kResTile;
  const int tid = threadIdx.x;

  __shared__ float2 zs[kResWcap];
  // the staged samples times their five delay derivatives (one product per
  // sample instead of one per tap)
  __shared__ float2 zqs[5][kResWcap];
  __shared__ double2 nodes[3][kNodeCap];
  __shared__ int64_t win_lo, win_hi;
  __shared__ int bad;
  __shared__ double red[kResThreads / 64][kGradParams];

  if (tp.status != 0) {
    if (tid < 8) partial[tid] = 0.0;
    return;
  }
  if (tid == 0) bad = 0;
  bool oob = false;
  const bool binary = tp.asini != 0.0;

  // adjoint weights W_k = X_k E_k (the conjugate pass stored conj(X))
  float2 Wa[kResPerThread], Wb[kResPerThread];
#pragma unroll
  for (int i = 0; i < kResPerThread; ++i) {
    const int64_t k = k_s + tid + i * kResThreads;
    const float2 e = spindown_rotation(tp.sd, k);
    if (ONEHOT) {
      const float2 tw = bin_twiddle(tp.bin_nat, k, P.n_fft);
      Wa[i] = cmul(cmul(make_float2(float(tp.hbin[0]), float(tp.hbin[1])), tw), e);
      Wb[i] = cmul(cmul(make_float2(float(tp.hbin[2]), float(tp.hbin[3])), tw), e);
    } else {
      const float2 ya = slot_buf(ws, P, slot, 0)[k], yb = slot_buf(ws, P, slot, 1)[k];
      Wa[i] = cmul(make_float2(ya.x, -ya.y), e);
      Wb[i] = cmul(make_float2(yb.x, -yb.y), e);
    }
  }
  double acc[kGradParams];
#pragma unroll
  for (int q = 0; q < kGradParams; ++q) acc[q] = 0.0;

  const double pad = P.max_delay + double(D + 2) * P.dt;
  const double t_first = P.tau0 + P.dt * double(k_s) - pad;
  const double t_last = P.tau0 + P.dt * double(k_s + kResTile - 1) + pad;
  int64_t n_lo = int64_t(floor((t_first - P.eph_t0) * P.inv_eph_dt)) - 1;
  n_lo = n_lo < 0 ? 0 : (n_lo > P.n_eph - 2 ? P.n_eph - 2 : n_lo);
  int64_t n_hi = int64_t(floor((t_last - P.eph_t0) * P.inv_eph_dt)) + 2;
  n_hi = n_hi > P.n_eph - 1 ? P.n_eph - 1 : n_hi;
  int n_count = int(n_hi - n_lo + 1);
  n_count = n_count > kNodeCap ? kNodeCap : (n_count < 2 ? 2 : n_count);
  const double node_t0 = P.eph_t0 + double(n_lo) * P.eph_dt;
  const NodeRoemer re{nodes[0], n_count, node_t0, P.eph_dt, P.inv_eph_dt};
  const NodeRoemer3 re3{nodes[0], nodes[1], nodes[2], n_count, node_t0, P.eph_dt, P.inv_eph_dt};
  const double tau_s = P.tau0 + P.dt * double(k_s);
  const double omega = 2.0 * kPi * P.sid_rate_cyc;
  const float two_pi_fh = float(2.0 * kPi * P.f_het);

  for (int X = 0; X < P.ndet; ++X) {
    const DetConst& d = P.det[X];
    for (int i = tid; i < n_count; i += kResThreads) {
      const double* e = d.ephem + 6 * (n_lo + i);
      nodes[0][i] = make_double2(tp.nhat[0] * e[0] + tp.nhat[1] * e[1] + tp.nhat[2] * e[2],
                                 tp.nhat[0] * e[3] + tp.nhat[1] * e[4] + tp.nhat[2] * e[5]);
      nodes[1][i] = make_double2(
          tp.dnhat[0][0] * e[0] + tp.dnhat[0][1] * e[1] + tp.dnhat[0][2] * e[2],
          tp.dnhat[0][0] * e[3] + tp.dnhat[0][1] * e[4] + tp.dnhat[0][2] * e[5]);
      nodes[2][i] = make_double2(
          tp.dnhat[1][0] * e[0] + tp.dnhat[1][1] * e[1] + tp.dnhat[1][2] * e[2],
          tp.dnhat[1][0] * e[3] + tp.dnhat[1][1] * e[4] + tp.dnhat[1][2] * e[5]);
    }
    __syncthreads();
    // epochs of the grid points (as the forward kernel) and their derivatives
    const double rb0 = binary_delay<KEP>(tp, tau_s);
    double x0;
    double d0 = grid_delay<KEP>(re, tp, tau_s, oob);
    d0 = grid_delay_newton(re, tau_s, rb0, d0, x0, oob);
    d0 = grid_delay_newton(re, tau_s, rb0, d0, x0, oob);
    const double inv0 = 1.0 - x0 * (1.0 - x0 * (1.0 - x0));
    double dly[kResPerThread];
    float dT[kResPerThread][5];
    int64_t j0[kResPerThread];
    float fr[kResPerThread];
#pragma unroll
    for (int i = 0; i < kResPerThread; ++i) {
      const int64_t kk = tid + i * kResThreads;
      const double dtau = P.dt * double(kk);
      const double tau = tau_s + dtau;
      const double rb = binary_delay<KEP>(tp, tau);
      const double guess = d0 + (dtau + rb - rb0) * inv0 - dtau;
      double x;
      dly[i] = grid_delay_newton(re, tau, rb, guess, x, oob);
      split_u(double(k_s + kk) + d.off + dly[i] * P.inv_dt, j0[i], fr[i]);
      double rv, rd, ra, rdl;
      re3(tau + dly[i], rv, rd, ra, rdl, oob);
      const double inv = 1.0 - rd * (1.0 - rd * (1.0 - rd));
      // the orbit's delay R and rate R' at tau: dR/d asini = R / asini,
      // dR/d porb = -R' (tau - tp) / porb, dR/d tp = -R' (circular or Keplerian)
      double rbv = 0.0, rbp = 0.0;
      if (binary) orbit_delay<KEP>(tp, tau, rbv, rbp);
      dT[i][0] = float(-ra * inv);
      dT[i][1] = float(-rdl * inv);
      dT[i][2] = float(binary ? rbv / tp.asini * inv : 0.0);
      dT[i][3] = float(-rbp * (tau - tp.tp) / tp.porb * inv);
      dT[i][4] = float(-rbp * inv);
    }
    if (tid == 0) win_lo = j0[0] - D + 1;
    if (tid == kResThreads - 1) win_hi = j0[kResPerThread - 1] + D;
    __syncthreads();
    const int64_t lo = win_lo;
    const int64_t nwin = win_hi - lo + 1;
    if (nwin > kResWcap || nwin < 2 * D) {
      if (tid < 8) partial[tid] = __builtin_nan("");
      return;
    }
    const int W = int(nwin);
    // corrected input samples and the derivatives of their delays
    for (int w = tid; w < W; w += kResThreads) {
      const int64_t j = lo + w;
      float2 z = make_float2(0.f, 0.f);
      float dz[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
      if (j >= 0 && j < d.n) {
        const float2 xv = d.x[j];
        const double t = d.t0 + P.dt * double(j);
        double dr, ddr, da, ddl;
        re3(t, dr, ddr, da, ddl, oob);
        double r = 0.0, invb = 1.0, rs = 0.0, rsp = 0.0, tsrc = t;
        if (binary) {
          const double tb = t + dr;
          r = orbit_inverse<KEP>(tp, tb);
          tsrc = tb - r;
          orbit_delay<KEP>(tp, tsrc, rs, rsp);
          invb = 1.0 / (1.0 + rsp);
        }
        const float2 e = cis_cycles(P.f_het * (dr - r));
        z = make_float2(xv.x * e.x + xv.y * e.y, xv.y * e.x - xv.x * e.y);
        dz[0] = float(da * invb - tp.dshift[0]);
        dz[1] = float(ddl * invb - tp.dshift[1]);
        if (binary) {
          dz[2] = float(-rs / tp.asini * invb);
          dz[3] = float(rsp * (tsrc - tp.tp) / tp.porb * invb);
          dz[4] = float(rsp * invb);
        }
      }
      zs[w] = z;
#pragma unroll
      for (int q = 0; q < 5; ++q) zqs[q][w] = make_float2(dz[q] * z.x, dz[q] * z.y);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kResPerThread; ++i) {
      const float f = fr[i];
      int base = int(j0[i] - lo) - (D - 1);
      base = base < 0 ? 0 : (base > W - 2 * D ? W - 2 * D : base);
      float2 Sz = make_float2(0.f, 0.f), Sd = Sz;
      float2 S[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) S[q] = make_float2(0.f, 0.f);
      const float2 pcs = cis_cycles_f32(0.5f * f);
      const float2 wcs = cis_cycles_f32(f * (0.5f / float(D)));
      const float sp = pcs.y, cp = pcs.x, ws_ = wcs.y, wc_ = wcs.x;
      const float inv_pi = 0.318309886183790671f;
#pragma unroll 2
      for (int t = 0; t < 2 * D; ++t) {
        const int c = D - 1 - t;
        const float sg = (c & 1) ? -1.0f : 1.0f;
        const float Ct = kTaps<D>.Ct[t], St = kTaps<D>.St[t];
        const float cosw = wc_ * Ct - ws_ * St, sinw = ws_ * Ct + wc_ * St;
        const float w = 0.5f * (1.0f + cosw);
        const float dw = -0.5f * float(kPi) / float(D) * sinw;
        float h, hp;
        if (f == 0.0f) {
          // integer offset: h = delta_{c0}, h'(c) = (-1)^c w(c) / c
          h = c == 0 ? 1.0f : 0.0f;
          hp = c == 0 ? 0.0f : sg * w / float(c);
        } else {
          const float r = __builtin_amdgcn_rcpf(f + float(c));
          const float sinc = sg * sp * inv_pi * r;
          const float dsinc = (sg * cp - sinc) * r;
          h = sinc * w;
          hp = dsinc * w + sinc * dw;
        }
        const float2 zv = zs[base + t];
        Sz.x = fmaf(h, zv.x, Sz.x);
        Sz.y = fmaf(h, zv.y, Sz.y);
        Sd.x = fmaf(hp, zv.x, Sd.x);
        Sd.y = fmaf(hp, zv.y, Sd.y);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const float2 zq = zqs[q][base + t];
          S[q].x = fmaf(h, zq.x, S[q].x);
          S[q].y = fmaf(h, zq.y, S[q].y);
        }
      }
      // antenna patterns and their x derivatives at T_k
      const double tau = tau_s + P.dt * double(tid + i * kResThreads);
      const float2 ex = cis_cycles(tp.alpha_cyc[X] - P.sid_rate_cyc * (tau + dly[i]));
      const float cx = ex.x, sx = ex.y;
      const float c2 = cx * cx - sx * sx, s2 = 2.0f * sx * cx;
      const float bas[5] = {1.0f, cx, sx, c2, s2};
      const float dbas[5] = {0.0f, -sx, cx, -2.0f * s2, 2.0f * c2};
      float a = 0.f, ax = 0.f, b = 0.f, bx = 0.f, daa = 0.f, dad = 0.f, dba = 0.f, dbd = 0.f;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        a = fmaf(tp.ca[X][q], bas[q], a);
        ax = fmaf(tp.ca[X][q], dbas[q], ax);
        b = fmaf(tp.cb[X][q], bas[q], b);
        bx = fmaf(tp.cb[X][q], dbas[q], bx);
        daa = fmaf(tp.dca[0][X][q], bas[q], daa);
        dad = fmaf(tp.dca[1][X][q], bas[q], dad);
        dba = fmaf(tp.dcb[0][X][q], bas[q], dba);
        dbd = fmaf(tp.dcb[1][X][q], bas[q], dbd);
      }
      const float2 wa = Wa[i], wb = Wb[i];
      // df and f1dot: d y' = -2 pi i (phase derivative) y'
      {
        const float2 ya = cscale(Sz, a), yb = cscale(Sz, b);
        const float2 m = cadd(cmul(wa, ya), cmul(wb, yb));
        const double dtau0 = P.dt * double(k_s + tid + i * kResThreads);
        const double dtr = tau - P.t_ref;
        acc[0] += 4.0 * 2.0 * kPi * dtau0 * double(m.y);
        acc[1] += 4.0 * 2.0 * kPi * 0.5 * dtr * dtr * double(m.y);
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const float dx = (q == 0 ? 1.0f : 0.0f) - float(omega) * dT[i][q];
        const float du = dT[i][q] * float(P.inv_dt);
        // d zhat = Sd du - 2 pi i f_h S_q
        const float2 dzh = make_float2(Sd.x * du + two_pi_fh * S[q].y,
                                       Sd.y * du - two_pi_fh * S[q].x);
        const float dA = (q == 0 ? daa : q == 1 ? dad : 0.0f) + ax * dx;
        const float dB = (q == 0 ? dba : q == 1 ? dbd : 0.0f) + bx * dx;
        const float2 dya = make_float2(dA * Sz.x + a * dzh.x, dA * Sz.y + a * dzh.y);
        const float2 dyb = make_float2(dB * Sz.x + b * dzh.x, dB * Sz.y + b * dzh.y);
        const float2 m = cadd(cmul(wa, dya), cmul(wb, dyb));
        acc[2 + q] += 4.0 * double(m.x);
      }
    }
    __syncthreads();
  }
  if (oob) bad = 1;
  // block reduction of the seven sums: wavefront shuffles, then LDS
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int q = 0; q < kGradParams; ++q) {
    double v = acc[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  if (tid < kGradParams) {
    double v = 0.0;
    for (int w = 0; w < kResThreads / 64; ++w) v += red[w][tid];
    partial[tid] = bad ? __builtin_nan("") : v;
  }
}

// Per template (one workgroup each): the totals of the tile partials in a
// fixed order; NaN for a flagged template; zero orbit derivatives for an
// isolated one.
__global__ __launch_bounds__(kFinalThreads) void k_grad_final(PlanConst P, void* ws, ChunkMap map,
                                                              int64_t ntiles,
                                                              double* __restrict__ grad) {
  const int slot = blockIdx.x;
  double s[kGradParams];
  tile_sums<kGradParams>(slot_partials(ws, P, slot), ntiles, s);
  if (threadIdx.x != 0) return;
  const TmplParams& tp = *slot_params(ws, P, slot);
#pragma unroll
  for (int q = 0; q < kGradParams; ++q) {
    double v = s[q];
    if (tp.status != 0) v = __builtin_nan("");
    if (tp.asini == 0.0 && q >= 4 && tp.status == 0) v = 0.0;
    grad[map.tmpl[slot] * kGradParams + q] = v;
  }
}

}  // namespace fstat
