// Per-data-set antenna moments and the per-template prologue.
//
// A, B, C of eq. Fstat (Sec. 2) are noise-weighted sums of products of a(t),
// b(t) over the valid samples.  a and b are trigonometric polynomials of
// degree two in x = alpha - phi(t) (phi: local sidereal angle), so
//   sum_j v_j P(x_j) Q(x_j) = 1/2 Re sum_{h,g} [p_h q_g S_{h+g} + p_h conj(q_g) S_{h-g}]
// with P = Re sum_h p_h e^{i h x}, Q = Re sum_g q_g e^{i g x}, and
//   S_n = sum_j v_j e^{i n x_j} = e^{i n alpha} conj(M_n),  M_n = sum_j v_j e^{i n phi_j}.
// The moments M_0..M_4 depend on the data set only; the prologue combines
// them with the sky position in O(1) per template.
#pragma once

#include "fstat_common.hpp"

namespace fstat {

// Partial moments: block b of detector X sums a contiguous chunk of samples.
__global__ __launch_bounds__(kMomThreads) void k_moments_partial(PlanConst P, double* partial) {
  const int X = blockIdx.y;
  const DetConst& d = P.det[X];
  const int64_t n = d.n;
  const int64_t chunk = (n + kMomBlocks - 1) / kMomBlocks;
  const int64_t j_beg = int64_t(blockIdx.x) * chunk;
  const int64_t j_end = j_beg + chunk < n ? j_beg + chunk : n;
  double acc[10];
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  const double two_pi = 2.0 * kPi;
  for (int64_t j = j_beg + threadIdx.x; j < j_end; j += kMomThreads) {
    double v = d.valid ? double(d.valid[j]) : 1.0;
    if (v == 0.0) continue;
    double cyc = d.lst0_cyc + P.sid_rate_cyc * (d.t0 + P.dt * double(j));
    cyc -= rint(cyc);
    double s1, c1;
    sincos(two_pi * cyc, &s1, &c1);
    double cr = 1.0, ci = 0.0;
    for (int h = 0; h < 5; ++h) {
      acc[2 * h] += v * cr;
      acc[2 * h + 1] += v * ci;
      double nr = cr * c1 - ci * s1;
      ci = cr * s1 + ci * c1;
      cr = nr;
    }
  }
  __shared__ double red[kMomThreads];
  for (int q = 0; q < 10; ++q) {
    red[threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = kMomThreads / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t(X) * kMomBlocks + blockIdx.x) * 10 + q] = red[0];
    __syncthreads();
  }
}

// Final sum of the partials in block order.
__global__ void k_moments_final(int ndet, const double* partial, double* moments) {
  int t = threadIdx.x;
  if (t >= ndet * 10) return;
  int X = t / 10, q = t % 10;
  double s = 0.0;
  for (int b = 0; b < kMomBlocks; ++b) s += partial[(size_t(X) * kMomBlocks + b) * 10 + q];
  moments[X * 10 + q] = s;
}

struct cd {
  double r, i;
};
__host__ __device__ inline cd cd_mul(cd a, cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__host__ __device__ inline cd cd_conj(cd a) { return {a.r, -a.i}; }

// sum_j v_j P(x_j) Q(x_j) for degree-2 polynomials p, q (complex coefficients)
// given S_0..S_4.
__host__ __device__ inline double moment_product(const cd p[3], const cd q[3], const cd S[5]) {
  double acc = 0.0;
#pragma unroll
  for (int h = 0; h < 3; ++h)
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      cd t1 = cd_mul(cd_mul(p[h], q[g]), S[h + g]);
      int dn = h - g;
      cd sd = dn >= 0 ? S[dn] : cd_conj(S[-dn]);
      cd t2 = cd_mul(cd_mul(p[h], cd_conj(q[g])), sd);
      acc += t1.r + t2.r;
    }
  return 0.5 * acc;
}

// Coefficients of a(t), b(t) (Jaranowski, Krolak & Schutz 1998 eqs. 12-13,
// cited in Sec. 2) in the basis (1, cos x, sin x, cos 2x, sin 2x) of
// x = alpha - phi(t), for one detector at declination delta, and their delta
// derivatives (d sin 2delta = 2 cos 2delta, d cos 2delta = -2 sin 2delta).
struct Jks {
  double pa[5], pb[5], dpa[5], dpb[5];
};
__host__ __device__ inline Jks jks_coeffs(const DetConst& d, double sd, double cdl) {
  const double sl = d.sl, cl = d.cl, sg = d.s2g, cg = d.c2g;
  const double s2l = 2.0 * sl * cl, c2l = cl * cl - sl * sl;
  const double s2d = 2.0 * sd * cdl, c2d = cdl * cdl - sd * sd;
  Jks k;
  k.pa[0] = 0.75 * sg * cl * cl * cdl * cdl;
  k.pa[1] = 0.25 * sg * s2l * s2d;
  k.pa[2] = -0.5 * cg * cl * s2d;
  k.pa[3] = sg * (3.0 - c2l) * (3.0 - c2d) / 16.0;
  k.pa[4] = -0.25 * cg * sl * (3.0 - c2d);
  k.pb[0] = 0.0;
  k.pb[1] = cg * cl * cdl;
  k.pb[2] = 0.5 * sg * s2l * cdl;
  k.pb[3] = cg * sl * sd;
  k.pb[4] = 0.25 * sg * (3.0 - c2l) * sd;
  k.dpa[0] = -0.75 * sg * cl * cl * s2d;
  k.dpa[1] = 0.5 * sg * s2l * c2d;
  k.dpa[2] = -cg * cl * c2d;
  k.dpa[3] = sg * (3.0 - c2l) * s2d / 8.0;
  k.dpa[4] = -0.5 * cg * sl * s2d;
  k.dpb[0] = 0.0;
  k.dpb[1] = -cg * cl * sd;
  k.dpb[2] = -0.5 * sg * s2l * sd;
  k.dpb[3] = cg * sl * cdl;
  k.dpb[4] = 0.25 * sg * (3.0 - c2l) * cdl;
  return k;
}

// Per template: sky vector, antenna coefficients, A, B, C, D of eq. Fstat,
// the whitening of (a, b) and the alpha/delta derivatives of the whitened
// coefficients.  The detector loops run over the compile-time maximum so that
// every index is static and the parameter block stays in registers.
__host__ __device__ inline void template_params(const PlanConst& P, const double* row,
                                                TmplParams& tp) {
  double alpha = row[0], delta = row[1];
  tp.df = row[2];
  tp.f1dot = row[3];
  tp.f2dot = row[4];
  tp.asini = row[5];
  double porb = row[6];
  tp.tp = row[7];
  const double ecc = P.tmpl_stride >= FSTAT_TEMPLATE_STRIDE_KEPLER ? row[8] : 0.0;
  const double argp = P.tmpl_stride >= FSTAT_TEMPLATE_STRIDE_KEPLER ? row[9] : 0.0;
  int status = 0;
  // porb and tp describe the orbit only when asini != 0: an isolated
  // source (asini = 0) ignores them, whatever they hold
  if (!__builtin_isfinite(alpha) || !__builtin_isfinite(delta) || !__builtin_isfinite(tp.asini) ||
      (tp.asini != 0.0 && (!__builtin_isfinite(porb) || !__builtin_isfinite(tp.tp))))
    status |= kStatusTiming;
  if (!__builtin_isfinite(tp.df) || !__builtin_isfinite(tp.f1dot) ||
      !__builtin_isfinite(tp.f2dot))
    status |= kStatusPhase;
  if (tp.asini < 0.0 || (tp.asini != 0.0 && !(porb > 0.0))) status |= kStatusTiming;
  // Keplerian elements (used only when asini != 0)
  if (tp.asini != 0.0 && !(ecc >= 0.0 && ecc < 1.0 && __builtin_isfinite(argp)))
    status |= kStatusTiming;
  tp.kepler = (tp.asini != 0.0 && (ecc != 0.0 || argp != 0.0)) ? 1 : 0;
  tp.ecc = tp.kepler ? ecc : 0.0;
  tp.sq_e = sqrt(1.0 - tp.ecc * tp.ecc);
  if (tp.kepler) {
    sincos(argp, &tp.sin_w, &tp.cos_w);
  } else {
    tp.sin_w = 0.0;
    tp.cos_w = 1.0;
  }
  if (tp.asini > P.max_delay) status |= kStatusCoverage;
  tp.om_b = (tp.asini != 0.0 && porb > 0.0) ? 2.0 * kPi / porb : 0.0;
  tp.nu_b = (tp.asini != 0.0 && porb > 0.0) ? 1.0 / porb : 0.0;
  // Knot spacing of the resampling's timing: the largest G = 2^l <= 64 for
  // which the cubic Hermite bound (G dt)^4 / 384 max|delay''''| stays below
  // 2e-7 cycles of the heterodyne phase f_h and 1e-7 samples of grid
  // position.  The binary delay contributes asini om^4; the Earth's motion,
  // tabulated as C1-joined cubics, contributes far less than the floor
  // taken here.  Below G = 4, every point is solved (knot_log2 = 0).
  {
    // the Keplerian delay's fourth derivative grows like (om / (1 - ecc)^2)^4
    // near periapsis (a bound, not the exact maximum)
    const double w = tp.om_b / ((1.0 - tp.ecc) * (1.0 - tp.ecc));
    const double om2 = w * w;
    const double d4 = fabs(tp.asini) * om2 * om2 + 1e-16;
    const double budget = fmin(2e-7 / fmax(fabs(P.f_het), 1.0), 1e-7 * P.dt);
    tp.knot_log2 = 0;
    for (int l = kKnotLogMax; l >= kKnotLogMin; --l) {
      const double h = double(1 << l) * P.dt, h2 = h * h;
      if (h2 * h2 / 384.0 * d4 <= budget) {
        tp.knot_log2 = l;
        break;
      }
    }
  }
  spindown_coefficients(P, tp.f1dot, tp.f2dot, tp.df, tp.sd);
  double sa, ca_, sd, cdl;
  sincos(alpha, &sa, &ca_);
  sincos(delta, &sd, &cdl);
  tp.nhat[0] = cdl * ca_;
  tp.nhat[1] = cdl * sa;
  tp.nhat[2] = sd;
  tp.porb = porb;
  // d nhat / d alpha, d nhat / d delta
  tp.dnhat[0][0] = -cdl * sa;
  tp.dnhat[0][1] = cdl * ca_;
  tp.dnhat[0][2] = 0.0;
  tp.dnhat[1][0] = -sd * ca_;
  tp.dnhat[1][1] = -sd * sa;
  tp.dnhat[1][2] = cdl;
  // e^{i n alpha}, n = 0..4
  cd ea[5];
  ea[0] = {1.0, 0.0};
  ea[1] = {ca_, sa};
#pragma unroll
  for (int n = 2; n < 5; ++n) ea[n] = cd_mul(ea[n - 1], ea[1]);
  double A = 0.0, B = 0.0, C = 0.0;
  // derivatives of A, B, C with respect to alpha (index 0) and delta (1)
  double dA[2] = {0.0, 0.0}, dB[2] = {0.0, 0.0}, dC[2] = {0.0, 0.0};
#pragma unroll
  for (int X = 0; X < kMaxDet; ++X) {
    tp.alpha_cyc[X] = 0.0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      tp.ca[X][q] = tp.cb[X][q] = 0.0f;
      tp.dca[0][X][q] = tp.dcb[0][X][q] = tp.dca[1][X][q] = tp.dcb[1][X][q] = 0.0f;
    }
    if (X >= P.ndet) continue;
    const DetConst& d = P.det[X];
    const Jks k = jks_coeffs(d, sd, cdl);
    tp.alpha_cyc[X] = alpha / (2.0 * kPi) - d.lst0_cyc;
    // S_n = e^{i n alpha} conj(M_n)
    cd S[5];
#pragma unroll
    for (int n = 0; n < 5; ++n)
      S[n] = cd_mul(ea[n], cd_conj({P.moments[X * 10 + 2 * n], P.moments[X * 10 + 2 * n + 1]}));
    const cd p[3] = {{k.pa[0], 0.0}, {k.pa[1], -k.pa[2]}, {k.pa[3], -k.pa[4]}};
    const cd q[3] = {{k.pb[0], 0.0}, {k.pb[1], -k.pb[2]}, {k.pb[3], -k.pb[4]}};
    A += d.w * moment_product(p, p, S);
    B += d.w * moment_product(q, q, S);
    C += d.w * moment_product(p, q, S);
    // alpha enters through S_n = e^{i n alpha} conj(M_n): dS_n = i n S_n
    cd dS[5];
#pragma unroll
    for (int n = 0; n < 5; ++n) dS[n] = {-double(n) * S[n].i, double(n) * S[n].r};
    dA[0] += d.w * moment_product(p, p, dS);
    dB[0] += d.w * moment_product(q, q, dS);
    dC[0] += d.w * moment_product(p, q, dS);
    // delta enters through the coefficients (the product is bilinear)
    const cd dp[3] = {{k.dpa[0], 0.0}, {k.dpa[1], -k.dpa[2]}, {k.dpa[3], -k.dpa[4]}};
    const cd dq[3] = {{k.dpb[0], 0.0}, {k.dpb[1], -k.dpb[2]}, {k.dpb[3], -k.dpb[4]}};
    dA[1] += d.w * 2.0 * moment_product(dp, p, S);
    dB[1] += d.w * 2.0 * moment_product(dq, q, S);
    dC[1] += d.w * (moment_product(dp, q, S) + moment_product(p, dq, S));
  }
  // 2F = 2 F^T M^-1 F is unchanged by a constant invertible map of (a, b).
  // Whitening by the Cholesky factor of M in FP64 makes M' = I, so the FP32
  // epilogue sums two squares instead of cancelling terms of size cond(M).
  double Dd = A * B - C * C;
  if (!(A > 0.0) || !(Dd > 0.0) || !__builtin_isfinite(Dd)) status |= kStatusTiming;
  const double l11 = sqrt(A), l21 = C / l11, l22 = sqrt(Dd / A);
  const double r = C / A;
  tp.l11 = static_cast<float>(l11);
  tp.l21 = static_cast<float>(l21);
  tp.l22 = static_cast<float>(l22);
  // derivatives of the whitened coefficients: a' = a / l11,
  // b' = (b - r a) / l22 with r = C/A, l11^2 = A, l22^2 = B - C^2/A
  double dl11[2], dr[2], dl22[2];
#pragma unroll
  for (int th = 0; th < 2; ++th) {
    dl11[th] = dA[th] / (2.0 * l11);
    dr[th] = (dC[th] * A - C * dA[th]) / (A * A);
    dl22[th] = (dB[th] - (2.0 * C * dC[th] * A - C * C * dA[th]) / (A * A)) / (2.0 * l22);
  }
#pragma unroll
  for (int X = 0; X < kMaxDet; ++X) {
    if (X >= P.ndet) continue;
    const double w = P.det[X].w;
    const Jks k = jks_coeffs(P.det[X], sd, cdl);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const double bq = k.pb[q] - r * k.pa[q];
      tp.ca[X][q] = static_cast<float>(w * k.pa[q] / l11);
      tp.cb[X][q] = static_cast<float>(w * bq / l22);
#pragma unroll
      for (int th = 0; th < 2; ++th) {
        const double dpaq = th == 1 ? k.dpa[q] : 0.0;
        const double dpbq = th == 1 ? k.dpb[q] : 0.0;
        const double dbq = dpbq - dr[th] * k.pa[q] - r * dpaq;
        tp.dca[th][X][q] =
            static_cast<float>(w * (dpaq / l11 - k.pa[q] * dl11[th] / (l11 * l11)));
        tp.dcb[th][X][q] = static_cast<float>(w * (dbq / l22 - bq * dl22[th] / (l22 * l22)));
      }
    }
  }
  tp.status = status;
}

// Everything the kernels need about one template: template_params plus the
// coverage check of the source-frame grid and the adjoint's sky shift.
__device__ inline void full_params(const PlanConst& P, const double* row, TmplParams& tp) {
  template_params(P, row, tp);
  int status = tp.status;
  // Coverage: every sample's source time lies inside the computed grid, and
  // the interpolation taps of the last sample end before the last computed
  // point, so grid points beyond k_pad are exactly zero.
  if ((status & kStatusGroupMask) == 0) {
#pragma unroll
    for (int X = 0; X < kMaxDet; ++X) {
      if (X >= P.ndet) continue;
      const DetConst& d = P.det[X];
      const GlobalRoemer re{d.ephem, tp.nhat, P.n_eph, P.eph_t0, P.eph_dt, P.inv_eph_dt};
      double u_first = 0.0 + d.off + grid_delay<true>(re, tp, P.tau0) * P.inv_dt;
      double k_last = double(P.k_pad - 1);
      double u_last = k_last + d.off + grid_delay<true>(re, tp, P.tau0 + k_last * P.dt) * P.inv_dt;
      if (!(u_first <= 0.0) || !(u_last >= double(d.n - 1 + P.D))) status |= kStatusCoverage;
    }
  }
  tp.status = status;
  const double t_mid = P.tau0 + 0.5 * double(P.k_pad) * P.dt;
  const DetConst& d0 = P.det[0];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const GlobalRoemer rq{d0.ephem, tp.dnhat[q], P.n_eph, P.eph_t0, P.eph_dt, P.inv_eph_dt};
    double v, dv;
    rq(t_mid, v, dv);
    tp.dshift[q] = v;
  }
}

// Parameter blocks of the templates of one chunk, into their slots.
__global__ __launch_bounds__(64) void k_prologue(PlanConst P, const double* __restrict__ templates,
                                                 ChunkMap map, void* ws) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= map.n_tmpl) return;
  TmplParams tp;
  full_params(P, templates + map.tmpl[g] * P.tmpl_stride, tp);
  *slot_params(ws, P, g) = tp;
}

// Search path, once per run: the parameter blocks of all templates into the
// per-template array P.params, the status words of the group buffers cleared
// for the first chunk, and the candidate count and per-template maxima of
// the run cleared (in a kernel, so that a captured graph needs no memset).
__global__ __launch_bounds__(64) void k_params(PlanConst P, const double* __restrict__ templates,
                                               int64_t ntmpl, void* ws, int slots,
                                               RowOutput out) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < slots) *group_status(ws, P, slots, int(t)) = 0;
  if (t == 0 && out.count) *out.count = 0ull;
  if (t >= ntmpl) return;
  if (out.best) out.best[t] = 0ull;
  TmplParams tp;
  full_params(P, templates + t * P.tmpl_stride, tp);
  *reinterpret_cast<TmplParams*>(P.params + size_t(t) * kParamBytes) = tp;
}

}  // namespace fstat
