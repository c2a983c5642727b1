// Host-only check of the per-template prologue: the analytic derivatives of
// the whitened antenna coefficients with respect to the sky position must
// match central finite differences of the coefficients themselves.  Built
// and run by tests/test_host_checks.py; no GPU is touched.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>

#include "fstat_prologue.hpp"

using namespace fstat;

int main() {
  PlanConst P;
  std::memset(&P, 0, sizeof P);
  P.ndet = 2;
  P.D = 8;
  P.dt = 60.0;
  P.max_delay = 600.0;
  const double rate = 2.0 * kPi / 86164.0905;
  const double lat[2] = {46.45 * kPi / 180, 30.56 * kPi / 180};
  const double lon[2] = {-119.41 * kPi / 180, -90.77 * kPi / 180};
  const double gam[2] = {170.9 * kPi / 180, 242.7 * kPi / 180};
  const double wgt[2] = {1.0, 0.8};
  static double moments[2 * 10];
  for (int X = 0; X < 2; ++X) {
    P.det[X].lat = lat[X];
    P.det[X].gamma = gam[X];
    P.det[X].sl = std::sin(lat[X]);
    P.det[X].cl = std::cos(lat[X]);
    P.det[X].s2g = std::sin(2.0 * gam[X]);
    P.det[X].c2g = std::cos(2.0 * gam[X]);
    P.det[X].w = wgt[X];
    P.det[X].lst0_cyc = lon[X] / (2 * kPi);
    // moments of 1.5 days of samples every 60 s with a gap
    for (int j = 0; j < 2160; ++j) {
      if (j > 700 && j < 900) continue;
      const double phi = lon[X] + rate * 60.0 * j;
      for (int n = 0; n < 5; ++n) {
        moments[X * 10 + 2 * n] += std::cos(n * phi);
        moments[X * 10 + 2 * n + 1] += std::sin(n * phi);
      }
    }
  }
  P.moments = moments;
  double row[8] = {1.3, -0.4, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
  TmplParams t0;
  template_params(P, row, t0);
  if (t0.status != 0) {
    printf("FAIL status %d\n", t0.status);
    return 1;
  }
  const double h = 1e-3;
  double worst = 0.0, scale = 0.0;
  for (int th = 0; th < 2; ++th) {
    double rp[8], rm[8];
    std::memcpy(rp, row, sizeof row);
    std::memcpy(rm, row, sizeof row);
    rp[th] += h;
    rm[th] -= h;
    TmplParams tpp, tpm;
    template_params(P, rp, tpp);
    template_params(P, rm, tpm);
    for (int X = 0; X < 2; ++X)
      for (int q = 0; q < 5; ++q) {
        // alpha moves x = alpha - phi too; the coefficients are per unit x,
        // so their alpha derivative at fixed x is what changes with alpha
        const double fa = (double(tpp.ca[X][q]) - double(tpm.ca[X][q])) / (2 * h);
        const double fb = (double(tpp.cb[X][q]) - double(tpm.cb[X][q])) / (2 * h);
        worst = std::fmax(worst, std::fabs(fa - t0.dca[th][X][q]));
        worst = std::fmax(worst, std::fabs(fb - t0.dcb[th][X][q]));
        scale = std::fmax(scale, std::fmax(std::fabs(t0.dca[th][X][q]), std::fabs(t0.dcb[th][X][q])));
      }
    for (int c = 0; c < 3; ++c) {
      const double fd = (tpp.nhat[c] - tpm.nhat[c]) / (2 * h);
      worst = std::fmax(worst, std::fabs(fd - t0.dnhat[th][c]));
    }
  }
  printf("scale %.3e worst %.3e\n", scale, worst);
  if (!(scale > 1e-3) || !(worst < 2e-3 * scale)) {
    printf("FAIL\n");
    return 1;
  }
  printf("OK\n");
  return 0;
}
