// Host side of the C ABI declared in include/fstat.h: plan validation,
// workspace sizing, FFT split selection and kernel launches.  All device
// memory belongs to the caller; nothing here allocates on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fstat_common.hpp"
#include "fstat_fft.hpp"
#include "fstat_prologue.hpp"
#include "fstat_resample.hpp"
#include "fstat_adjoint.hpp"
#include "fstat_sft.hpp"

using namespace fstat;

// Device scratch of the entry point that allocates nothing: one copy per GPU
// the library runs on, kept until the process ends.  Host code never uses
// the array's name as an address: each device's address comes from
// hipGetSymbolAddress (static_scratch below).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

struct fstat_plan {
  fstat_plan_desc desc;
  int log_n, log_rr, log_c;  // N = Rr * C
  int cols_lines, rows_lines;
  bool cols_half, rows_half;
  int fft_mlr;       // largest stage radix 2^fft_mlr
  int64_t k_pad, rows_act;
  double t_lo, t_hi;         // time range any timing evaluation may touch
};

namespace {

thread_local std::string g_err;

fstat_status fail(fstat_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fstat_status fail(fstat_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

fstat_status ok() {
  g_err.clear();
  return FSTAT_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

// Lines per workgroup of the column pass (NL) and rows per workgroup of the
// row pass (RQ): at most as many as fit 128 KiB of LDS, capped for
// coalescing, with 512 threads; or half of that with 256 threads, so that two
// workgroups share a compute unit.
int cols_lines_max(int log_rr) { return std::min(64, 16384 >> log_rr); }
int rows_lines_max(int log_c) { return std::min(32, 8192 >> log_c); }

using ColsFn = void (*)(PlanConst, void*, ChunkMap, int, int, int, int64_t);
using RowsFn = void (*)(PlanConst, void*, ChunkMap, int, int, RowOutput);

template <int LOGL>
constexpr int kColsMax = (16384 >> LOGL) < 64 ? (16384 >> LOGL) : 64;
template <int LOGL>
constexpr int kRowsMax = (8192 >> LOGL) < 32 ? (8192 >> LOGL) : 32;

struct FftVariant {
  const void* fn;
  int threads;
  size_t lds;    // dynamic LDS bytes
  int lines;     // columns (column pass) or rows of each array (row pass) per item
};

// Variant choice of the FFT passes: full or half line counts (512 or 256
// threads), largest stage radix 2^mlr (mlr 4 or 5; only line lengths 2^9 and
// 2^10 have a different stage plan with 2^5).
struct FftChoice {
  bool half;
  int mlr;
};

template <int LOGL, bool GROUPED, int MLR, int NL, int NT>
FftVariant cols_variant_n() {
  constexpr int R0 = kR0<LOGL, MLR>;
  constexpr size_t lds = kLdsBytes<1 << LOGL, R0, NL, NL>;
  return {reinterpret_cast<const void*>(&k_fft_cols<LOGL, NL, NT, GROUPED, MLR>), NT, lds, NL};
}
// Columns of 2^11 and 2^12 points at the full line count split each column
// in two halves that go through LDS one after the other (k_fft_cols_half),
// so two workgroups share a compute unit.
template <int LOGL, bool GROUPED, int MLR>
FftVariant cols_half_lds_variant() {
  constexpr int NL = kColsMax<LOGL>;
  constexpr int R0 = kR0<LOGL - 1, MLR>;
  constexpr size_t lds = kLdsBytes<1 << (LOGL - 1), R0, NL, NL>;
  return {reinterpret_cast<const void*>(&k_fft_cols_half<LOGL, NL, 512, GROUPED, MLR>), 512, lds,
          NL};
}
template <int LOGL, bool GROUPED, int MLR>
FftVariant cols_variant(bool half) {
  if (half) return cols_variant_n<LOGL, GROUPED, MLR, kColsMax<LOGL> / 2, 256>();
  if constexpr (LOGL >= 11) return cols_half_lds_variant<LOGL, GROUPED, MLR>();
  return cols_variant_n<LOGL, GROUPED, MLR, kColsMax<LOGL>, 512>();
}
template <int LOGL, int MODE, int MLR, int RQ, int NT>
FftVariant rows_variant_n() {
  constexpr int R0 = kR0<LOGL, MLR>;
  constexpr size_t lds = kLdsBytes<1 << LOGL, R0, RQ, 2 * RQ>;
  // rows of 2^12 at the full count: two halves through LDS one after the
  // other (k_fft_rows_half; every epilogue, so that they all give the plain
  // 2F pass's bits), two workgroups per compute unit for the plain 2F pass
  if constexpr (LOGL >= 12 && NT == 512 && RQ == kRowsMax<LOGL>) {
    constexpr int RH = kR0<LOGL - 1, MLR>;
    return {reinterpret_cast<const void*>(&k_fft_rows_half<LOGL, RQ, NT, MODE, MLR>), NT,
            kLdsBytes<1 << (LOGL - 1), RH, RQ, 2 * RQ>, RQ};
  }
  return {reinterpret_cast<const void*>(&k_fft_rows<LOGL, RQ, NT, MODE, MLR>), NT, lds, RQ};
}
// The plain 2F pass at the full row count holds one array at a time in LDS
// (k_fft_rows_split), so two 512-thread workgroups share a compute unit; with
// radix-32 stages that does not fit 128 VGPRs, and with fewer than 4 rows per
// item (lines of 2^12) the shorter 2F runs cost more than the occupancy
// gains (measured): there the pass keeps both arrays.
template <int LOGL, int MLR, int MODE>
FftVariant rows_split_variant() {
  constexpr int RQ = kRowsMax<LOGL>, R0 = kR0<LOGL, MLR>;
  return {reinterpret_cast<const void*>(&k_fft_rows_split<LOGL, RQ, 512, MLR, MODE>), 512,
          kLdsBytes<1 << LOGL, R0, RQ, RQ>, RQ};
}
// The adjoint, conjugate and extended epilogues of a radix-32 plan exceed 256
// VGPRs at the full count: they take the half count (the same arithmetic per
// point, so the same bits as the full-count plain 2F kernel).
// Candidates and loudest bin only: the split pass where the plain 2F pass
// takes it (no 2F array is written), else the extended epilogue.
template <int LOGL, int MODE, int MLR>
FftVariant rows_variant(bool half) {
  if constexpr (MODE == kRowCand) {
    if constexpr (kR0<LOGL, MLR> <= 16 && kRowsMax<LOGL> >= 4) {
      if (!half) return rows_split_variant<LOGL, MLR, kRowCand>();
    }
    // rows of 2^12: the half-LDS pass with the candidate epilogue
    if constexpr (LOGL >= 12) {
      if (!half) return rows_variant_n<LOGL, kRowCand, MLR, kRowsMax<LOGL>, 512>();
    }
    return rows_variant<LOGL, kRow2FExt, MLR>(half);
  } else if constexpr (MODE != kRow2F && kR0<LOGL, MLR> == 32) {
    return rows_variant_n<LOGL, MODE, MLR, kRowsMax<LOGL> / 2, 256>();
  } else {
    if (half) return rows_variant_n<LOGL, MODE, MLR, kRowsMax<LOGL> / 2, 256>();
    if constexpr (MODE == kRow2F && kR0<LOGL, MLR> <= 16 && kRowsMax<LOGL> >= 4)
      return rows_split_variant<LOGL, MLR, kRow2F>();
    return rows_variant_n<LOGL, MODE, MLR, kRowsMax<LOGL>, 512>();
  }
}

template <bool GROUPED, int MLR>
FftVariant pick_cols_v(int logl, bool half) {
  switch (logl) {
    case 6: return cols_variant<6, GROUPED, 4>(half);
    case 7: return cols_variant<7, GROUPED, 4>(half);
    case 8: return cols_variant<8, GROUPED, 4>(half);
    case 9: return cols_variant<9, GROUPED, MLR>(half);
    case 10: return cols_variant<10, GROUPED, MLR>(half);
    case 11: return cols_variant<11, GROUPED, 4>(half);
    case 12: return cols_variant<12, GROUPED, 4>(half);
    default: return {nullptr, 0, 0, 1};
  }
}
FftVariant pick_cols(int logl, const FftChoice& c, bool grouped) {
  if (c.mlr == 5) return grouped ? pick_cols_v<true, 5>(logl, c.half) : pick_cols_v<false, 5>(logl, c.half);
  return grouped ? pick_cols_v<true, 4>(logl, c.half) : pick_cols_v<false, 4>(logl, c.half);
}
template <int MODE, int MLR>
FftVariant pick_rows_v(int logl, bool half) {
  switch (logl) {
    case 6: return rows_variant<6, MODE, 4>(half);
    case 7: return rows_variant<7, MODE, 4>(half);
    case 8: return rows_variant<8, MODE, 4>(half);
    case 9: return rows_variant<9, MODE, MLR>(half);
    case 10: return rows_variant<10, MODE, MLR>(half);
    case 11: return rows_variant<11, MODE, 4>(half);
    case 12: return rows_variant<12, MODE, 4>(half);
    default: return {nullptr, 0, 0, 1};
  }
}
template <int MODE>
FftVariant pick_rows_m(int logl, const FftChoice& c) {
  return c.mlr == 5 ? pick_rows_v<MODE, 5>(logl, c.half) : pick_rows_v<MODE, 4>(logl, c.half);
}
FftVariant pick_rows(int logl, const FftChoice& c, int mode = kRow2F) {
  return mode == kRowAdjoint ? pick_rows_m<kRowAdjoint>(logl, c)
         : mode == kRowConj  ? pick_rows_m<kRowConj>(logl, c)
         : mode == kRow2FExt ? pick_rows_m<kRow2FExt>(logl, c)
         : mode == kRowCand  ? pick_rows_m<kRowCand>(logl, c)
                             : pick_rows_m<kRow2F>(logl, c);
}
// The forward epilogue a RowOutput needs: plain 2F stores, candidates and
// loudest bin without a 2F array, or the extended one.
int forward_row_mode(const RowOutput& out) {
  if (out.twoF && !out.fafb && !out.cand && !out.best && !out.acc) return kRow2F;
  if (!out.twoF && !out.fafb && !out.acc && (out.cand || out.best)) return kRowCand;
  return kRow2FExt;
}

FftChoice cols_choice(const fstat_plan* p) { return {p->cols_half, p->fft_mlr}; }
FftChoice rows_choice(const fstat_plan* p) { return {p->rows_half, p->fft_mlr}; }

fstat_status check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(FSTAT_EHIP, "%s: %s", what, hipGetErrorString(e));
  return FSTAT_OK;
}

fstat_status validate_desc(const fstat_plan_desc* d) {
  if (!d) return fail(FSTAT_EINVAL, "desc is NULL");
  if (d->flags & ~FSTAT_PLAN_KEPLER)
    return fail(FSTAT_EINVAL, "flags: only FSTAT_PLAN_KEPLER is defined");
  if (d->ndet < 1 || d->ndet > FSTAT_MAX_DET)
    return fail(FSTAT_EINVAL, "ndet=%d outside [1, %d]", d->ndet, FSTAT_MAX_DET);
  if (d->sinc_halfwidth != 4 && d->sinc_halfwidth != 6 && d->sinc_halfwidth != 8 &&
      d->sinc_halfwidth != 10 && d->sinc_halfwidth != 12 && d->sinc_halfwidth != 16)
    return fail(FSTAT_EINVAL, "sinc_halfwidth=%d not one of 4, 6, 8, 10, 12, 16",
                d->sinc_halfwidth);
  if (!finite_pos(d->dt)) return fail(FSTAT_EINVAL, "dt must be positive and finite");
  if (!std::isfinite(d->f_het) || !std::isfinite(d->t_ref) || !std::isfinite(d->tau0))
    return fail(FSTAT_EINVAL, "f_het, t_ref and tau0 must be finite");
  if (!(std::isfinite(d->max_delay) && d->max_delay >= 0.0))
    return fail(FSTAT_EINVAL, "max_delay must be finite and >= 0");
  if (!finite_pos(d->sid_rate) || !std::isfinite(d->sid_angle0))
    return fail(FSTAT_EINVAL, "sid_rate must be positive and finite, sid_angle0 finite");
  const int64_t n = d->n_fft;
  if (n < (int64_t(1) << 12) || n > (int64_t(1) << 24) || (n & (n - 1)) != 0)
    return fail(FSTAT_EINVAL, "n_fft=%lld must be a power of two in [2^12, 2^24]",
                (long long)n);
  if (d->n_bins < 1 || d->bin_lo < 0 || d->bin_lo + d->n_bins > n)
    return fail(FSTAT_EINVAL, "band [bin_lo, bin_lo+n_bins) must be non-empty inside [0, n_fft)");
  for (int X = 0; X < d->ndet; ++X) {
    const fstat_detector& t = d->det[X];
    if (t.n < 1) return fail(FSTAT_EINVAL, "detector %d: n must be >= 1", X);
    if (!finite_pos(t.noise_var)) return fail(FSTAT_EINVAL, "detector %d: noise_var must be positive and finite", X);
    if (!std::isfinite(t.t0) || !std::isfinite(t.lat) || !std::isfinite(t.lon) ||
        !std::isfinite(t.az_x) || !std::isfinite(t.az_y))
      return fail(FSTAT_EINVAL, "detector %d: geometry and t0 must be finite", X);
    if (std::fabs(std::fabs(std::remainder(t.az_y - t.az_x, M_PI)) - M_PI / 2) > 1e-6)
      return fail(FSTAT_EINVAL, "detector %d: arms must be orthogonal", X);
    if (d->tau0 + d->max_delay > t.t0)
      return fail(FSTAT_EINVAL,
                  "detector %d: grid origin tau0 + max_delay = %.6g is after the first sample %.6g",
                  X, d->tau0 + d->max_delay, t.t0);
  }
  return FSTAT_OK;
}

// Doubles per template row of a plan.
int tmpl_stride(const fstat_plan* p) {
  return (p->desc.flags & FSTAT_PLAN_KEPLER) ? FSTAT_TEMPLATE_STRIDE_KEPLER
                                             : FSTAT_TEMPLATE_STRIDE;
}

// Knot area of the search and plain forward paths (per detector: grid
// intervals, their integer parts, sample knots and tile records, at the
// capacities of the smallest knot spacing that is solved ahead of the
// resampling).
int64_t knot_gcap(const fstat_plan* p) { return knot_grid_cap(p->k_pad); }
int64_t knot_ioff(const fstat_plan* p) { return knot_gcap(p); }
int64_t knot_soff(const fstat_plan* p) { return knot_ioff(p) + (knot_gcap(p) + 3) / 4; }
int64_t knot_scap(const fstat_plan* p) {
  int64_t scap = 0;
  for (int X = 0; X < p->desc.ndet; ++X)
    scap = std::max<int64_t>(scap, knot_samp_cap(p->desc.det[X].n));
  return scap;
}
int64_t knot_toff(const fstat_plan* p) { return knot_soff(p) + 2 * knot_scap(p); }
int64_t knot_stride(const fstat_plan* p) {
  return knot_toff(p) + (p->k_pad >> kResTileLog) * kTileRecUnits;
}
size_t knot_area_bytes(const fstat_plan* p) {
  return (size_t(p->desc.ndet) * size_t(knot_stride(p)) * sizeof(double2) + 255) / 256 * 256;
}
// Plain-path slot: parameter block, y_a' and y_b' (n_fft each), knot area.
size_t plain_slot_bytes(const fstat_plan* p) {
  return slot_bytes(p->desc.n_fft, 2, knot_area_bytes(p));
}
int64_t plain_knot_offset(const fstat_plan* p) {
  return int64_t(kParamBytes + size_t(2) * p->desc.n_fft * sizeof(float2));
}

PlanConst make_const(const fstat_plan* p, const fstat_inputs* in) {
  const fstat_plan_desc& d = p->desc;
  PlanConst P;
  std::memset(&P, 0, sizeof P);
  P.ndet = d.ndet;
  P.D = d.sinc_halfwidth;
  P.tmpl_stride = tmpl_stride(p);
  P.dt = d.dt;
  P.inv_dt = 1.0 / d.dt;
  P.f_het = d.f_het;
  P.t_ref = d.t_ref;
  P.tau0 = d.tau0;
  P.max_delay = d.max_delay;
  P.sid_rate_cyc = d.sid_rate / (2.0 * M_PI);
  P.n_fft = d.n_fft;
  P.bin_lo = d.bin_lo;
  P.n_bins = d.n_bins;
  P.k_pad = p->k_pad;
  P.knot_stride = knot_stride(p);
  P.knot_gcap = knot_gcap(p);
  P.knot_ioff = knot_ioff(p);
  P.knot_soff = knot_soff(p);
  P.knot_toff = knot_toff(p);
  P.knot_bytes = int64_t(knot_area_bytes(p));
  P.res_taylor = std::fabs(2.0 * M_PI * P.sid_rate_cyc * d.dt) * double(kResTile / 2 + 1) <=
                 kTaylorMaxAngle;
  // the plain forward path's slot layout; the search and the adjoint paths
  // set their own
  P.slot_stride = int64_t(plain_slot_bytes(p));
  P.knot_offset = plain_knot_offset(p);
  if (in) {
    P.n_eph = in->n_eph;
    P.eph_t0 = in->eph_t0;
    P.eph_dt = in->eph_dt;
    P.inv_eph_dt = 1.0 / in->eph_dt;
    P.moments = in->moments;
  }
  for (int X = 0; X < d.ndet; ++X) {
    const fstat_detector& t = d.det[X];
    DetConst& c = P.det[X];
    c.t0 = t.t0;
    c.off = (d.tau0 - t.t0) / d.dt;
    c.lst0_cyc = (t.lon + d.sid_angle0) / (2.0 * M_PI);
    c.lat = t.lat;
    c.gamma = 0.5 * (t.az_x + t.az_y);
    c.sl = std::sin(c.lat);
    c.cl = std::cos(c.lat);
    c.s2g = std::sin(2.0 * c.gamma);
    c.c2g = std::cos(2.0 * c.gamma);
    c.w = 1.0 / t.noise_var;
    c.n = t.n;
    if (in) {
      c.x = static_cast<const float2*>(in->x[X]);
      c.valid = in->valid[X];
      c.ephem = in->ephem[X];
    }
  }
  return P;
}

fstat_status validate_inputs(const fstat_plan* p, const fstat_inputs* in, bool need_moments) {
  if (!in) return fail(FSTAT_EINVAL, "inputs is NULL");
  for (int X = 0; X < p->desc.ndet; ++X) {
    if (!in->x[X]) return fail(FSTAT_EINVAL, "inputs.x[%d] is NULL", X);
    if (!in->ephem[X]) return fail(FSTAT_EINVAL, "inputs.ephem[%d] is NULL", X);
  }
  if (need_moments && !in->moments) return fail(FSTAT_EINVAL, "inputs.moments is NULL");
  if (!finite_pos(in->eph_dt) || !std::isfinite(in->eph_t0) || in->n_eph < 4)
    return fail(FSTAT_EINVAL, "ephemeris: need eph_dt > 0, finite eph_t0, n_eph >= 4");
  const fstat_plan_desc& d = p->desc;
  const double span = kResTile * d.dt +
                      2.0 * (d.max_delay + (d.sinc_halfwidth + 2 + (1 << kKnotLogMax)) * d.dt);
  if (span / in->eph_dt + 4.0 > double(kNodeCap))
    return fail(FSTAT_EINVAL,
                "ephemeris spacing %.6g s too fine: a resampling tile spans %.6g s and stages at "
                "most %d nodes",
                in->eph_dt, span, kNodeCap);
  const double e_lo = in->eph_t0, e_hi = in->eph_t0 + double(in->n_eph - 1) * in->eph_dt;
  if (p->t_lo < e_lo || p->t_hi > e_hi)
    return fail(FSTAT_EINVAL, "ephemeris covers [%.6g, %.6g] but timing needs [%.6g, %.6g]", e_lo,
                e_hi, p->t_lo, p->t_hi);
  return FSTAT_OK;
}

fstat_status validate_ws(const fstat_plan* p, void* ws, size_t ws_bytes, int64_t* slots) {
  if (!ws) return fail(FSTAT_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(FSTAT_EINVAL, "workspace must be 256-byte aligned");
  const size_t sb = plain_slot_bytes(p);
  if (ws_bytes < kHeaderBytes + sb)
    return fail(FSTAT_EWORKSPACE, "workspace %zu bytes < %zu needed for one template", ws_bytes,
                kHeaderBytes + sb);
  *slots = int64_t((ws_bytes - kHeaderBytes) / sb);
  return FSTAT_OK;
}

// One workgroup per FFT work item.
unsigned fft_grid(const FftVariant&, int64_t n_items) {
  return unsigned(std::max<int64_t>(n_items, 1));
}
int64_t cols_items(const fstat_plan* p, const FftVariant& v, int n) {
  return ((int64_t(1) << p->log_c) / v.lines) * 2 * n;
}
int64_t rows_items(const fstat_plan* p, const FftVariant& v, int n) {
  return ((int64_t(1) << p->log_rr) / v.lines) * n;
}

// Resampling kernels for a supported interpolation half-width: knots solved
// ahead, and the tiles that solve their own timing.
using ResFn = void (*)(PlanConst, void*, ChunkMap, int);
template <bool GROUPED>
ResFn resample_kernel_g(int D) {
  switch (D) {
    case 4: return &k_resample<4, GROUPED>;
    case 6: return &k_resample<6, GROUPED>;
    case 8: return &k_resample<8, GROUPED>;
    case 10: return &k_resample<10, GROUPED>;
    case 12: return &k_resample<12, GROUPED>;
    case 16: return &k_resample<16, GROUPED>;
    default: return nullptr;
  }
}
template <bool GROUPED, bool KEP>
ResFn resample_own_kernel_g(int D) {
  switch (D) {
    case 4: return &k_resample_own<4, GROUPED, KEP>;
    case 6: return &k_resample_own<6, GROUPED, KEP>;
    case 8: return &k_resample_own<8, GROUPED, KEP>;
    case 10: return &k_resample_own<10, GROUPED, KEP>;
    case 12: return &k_resample_own<12, GROUPED, KEP>;
    case 16: return &k_resample_own<16, GROUPED, KEP>;
    default: return nullptr;
  }
}
// Plans with Keplerian rows take the kernels that carry the Kepler solver.
bool kepler_plan(const fstat_plan* p) { return (p->desc.flags & FSTAT_PLAN_KEPLER) != 0; }
using KnotFn = void (*)(PlanConst, void*, ChunkMap, int);
KnotFn knot_kernel(const fstat_plan* p, bool grouped) {
  if (kepler_plan(p)) return grouped ? &k_knots<true, true> : &k_knots<false, true>;
  return grouped ? &k_knots<true, false> : &k_knots<false, false>;
}
// Timing knots of the chunk's groups (grouped) or slots, ahead of the
// resampling (templates with a coarser knot spacing only; the kernel skips
// the others).  Nothing when the slots carry no knot area.
void launch_knots(const fstat_plan* p, const PlanConst& P, const ChunkMap& map, int slots,
                  bool grouped, int n_res, void* ws, hipStream_t st) {
  if (n_res < 1 || (!grouped && P.knot_offset == 0)) return;
  // at the coarsest knot spacing (finer ones loop)
  int64_t scap = 0;
  for (int X = 0; X < P.ndet; ++X)
    scap = std::max<int64_t>(scap, ((P.det[X].n - 1) >> kKnotLogMax) + 2);
  const int64_t blocks = knot_grid_blocks((P.k_pad >> kKnotLogMax) + 1) +
                         knot_tile_blocks(P.k_pad) + knot_samp_blocks(scap);
  hipLaunchKernelGGL(knot_kernel(p, grouped), dim3(unsigned(blocks), n_res, p->desc.ndet),
                     dim3(kKnotThreads), 0, st, P, ws, map, slots);
}

ResFn resample_kernel(const fstat_plan* p, bool grouped) {
  const int D = p->desc.sinc_halfwidth;
  return grouped ? resample_kernel_g<true>(D) : resample_kernel_g<false>(D);
}
ResFn resample_own_kernel(const fstat_plan* p, bool grouped) {
  const int D = p->desc.sinc_halfwidth;
  if (kepler_plan(p))
    return grouped ? resample_own_kernel_g<true, true>(D) : resample_own_kernel_g<false, true>(D);
  return grouped ? resample_own_kernel_g<true, false>(D) : resample_own_kernel_g<false, false>(D);
}
// Both resampling kernels over the chunk's groups (grouped) or slots; each
// skips the templates the other takes.  The own-timing kernel walks the tiles
// with at most 256 blocks per template.
void launch_resample(const fstat_plan* p, const PlanConst& P, const ChunkMap& map, int slots,
                     bool grouped, int n_res, void* ws, hipStream_t st) {
  const int64_t tiles = p->k_pad / kResTile;
  hipLaunchKernelGGL(resample_kernel(p, grouped), dim3(unsigned(tiles), n_res),
                     dim3(kResThreads), 0, st, P, ws, map, slots);
  hipLaunchKernelGGL(resample_own_kernel(p, grouped),
                     dim3(unsigned(std::min<int64_t>(tiles, 256)), n_res), dim3(kResThreads), 0,
                     st, P, ws, map, slots);
}

// Optional per-kernel timing: events recorded before and after each launch.
// Per-kernel device time from HIP events on the launch stream: open(k)
// records an event where kernel k starts, which also ends the kernel opened
// before it (launches follow one another on the stream); close() ends the
// last one.  One event per launch boundary.
struct KernelTimer {
  static constexpr int kKernels = 4;
  std::vector<hipEvent_t> ev;
  std::vector<int> who;  // kernel that starts at ev[i] (-1: none)
  bool on = false;
  hipStream_t st = nullptr;
  fstat_status record(int k) {
    if (!on) return FSTAT_OK;
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r == hipSuccess) r = hipEventRecord(e, st);
    if (r != hipSuccess) return check_hip(r, "timing event");
    ev.push_back(e);
    who.push_back(k);
    return FSTAT_OK;
  }
  fstat_status open(int k) { return record(k); }
  fstat_status close() { return record(-1); }
  ~KernelTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

// Launch the whole path for the template slots of one chunk.  grouped: the
// chunk's map names the sky/orbit groups to resample (possibly none, when a
// group continues from the previous chunk) and the group buffer every slot
// reads.  y_out: diagnostic path (resampled series only, per template).
RowOutput row_output(float* twoF, float2* fafb) {
  RowOutput o;
  std::memset(&o, 0, sizeof o);
  o.twoF = twoF;
  o.fafb = fafb;
  return o;
}

fstat_status launch_chunk(const fstat_plan* p, const PlanConst& P, const double* templates,
                          const ChunkMap& map, int slots, bool grouped, const RowOutput& out,
                          float2* y_out, void* ws, hipStream_t st, KernelTimer& tm) {
  fstat_status s;
  const int n = map.n_tmpl;
  if (!grouped) {
    // the grouped (search) path computed every parameter block up front
    if ((s = tm.open(0)) != FSTAT_OK) return s;
    hipLaunchKernelGGL(k_prologue, dim3((n + 63) / 64), dim3(64), 0, st, P, templates, map, ws);
  }
  const int n_res = grouped ? map.n_grp : n;
  const FftVariant cv = pick_cols(p->log_rr, cols_choice(p), grouped);
  const FftVariant rv = pick_rows(p->log_c, rows_choice(p), forward_row_mode(out));
  if (!resample_kernel(p, grouped) || !resample_own_kernel(p, grouped) || !cv.fn || !rv.fn)
    return fail(FSTAT_EINTERNAL, "no kernel for D=%d, FFT lines 2^%d x 2^%d",
                p->desc.sinc_halfwidth, p->log_rr, p->log_c);
  if (n_res > 0) {
    // (the knots are timed with the prologue)
    if ((s = tm.open(0)) != FSTAT_OK) return s;
    launch_knots(p, P, map, slots, grouped, n_res, ws, st);
    if ((s = tm.open(1)) != FSTAT_OK) return s;
    launch_resample(p, P, map, slots, grouped, n_res, ws, st);
  }
  if (y_out) {
    if ((s = tm.close()) != FSTAT_OK) return s;
    hipLaunchKernelGGL(k_copy_series, dim3(256, n), dim3(256), 0, st, P, ws, map, y_out);
    return check_hip(hipGetLastError(), "resample launch");
  }
  if ((s = tm.open(2)) != FSTAT_OK) return s;
  hipLaunchKernelGGL(reinterpret_cast<ColsFn>(const_cast<void*>(cv.fn)),
                     dim3(fft_grid(cv, cols_items(p, cv, n))), dim3(cv.threads), cv.lds, st, P, ws, map,
                     slots, 0, p->log_c,
                     p->rows_act);
  if ((s = tm.open(3)) != FSTAT_OK) return s;
  hipLaunchKernelGGL(reinterpret_cast<RowsFn>(const_cast<void*>(rv.fn)),
                     dim3(fft_grid(rv, rows_items(p, rv, n))), dim3(rv.threads), rv.lds, st, P, ws, map,
                     slots, p->log_rr, out);
  return check_hip(hipGetLastError(), "kernel launch");
}

// End the last kernel, wait for the stream, then sum each kernel's event
// intervals.
fstat_status finish_timer(KernelTimer& tm, hipStream_t st, float* kernel_ms, int64_t* launches) {
  fstat_status s = tm.close();
  if (s != FSTAT_OK) return s;
  s = check_hip(hipStreamSynchronize(st), "timing synchronise");
  if (s != FSTAT_OK) return s;
  for (int k = 0; k < KernelTimer::kKernels; ++k) {
    kernel_ms[k] = 0.f;
    launches[k] = 0;
  }
  for (size_t i = 0; i + 1 < tm.ev.size(); ++i) {
    const int k = tm.who[i];
    if (k < 0) continue;
    float ms = 0.f;
    s = check_hip(hipEventElapsedTime(&ms, tm.ev[i], tm.ev[i + 1]), "event time");
    if (s != FSTAT_OK) return s;
    kernel_ms[k] += ms;
    launches[k] += 1;
  }
  g_err.clear();
  return FSTAT_OK;
}

fstat_status set_lds_limits(const fstat_plan* p) {
  hipError_t e = hipSuccess;
  for (bool grouped : {false, true}) {
    const FftVariant v = pick_cols(p->log_rr, cols_choice(p), grouped);
    if (!v.fn) return fail(FSTAT_EINTERNAL, "no column kernel for lines of 2^%d", p->log_rr);
    e = hipFuncSetAttribute(v.fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(v.lds));
    if (e != hipSuccess) return check_hip(e, "hipFuncSetAttribute(cols)");
  }
  for (int mode : {int(kRow2F), int(kRowAdjoint), int(kRowConj), int(kRow2FExt), int(kRowCand)}) {
    const FftVariant v = pick_rows(p->log_c, rows_choice(p), mode);
    if (!v.fn) return fail(FSTAT_EINTERNAL, "no row kernel for lines of 2^%d", p->log_c);
    e = hipFuncSetAttribute(v.fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(v.lds));
    if (e != hipSuccess) return check_hip(e, "hipFuncSetAttribute(rows)");
  }
  return FSTAT_OK;
}

fstat_status run(const fstat_plan* p, const fstat_inputs* in, const double* templates,
                 int64_t ntmpl, float* twoF, void* fafb, void* y_out, void* ws, size_t ws_bytes,
                 void* stream, int64_t max_slots, KernelTimer* timer = nullptr) {
  if (!p) return fail(FSTAT_EINVAL, "plan is NULL");
  if (ntmpl < 0) return fail(FSTAT_EINVAL, "ntmpl < 0");
  if (ntmpl > 0 && !templates) return fail(FSTAT_EINVAL, "templates is NULL");
  if (ntmpl > 0 && !twoF && !y_out) return fail(FSTAT_EINVAL, "twoF is NULL");
  fstat_status s = validate_inputs(p, in, true);
  if (s != FSTAT_OK) return s;
  int64_t slots = 0;
  s = validate_ws(p, ws, ws_bytes, &slots);
  if (s != FSTAT_OK) return s;
  if (ntmpl == 0) return ok();
  slots = std::min(slots, max_slots);
  slots = std::min<int64_t>(slots, kMaxSlots);
  s = set_lds_limits(p);
  if (s != FSTAT_OK) return s;
  PlanConst P = make_const(p, in);
  hipStream_t st = static_cast<hipStream_t>(stream);
  KernelTimer none;
  KernelTimer& tm = timer ? *timer : none;
  tm.st = st;
  hipLaunchKernelGGL(k_twiddles, dim3(kTwLen / 256), dim3(256), 0, st, ws);
  for (int64_t t = 0; t < ntmpl; t += slots) {
    ChunkMap map;
    std::memset(&map, 0, sizeof map);
    map.n_tmpl = int(std::min<int64_t>(slots, ntmpl - t));
    for (int i = 0; i < map.n_tmpl; ++i) map.tmpl[i] = t + i;
    s = launch_chunk(p, P, templates, map, int(slots), false,
                     row_output(twoF, static_cast<float2*>(fafb)), static_cast<float2*>(y_out),
                     ws, st, tm);
    if (s != FSTAT_OK) return s;
  }
  return ok();
}

// Adjoint workspace slot: parameters, four arrays (y' / F', then the adjoint
// spectrum and its transform), 8 doubles of gradient partials per resampling
// tile (padded to 256 bytes), and the knot area of the forward resampling
// (so that its 2F is the forward path's, bit for bit).
size_t grad_part_bytes(const fstat_plan* p) {
  return (size_t(p->k_pad / kResTile) * 8 * sizeof(double) + 255) / 256 * 256;
}
size_t grad_slot_bytes(const fstat_plan* p) {
  return slot_bytes(p->desc.n_fft, 4, grad_part_bytes(p) + knot_area_bytes(p));
}

using GradFn = void (*)(PlanConst, void*);
template <bool ONEHOT, bool KEP>
GradFn grad_kernel_o(int D) {
  switch (D) {
    case 4: return &k_grad<4, ONEHOT, KEP>;
    case 6: return &k_grad<6, ONEHOT, KEP>;
    case 8: return &k_grad<8, ONEHOT, KEP>;
    case 10: return &k_grad<10, ONEHOT, KEP>;
    case 12: return &k_grad<12, ONEHOT, KEP>;
    case 16: return &k_grad<16, ONEHOT, KEP>;
    default: return nullptr;
  }
}
GradFn grad_kernel(const fstat_plan* p, bool onehot) {
  const int D = p->desc.sinc_halfwidth;
  if (kepler_plan(p))
    return onehot ? grad_kernel_o<true, true>(D) : grad_kernel_o<false, true>(D);
  return onehot ? grad_kernel_o<true, false>(D) : grad_kernel_o<false, false>(D);
}

using BinFn = void (*)(PlanConst, void*, ChunkMap, const int64_t*);
template <bool KEP>
BinFn resample_bin_kernel_k(int D) {
  switch (D) {
    case 4: return &k_resample_bin<4, KEP>;
    case 6: return &k_resample_bin<6, KEP>;
    case 8: return &k_resample_bin<8, KEP>;
    case 10: return &k_resample_bin<10, KEP>;
    case 12: return &k_resample_bin<12, KEP>;
    case 16: return &k_resample_bin<16, KEP>;
    default: return nullptr;
  }
}
BinFn resample_bin_kernel(const fstat_plan* p) {
  return kepler_plan(p) ? resample_bin_kernel_k<true>(p->desc.sinc_halfwidth)
                        : resample_bin_kernel_k<false>(p->desc.sinc_halfwidth);
}

// Single-bin adjoint slot: the parameter block and 8 doubles of partials per
// resampling tile, padded to 256 bytes.
size_t grad_bin_slot_bytes(const fstat_plan* p) {
  const size_t tiles = size_t(p->k_pad / kResTile);
  return kParamBytes + (tiles * 8 * sizeof(double) + 255) / 256 * 256;
}

// Single-bin launch sequence: prologue, resampling with the one-bin direct
// transform reduced per tile, F'(m) / 2F(m) / H per template, the gradient
// sums with X in closed form, and their per-template totals.
fstat_status launch_grad_bin_chunk(const fstat_plan* p, const PlanConst& P,
                                   const double* templates, const ChunkMap& map, int slots,
                                   const int64_t* bins, float* twoF, double* grad, void* ws,
                                   hipStream_t st) {
  const int n = map.n_tmpl;
  const unsigned tiles = unsigned(p->k_pad / kResTile);
  hipLaunchKernelGGL(k_prologue, dim3((n + 63) / 64), dim3(64), 0, st, P, templates, map, ws);
  hipLaunchKernelGGL(resample_bin_kernel(p), dim3(tiles, n),
                     dim3(kResThreads), 0, st, P, ws, map, bins);
  hipLaunchKernelGGL(k_bin_final, dim3(n), dim3(kFinalThreads), 0, st, P, ws, map,
                     int64_t(tiles), bins, twoF);
  hipLaunchKernelGGL(grad_kernel(p, true), dim3(tiles, n),
                     dim3(kResThreads), 0, st, P, ws);
  hipLaunchKernelGGL(k_grad_final, dim3(n), dim3(kFinalThreads), 0, st, P, ws, map,
                     int64_t(tiles), grad);
  return check_hip(hipGetLastError(), "single-bin adjoint launch");
}

// Adjoint launch sequence for the template slots of one chunk: the forward
// path up to F' (with 2F when twoF is set), H = g conj(F') into arrays 2/3,
// X = FFT(H) (conjugated) back into arrays 0/1, then the per-tile gradient
// sums and their per-template totals.
fstat_status launch_grad_chunk(const fstat_plan* p, const PlanConst& P, const double* templates,
                               const ChunkMap& map, int slots, const float* gin, double* grad,
                               float* twoF, void* ws, hipStream_t st) {
  const int n = map.n_tmpl;
  const unsigned tiles = unsigned(p->k_pad / kResTile);
  hipLaunchKernelGGL(k_prologue, dim3((n + 63) / 64), dim3(64), 0, st, P, templates, map, ws);
  launch_knots(p, P, map, slots, false, n, ws, st);
  launch_resample(p, P, map, slots, false, n, ws, st);
  const FftVariant cv = pick_cols(p->log_rr, cols_choice(p), false);
  const ColsFn cols = reinterpret_cast<ColsFn>(const_cast<void*>(cv.fn));
  const dim3 cgrid(fft_grid(cv, cols_items(p, cv, n)));
  const FftVariant ra = pick_rows(p->log_c, rows_choice(p), kRowAdjoint);
  const FftVariant rc = pick_rows(p->log_c, rows_choice(p), kRowConj);
  const dim3 rgrid_a(fft_grid(ra, rows_items(p, ra, n))),
      rgrid_c(fft_grid(rc, rows_items(p, rc, n)));
  hipLaunchKernelGGL(cols, cgrid, dim3(cv.threads), cv.lds, st, P, ws, map, slots, 0,
                     p->log_c, p->rows_act);
  RowOutput oa = row_output(twoF, nullptr);
  oa.gin = gin;
  hipLaunchKernelGGL(reinterpret_cast<RowsFn>(const_cast<void*>(ra.fn)), rgrid_a, dim3(ra.threads),
                     ra.lds, st, P, ws, map, slots, p->log_rr, oa);
  hipLaunchKernelGGL(cols, cgrid, dim3(cv.threads), cv.lds, st, P, ws, map, slots, 2,
                     p->log_c, int64_t(1) << p->log_rr);
  hipLaunchKernelGGL(reinterpret_cast<RowsFn>(const_cast<void*>(rc.fn)), rgrid_c, dim3(rc.threads),
                     rc.lds, st, P, ws, map, slots, p->log_rr,
                     row_output(nullptr, nullptr));
  hipLaunchKernelGGL(grad_kernel(p, false), dim3(tiles, n),
                     dim3(kResThreads), 0, st, P, ws);
  hipLaunchKernelGGL(k_grad_final, dim3(n), dim3(kFinalThreads), 0, st, P, ws, map,
                     int64_t(tiles), grad);
  return check_hip(hipGetLastError(), "adjoint launch");
}

}  // namespace

// A template bank planned for the grouped path.
struct fstat_search {
  const fstat_plan* plan;
  int slots;
  uint32_t flags;
  int64_t ntmpl, ngroups;
  std::vector<ChunkMap> chunks;
  // captured launch sequence and the arguments it was captured with
  hipGraphExec_t exec = nullptr;
  std::vector<uint64_t> key;
  ~fstat_search() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

// Independent searches captured together: one HIP graph whose branches
// (lanes) run the searches' launch sequences concurrently.
struct fstat_batch {
  std::vector<fstat_search*> searches;
  std::vector<int> lane_of;  // lane of each search (balanced by estimated work)
  int lanes = 1;
  int device = -1;
  std::vector<hipStream_t> lane_st;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraphExec_t exec = nullptr;
  std::vector<uint64_t> key;
  ~fstat_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (hipStream_t s : lane_st) (void)hipStreamDestroy(s);
    for (hipEvent_t e : join) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
  }
};

namespace {

uint64_t key_ptr(const void* q) { return uint64_t(reinterpret_cast<uintptr_t>(q)); }
uint64_t key_f64(double v) {
  uint64_t b;
  std::memcpy(&b, &v, sizeof b);
  return b;
}
// Everything of the inputs that a captured launch sequence bakes into its
// kernel arguments (make_const): the device pointers and ephemeris scalars
// of the plan's detectors and the moments.
void inputs_key(const fstat_plan* p, const fstat_inputs* in, std::vector<uint64_t>& key) {
  for (int X = 0; X < p->desc.ndet; ++X) {
    key.push_back(key_ptr(in->x[X]));
    key.push_back(key_ptr(in->valid[X]));
    key.push_back(key_ptr(in->ephem[X]));
  }
  key.push_back(uint64_t(in->n_eph));
  key.push_back(key_f64(in->eph_t0));
  key.push_back(key_f64(in->eph_dt));
  key.push_back(key_ptr(in->moments));
}

// Templates with the same sky position and orbit share the resampled series;
// an isolated source (asini = 0) ignores porb and tp (and the Keplerian
// elements of rows of `stride` 10).
bool same_timing(const double* a, const double* b, int stride) {
  if (a[0] != b[0] || a[1] != b[1] || a[5] != b[5]) return false;
  if (a[5] == 0.0) return true;
  if (stride >= FSTAT_TEMPLATE_STRIDE_KEPLER && (a[8] != b[8] || a[9] != b[9])) return false;
  return a[6] == b[6] && a[7] == b[7];
}

// Search workspace: header, template slots, group buffers, then one
// parameter block per template.
size_t search_params_offset(const fstat_search* sr) {
  const fstat_plan* p = sr->plan;
  return kHeaderBytes + size_t(sr->slots) * slot_bytes(p->desc.n_fft) +
         size_t(sr->slots) * group_bytes(p->k_pad, int64_t(knot_area_bytes(p)));
}
size_t search_ws_bytes(const fstat_search* sr) {
  return search_params_offset(sr) + size_t(sr->ntmpl) * kParamBytes;
}

fstat_status search_launch(fstat_search* sr, const fstat_inputs* in, const double* templates,
                           const RowOutput& out, void* ws, hipStream_t st, KernelTimer& tm) {
  const fstat_plan* p = sr->plan;
  PlanConst P = make_const(p, in);
  // template slots hold parameters and transforms only; the knots live in the
  // group buffers
  P.slot_stride = int64_t(slot_bytes(p->desc.n_fft));
  P.knot_offset = 0;
  P.params = static_cast<char*>(ws) + search_params_offset(sr);
  hipLaunchKernelGGL(k_twiddles, dim3(kTwLen / 256), dim3(256), 0, st, ws);
  fstat_status s0 = tm.open(0);
  if (s0 != FSTAT_OK) return s0;
  const int64_t nt = std::max<int64_t>(sr->ntmpl, sr->slots);
  hipLaunchKernelGGL(k_params, dim3(unsigned((nt + 63) / 64)), dim3(64), 0, st, P, templates,
                     sr->ntmpl, ws, sr->slots, out);
  for (const ChunkMap& map : sr->chunks) {
    fstat_status s = launch_chunk(p, P, templates, map, sr->slots, true, out, nullptr, ws, st, tm);
    if (s != FSTAT_OK) return s;
  }
  return FSTAT_OK;
}

fstat_status search_check(fstat_search* sr, const fstat_inputs* in, const double* templates,
                          bool have_output, void* ws, size_t ws_bytes) {
  if (!sr) return fail(FSTAT_EINVAL, "search is NULL");
  if (sr->ntmpl > 0 && (!templates || !have_output))
    return fail(FSTAT_EINVAL, "templates or output is NULL");
  fstat_status s = validate_inputs(sr->plan, in, true);
  if (s != FSTAT_OK) return s;
  if (!ws) return fail(FSTAT_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(FSTAT_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < search_ws_bytes(sr))
    return fail(FSTAT_EWORKSPACE, "workspace %zu bytes < %zu for this search", ws_bytes,
                search_ws_bytes(sr));
  return set_lds_limits(sr->plan);
}

// Run a checked search: directly, or (FSTAT_SEARCH_GRAPH) by replaying the
// launch sequence captured for exactly these arguments.
fstat_status search_run_out(fstat_search* search, const fstat_inputs* in,
                            const double* templates, const RowOutput& out, void* workspace,
                            size_t ws_bytes, void* stream) {
  if (search->ntmpl == 0) return ok();
  hipStream_t st = static_cast<hipStream_t>(stream);
  KernelTimer none;
  none.st = st;
  fstat_status s;
  if (!(search->flags & FSTAT_SEARCH_GRAPH)) {
    s = search_launch(search, in, templates, out, workspace, st, none);
    return s == FSTAT_OK ? ok() : s;
  }
  if (!st) return fail(FSTAT_EINVAL, "graph replay needs a non-null stream");
  uint32_t thr = 0;
  std::memcpy(&thr, &out.threshold, sizeof thr);
  std::vector<uint64_t> key;
  inputs_key(search->plan, in, key);
  for (uint64_t v : {key_ptr(templates), key_ptr(out.twoF), key_ptr(out.fafb), key_ptr(out.cand),
                     key_ptr(out.count), key_ptr(out.best), uint64_t(out.cap),
                     uint64_t(thr) | (uint64_t(out.acc) << 32), key_ptr(workspace),
                     uint64_t(ws_bytes)})
    key.push_back(v);
  if (!search->exec || key != search->key) {
    if (search->exec) {
      (void)hipGraphExecDestroy(search->exec);
      search->exec = nullptr;
    }
    s = check_hip(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
    if (s != FSTAT_OK) return s;
    fstat_status ls = search_launch(search, in, templates, out, workspace, st, none);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (ls != FSTAT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return ls;
    }
    if ((s = check_hip(e, "end capture")) != FSTAT_OK) return s;
    e = hipGraphInstantiate(&search->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if ((s = check_hip(e, "graph instantiate")) != FSTAT_OK) return s;
    search->key = key;
  }
  s = check_hip(hipGraphLaunch(search->exec, st), "graph launch");
  return s == FSTAT_OK ? ok() : s;
}

}  // namespace

extern "C" {

fstat_status fstat_search_create(const fstat_plan* plan, const double* templates, int64_t ntmpl,
                                 int32_t slots, uint32_t flags, fstat_search** out) {
  if (!out) return fail(FSTAT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!plan) return fail(FSTAT_EINVAL, "plan is NULL");
  if (ntmpl < 0 || (ntmpl > 0 && !templates)) return fail(FSTAT_EINVAL, "templates / ntmpl invalid");
  if (slots < 1 || slots > kMaxSlots)
    return fail(FSTAT_EINVAL, "slots=%d outside [1, %d]", slots, kMaxSlots);
  if (flags & ~uint32_t(FSTAT_SEARCH_GRAPH | FSTAT_SEARCH_ACCUMULATE))
    return fail(FSTAT_EINVAL, "unknown flags");
  fstat_search* sr = new (std::nothrow) fstat_search;
  if (!sr) return fail(FSTAT_EINVAL, "host allocation failed");
  sr->plan = plan;
  sr->slots = slots;
  sr->flags = flags;
  sr->ntmpl = ntmpl;
  // group = maximal run of consecutive templates with the same timing; the
  // group buffer of group number g is g mod slots (a chunk holds at most
  // `slots` templates, so at most `slots` groups, all distinct mod slots).
  // A group that fits a chunk is never split: the chunk closes early instead
  // (measured: chunks that end on group boundaries run the column pass ~20 %
  // faster than full chunks that split groups); larger groups fill chunks.
  std::vector<int64_t> gstart;
  const int stride = tmpl_stride(plan);
  for (int64_t t = 0; t < ntmpl; ++t) {
    const double* row = templates + t * stride;
    if (t == 0 || !same_timing(row, row - stride, stride)) gstart.push_back(t);
  }
  gstart.push_back(ntmpl);
  ChunkMap map;
  std::memset(&map, 0, sizeof map);
  auto close_chunk = [&]() {
    sr->chunks.push_back(map);
    std::memset(&map, 0, sizeof map);
  };
  const int64_t ngroups = int64_t(gstart.size()) - 1;
  for (int64_t group = 0; group < ngroups; ++group) {
    const int64_t size = gstart[group + 1] - gstart[group];
    if (map.n_tmpl > 0 && size <= slots && map.n_tmpl + size > slots) close_chunk();
    for (int64_t t = gstart[group]; t < gstart[group + 1]; ++t) {
      if (map.n_tmpl == slots) close_chunk();
      const int slot = map.n_tmpl++;
      if (t == gstart[group]) {
        map.grp_slot[map.n_grp] = slot;
        map.grp_buf[map.n_grp] = int32_t(group % slots);
        ++map.n_grp;
      }
      map.tmpl[slot] = t;
      map.tmpl_buf[slot] = int32_t(group % slots);
    }
  }
  if (map.n_tmpl > 0) sr->chunks.push_back(map);
  sr->ngroups = ngroups;
  // the row pass of chunk i clears the status words of the group buffers
  // chunk i + 1 resamples (k_params clears them all for chunk 0)
  for (size_t i = 0; i + 1 < sr->chunks.size(); ++i) {
    ChunkMap& cur = sr->chunks[i];
    const ChunkMap& nx = sr->chunks[i + 1];
    cur.n_reset = nx.n_grp;
    for (int k = 0; k < nx.n_grp; ++k) cur.reset_buf[k] = nx.grp_buf[k];
  }
  *out = sr;
  return ok();
}

void fstat_search_destroy(fstat_search* search) { delete search; }

fstat_status fstat_search_info(const fstat_search* search, size_t* ws_bytes, int64_t* ngroups,
                               int64_t* nchunks) {
  if (!search) return fail(FSTAT_EINVAL, "search is NULL");
  if (ws_bytes) *ws_bytes = search_ws_bytes(search);
  if (ngroups) *ngroups = search->ngroups;
  if (nchunks) *nchunks = int64_t(search->chunks.size());
  return ok();
}

fstat_status fstat_search_run(fstat_search* search, const fstat_inputs* in,
                              const double* templates, float* twoF, void* fafb, void* workspace,
                              size_t ws_bytes, void* stream) {
  fstat_status s = search_check(search, in, templates, twoF != nullptr, workspace, ws_bytes);
  if (s != FSTAT_OK) return s;
  RowOutput out = row_output(twoF, static_cast<float2*>(fafb));
  out.acc = (search->flags & FSTAT_SEARCH_ACCUMULATE) ? 1 : 0;
  return search_run_out(search, in, templates, out, workspace, ws_bytes, stream);
}

fstat_status fstat_search_run_candidates(fstat_search* search, const fstat_inputs* in,
                                         const double* templates, float threshold,
                                         fstat_candidate* cand, int64_t capacity,
                                         int64_t* count, uint64_t* best, void* workspace,
                                         size_t ws_bytes, void* stream) {
  if (!count) return fail(FSTAT_EINVAL, "count is NULL");
  if (capacity < 0 || (capacity > 0 && !cand)) return fail(FSTAT_EINVAL, "cand / capacity invalid");
  if (!std::isfinite(threshold)) return fail(FSTAT_EINVAL, "threshold must be finite");
  fstat_status s = search_check(search, in, templates, true, workspace, ws_bytes);
  if (s != FSTAT_OK) return s;
  RowOutput out = row_output(nullptr, nullptr);
  out.cand = cand;
  out.cap = capacity;
  out.count = reinterpret_cast<unsigned long long*>(count);
  out.best = reinterpret_cast<unsigned long long*>(best);
  out.threshold = threshold;
  return search_run_out(search, in, templates, out, workspace, ws_bytes, stream);
}

fstat_status fstat_search_run_profiled(fstat_search* search, const fstat_inputs* in,
                                       const double* templates, float* twoF, void* workspace,
                                       size_t ws_bytes, void* stream, float* kernel_ms,
                                       int64_t* launches) {
  if (!kernel_ms || !launches) return fail(FSTAT_EINVAL, "kernel_ms or launches is NULL");
  fstat_status s = search_check(search, in, templates, twoF != nullptr, workspace, ws_bytes);
  if (s != FSTAT_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KernelTimer tm;
  tm.on = true;
  tm.st = st;
  if (search->ntmpl > 0) {
    RowOutput out = row_output(twoF, nullptr);
    out.acc = (search->flags & FSTAT_SEARCH_ACCUMULATE) ? 1 : 0;
    s = search_launch(search, in, templates, out, workspace, st, tm);
    if (s != FSTAT_OK) return s;
  }
  return finish_timer(tm, st, kernel_ms, launches);
}


fstat_status fstat_batch_create(fstat_search* const* searches, int32_t n, int32_t lanes,
                                fstat_batch** out) {
  if (!out) return fail(FSTAT_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || !searches) return fail(FSTAT_EINVAL, "searches / n invalid");
  if (lanes < 1 || lanes > FSTAT_MAX_BATCH_LANES)
    return fail(FSTAT_EINVAL, "lanes=%d outside [1, %d]", lanes, FSTAT_MAX_BATCH_LANES);
  for (int32_t i = 0; i < n; ++i)
    if (!searches[i]) return fail(FSTAT_EINVAL, "search %d is NULL", i);
  fstat_batch* b = new (std::nothrow) fstat_batch;
  if (!b) return fail(FSTAT_EINVAL, "host allocation failed");
  b->searches.assign(searches, searches + n);
  b->lanes = std::min<int32_t>(lanes, n);
  // longest first onto the least loaded lane; work ~ templates x FFT length
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto cost = [&](int i) {
    return double(searches[i]->ntmpl) * double(searches[i]->plan->desc.n_fft);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost(a) > cost(c); });
  std::vector<double> load(b->lanes, 0.0);
  b->lane_of.assign(n, 0);
  for (int i : order) {
    const int l = int(std::min_element(load.begin(), load.end()) - load.begin());
    b->lane_of[i] = l;
    load[l] += cost(i);
  }
  *out = b;
  return ok();
}

void fstat_batch_destroy(fstat_batch* batch) { delete batch; }

fstat_status fstat_batch_run(fstat_batch* b, const fstat_inputs* const* in,
                             const double* const* templates, float* const* twoF,
                             void* const* workspace, const size_t* ws_bytes, void* stream) {
  if (!b) return fail(FSTAT_EINVAL, "batch is NULL");
  if (!in || !templates || !twoF || !workspace || !ws_bytes)
    return fail(FSTAT_EINVAL, "argument arrays must not be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!st) return fail(FSTAT_EINVAL, "a batch runs from a graph: it needs a non-null stream");
  const int n = int(b->searches.size());
  std::vector<uint64_t> key;
  key.reserve(size_t(n) * 24);
  for (int i = 0; i < n; ++i) {
    if (!in[i]) return fail(FSTAT_EINVAL, "inputs %d is NULL", i);
    fstat_status s = search_check(b->searches[i], in[i], templates[i], twoF[i] != nullptr,
                                  workspace[i], ws_bytes[i]);
    if (s != FSTAT_OK) return s;
    inputs_key(b->searches[i]->plan, in[i], key);
    key.push_back(key_ptr(templates[i]));
    key.push_back(key_ptr(twoF[i]));
    key.push_back(key_ptr(workspace[i]));
    key.push_back(uint64_t(ws_bytes[i]));
  }
  int dev = 0;
  fstat_status s = check_hip(hipGetDevice(&dev), "get device");
  if (s != FSTAT_OK) return s;
  if (b->device != dev) {
    // lane streams and events belong to the device current at first use
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    for (hipStream_t x : b->lane_st) (void)hipStreamDestroy(x);
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    b->lane_st.assign(b->lanes, nullptr);
    b->join.assign(b->lanes, nullptr);
    b->fork = nullptr;
    b->device = -1;
    for (int l = 0; l < b->lanes; ++l) {
      if ((s = check_hip(hipStreamCreateWithFlags(&b->lane_st[l], hipStreamNonBlocking),
                         "lane stream")) != FSTAT_OK)
        return s;
      if ((s = check_hip(hipEventCreateWithFlags(&b->join[l], hipEventDisableTiming),
                         "lane event")) != FSTAT_OK)
        return s;
    }
    if ((s = check_hip(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "fork event")) !=
        FSTAT_OK)
      return s;
    b->device = dev;
  }
  if (!b->exec || key != b->key) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    if ((s = check_hip(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal),
                       "begin capture")) != FSTAT_OK)
      return s;
    hipError_t e = hipEventRecord(b->fork, st);
    for (int l = 0; l < b->lanes && e == hipSuccess; ++l)
      e = hipStreamWaitEvent(b->lane_st[l], b->fork, 0);
    fstat_status ls = check_hip(e, "fork");
    KernelTimer none;
    for (int i = 0; i < n && ls == FSTAT_OK; ++i) {
      fstat_search* sr = b->searches[i];
      if (sr->ntmpl == 0) continue;
      RowOutput out = row_output(twoF[i], nullptr);
      out.acc = (sr->flags & FSTAT_SEARCH_ACCUMULATE) ? 1 : 0;
      hipStream_t ls_st = b->lane_st[b->lane_of[i]];
      none.st = ls_st;
      ls = search_launch(sr, in[i], templates[i], out, workspace[i], ls_st, none);
    }
    for (int l = 0; l < b->lanes && ls == FSTAT_OK; ++l) {
      e = hipEventRecord(b->join[l], b->lane_st[l]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, b->join[l], 0);
      ls = check_hip(e, "join");
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (ls != FSTAT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return ls;
    }
    if ((s = check_hip(e, "end capture")) != FSTAT_OK) return s;
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if ((s = check_hip(e, "graph instantiate")) != FSTAT_OK) return s;
    b->key = key;
  }
  s = check_hip(hipGraphLaunch(b->exec, st), "graph launch");
  return s == FSTAT_OK ? ok() : s;
}

const char* fstat_version(void) { return "fstat-gfx950 0.1"; }

const char* fstat_last_error(void) { return g_err.c_str(); }

fstat_status fstat_plan_create(const fstat_plan_desc* desc, fstat_plan** out) {
  if (!out) return fail(FSTAT_EINVAL, "out is NULL");
  *out = nullptr;
  fstat_status s = validate_desc(desc);
  if (s != FSTAT_OK) return s;
  fstat_plan* p = new (std::nothrow) fstat_plan;
  if (!p) return fail(FSTAT_EINVAL, "host allocation failed");
  p->desc = *desc;
  p->log_n = ilog2(desc->n_fft);
  // column length 2^floor(log N / 2): the shorter column pass gets the wider
  // (better coalesced) line groups
  p->log_rr = desc->tune_col_log_len ? desc->tune_col_log_len : p->log_n / 2;
  p->log_c = p->log_n - p->log_rr;
  if (p->log_rr < 6 || p->log_rr > 12 || p->log_c < 6 || p->log_c > 12) {
    delete p;
    return fail(FSTAT_EINVAL, "tune_col_log_len=%d: both FFT passes need lengths 2^6..2^12",
                desc->tune_col_log_len);
  }
  const int cmax = cols_lines_max(p->log_rr), rmax = rows_lines_max(p->log_c);
  const int tc = desc->tune_col_lines, tr = desc->tune_row_lines;
  if ((tc != 0 && tc != cmax && tc != cmax / 2) || (tr != 0 && tr != rmax && tr != rmax / 2)) {
    delete p;
    return fail(FSTAT_EINVAL,
                "tune_col_lines=%d / tune_row_lines=%d: accepted 0, %d or %d / 0, %d or %d", tc,
                tr, cmax, cmax / 2, rmax, rmax / 2);
  }
  if (desc->tune_fft_radix != 0 && desc->tune_fft_radix != 16 && desc->tune_fft_radix != 32) {
    delete p;
    return fail(FSTAT_EINVAL, "tune_fft_radix=%d: accepted 0, 16 or 32", desc->tune_fft_radix);
  }
  p->fft_mlr = desc->tune_fft_radix == 16 ? 4 : 5;
  // automatic (measured): columns in the half line count (256-thread
  // workgroups, two per compute unit) while that still gives 8 columns
  // (64-byte runs per row; at 2^11-point columns the 4-column half count ran
  // the pass 24 % slower than 8 columns in one workgroup), rows in the full
  // count (512 threads)
  p->cols_half = (tc == 0 ? cmax / 2 >= 8 : tc == cmax / 2) && cmax > 1;
  p->rows_half = tr == rmax / 2 && rmax > 1;
  p->cols_lines = p->cols_half ? cmax / 2 : cmax;
  p->rows_lines = p->rows_half ? rmax / 2 : rmax;
  // grid points that can be non-zero: up to the last sample plus the delay
  // bound plus the interpolation half-width
  double t_end = -INFINITY, t_beg = INFINITY;
  for (int X = 0; X < desc->ndet; ++X) {
    t_end = std::max(t_end, desc->det[X].t0 + double(desc->det[X].n - 1) * desc->dt);
    t_beg = std::min(t_beg, desc->det[X].t0);
  }
  const double k_act =
      std::ceil((t_end + desc->max_delay - desc->tau0) / desc->dt) + desc->sinc_halfwidth + 2;
  const int64_t quant = std::max<int64_t>(kResTile, int64_t(1) << p->log_c);
  p->k_pad = (int64_t(k_act) + quant - 1) / quant * quant;
  if (p->k_pad > desc->n_fft) {
    delete p;
    return fail(FSTAT_EINVAL,
                "n_fft=%lld too short: data span plus delays needs %lld grid points (padded)",
                (long long)desc->n_fft, (long long)(int64_t(k_act)));
  }
  p->rows_act = p->k_pad >> p->log_c;
  // a tile evaluates the timing up to D + 2 + G samples beyond the delay
  // bound (the staged window and its last phase knot)
  const double margin =
      desc->max_delay + double(desc->sinc_halfwidth + 2 + (1 << kKnotLogMax)) * desc->dt + 1.0;
  p->t_lo = std::min(desc->tau0, t_beg) - margin;
  p->t_hi = std::max(desc->tau0 + double(p->k_pad) * desc->dt, t_end) + margin;
  *out = p;
  return ok();
}

void fstat_plan_destroy(fstat_plan* plan) { delete plan; }

fstat_status fstat_plan_info(const fstat_plan* plan, int64_t* k_pad, int32_t* log_col_len,
                             int32_t* log_row_len) {
  if (!plan) return fail(FSTAT_EINVAL, "plan is NULL");
  if (k_pad) *k_pad = plan->k_pad;
  if (log_col_len) *log_col_len = plan->log_rr;
  if (log_row_len) *log_row_len = plan->log_c;
  return ok();
}

fstat_status fstat_workspace_size(const fstat_plan* plan, int64_t batch, size_t* bytes) {
  if (!plan || !bytes) return fail(FSTAT_EINVAL, "plan or bytes is NULL");
  if (batch < 1) return fail(FSTAT_EINVAL, "batch must be >= 1");
  *bytes = kHeaderBytes + size_t(batch) * plain_slot_bytes(plan);
  return ok();
}

fstat_status fstat_antenna_moments(const fstat_plan* plan, const fstat_inputs* in,
                                   double* moments, void* workspace, size_t ws_bytes,
                                   void* stream) {
  if (!plan) return fail(FSTAT_EINVAL, "plan is NULL");
  if (!moments) return fail(FSTAT_EINVAL, "moments is NULL");
  if (!in) return fail(FSTAT_EINVAL, "inputs is NULL");
  if (!workspace) return fail(FSTAT_EINVAL, "workspace is NULL");
  if (ws_bytes < kHeaderBytes)
    return fail(FSTAT_EWORKSPACE, "workspace %zu bytes < %zu", ws_bytes, kHeaderBytes);
  PlanConst P = make_const(plan, in);
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* partial = static_cast<double*>(workspace);
  hipLaunchKernelGGL(k_moments_partial, dim3(kMomBlocks, plan->desc.ndet), dim3(kMomThreads), 0,
                     st, P, partial);
  hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(64), 0, st, plan->desc.ndet, partial, moments);
  fstat_status s = check_hip(hipGetLastError(), "moments launch");
  return s == FSTAT_OK ? ok() : s;
}

fstat_status fstat_compute_2f(const fstat_plan* plan, const fstat_inputs* in,
                              const double* templates, int64_t ntmpl, float* twoF, void* fafb,
                              void* workspace, size_t ws_bytes, void* stream) {
  return run(plan, in, templates, ntmpl, twoF, fafb, nullptr, workspace, ws_bytes, stream, 1);
}

fstat_status fstat_compute_2f_batched(const fstat_plan* plan, const fstat_inputs* in,
                                      const double* templates, int64_t ntmpl, float* twoF,
                                      void* fafb, void* workspace, size_t ws_bytes,
                                      void* stream) {
  return run(plan, in, templates, ntmpl, twoF, fafb, nullptr, workspace, ws_bytes, stream,
             int64_t(1) << 40);
}

fstat_status fstat_compute_2f_profiled(const fstat_plan* plan, const fstat_inputs* in,
                                       const double* templates, int64_t ntmpl, float* twoF,
                                       void* workspace, size_t ws_bytes, int64_t max_batch,
                                       void* stream, float* kernel_ms, int64_t* launches) {
  if (!kernel_ms || !launches) return fail(FSTAT_EINVAL, "kernel_ms or launches is NULL");
  if (max_batch < 1) return fail(FSTAT_EINVAL, "max_batch must be >= 1");
  KernelTimer tm;
  tm.on = true;
  fstat_status s = run(plan, in, templates, ntmpl, twoF, nullptr, nullptr, workspace, ws_bytes,
                       stream, max_batch, &tm);
  if (s != FSTAT_OK) return s;
  return finish_timer(tm, static_cast<hipStream_t>(stream), kernel_ms, launches);
}

fstat_status fstat_autotune(const fstat_plan_desc* desc, const fstat_inputs* in,
                            const double* templates, int64_t ntmpl, float* twoF, void* workspace,
                            size_t ws_bytes, void* stream, fstat_plan_desc* best,
                            float* best_ms) {
  if (!best || !best_ms) return fail(FSTAT_EINVAL, "best or best_ms is NULL");
  fstat_status s = validate_desc(desc);
  if (s != FSTAT_OK) return s;
  if (ntmpl < 1 || !templates || !twoF) return fail(FSTAT_EINVAL, "need ntmpl >= 1 sample templates and twoF");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((s = check_hip(hipEventCreate(&e0), "event")) != FSTAT_OK) return s;
  if ((s = check_hip(hipEventCreate(&e1), "event")) != FSTAT_OK) {
    (void)hipEventDestroy(e0);
    return s;
  }
  const int log_n = ilog2(desc->n_fft);
  const int splits[2] = {log_n / 2, (log_n + 1) / 2};
  float best_t = INFINITY;
  fstat_plan_desc cand_best = *desc;
  fstat_status last = FSTAT_OK;
  std::string last_msg;
  for (int si = 0; si < 2; ++si) {
    if (si == 1 && splits[1] == splits[0]) break;
    const int lr = splits[si], lc = log_n - lr;
    if (lr < 6 || lr > 12 || lc < 6 || lc > 12) continue;
    for (int ch = 0; ch < 2; ++ch)
      for (int rh = 0; rh < 2; ++rh)
        for (int radix = 16; radix <= 32; radix *= 2) {
          fstat_plan_desc d = *desc;
          d.tune_col_log_len = lr;
          d.tune_col_lines = ch ? cols_lines_max(lr) / 2 : cols_lines_max(lr);
          d.tune_row_lines = rh ? rows_lines_max(lc) / 2 : rows_lines_max(lc);
          d.tune_fft_radix = radix;
          if (d.tune_col_lines < 1 || d.tune_row_lines < 1) continue;
          fstat_plan* p = nullptr;
          if (fstat_plan_create(&d, &p) != FSTAT_OK) continue;
          float ms = INFINITY;
          // one untimed run, then one timed with events on the stream
          fstat_status r = run(p, in, templates, ntmpl, twoF, nullptr, nullptr, workspace,
                               ws_bytes, stream, int64_t(1) << 40);
          if (r == FSTAT_OK) r = check_hip(hipEventRecord(e0, st), "event record");
          if (r == FSTAT_OK)
            r = run(p, in, templates, ntmpl, twoF, nullptr, nullptr, workspace, ws_bytes,
                    stream, int64_t(1) << 40);
          if (r == FSTAT_OK) r = check_hip(hipEventRecord(e1, st), "event record");
          if (r == FSTAT_OK) r = check_hip(hipEventSynchronize(e1), "event synchronise");
          if (r == FSTAT_OK) r = check_hip(hipEventElapsedTime(&ms, e0, e1), "event time");
          fstat_plan_destroy(p);
          if (r != FSTAT_OK) {
            last = r;
            last_msg = g_err;
            if (r == FSTAT_EHIP) break;
            continue;
          }
          if (ms < best_t) {
            best_t = ms;
            cand_best = d;
          }
        }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!(best_t < INFINITY)) {
    return fail(last != FSTAT_OK ? last : FSTAT_EINVAL, "autotune: no launch shape ran (%s)",
                last_msg.c_str());
  }
  *best = cand_best;
  *best_ms = best_t;
  return ok();
}

}  // extern "C"

namespace {

// Autotune cache: one JSON object per line,
//   {"key": "<key>", "tune": [col_log_len, col_lines, row_lines, radix], "ms": <median>}
// with the key built from the set-up fields that decide the shapes' speed.
std::string tune_key(const fstat_plan_desc* d, int32_t slots) {
  char buf[256];
  const int n = std::snprintf(buf, sizeof buf, "n_fft=%lld ndet=%d D=%d flags=%u slots=%d",
                              static_cast<long long>(d->n_fft), d->ndet, d->sinc_halfwidth,
                              static_cast<unsigned>(d->flags), slots);
  std::string k(buf, size_t(n));
  for (int X = 0; X < d->ndet; ++X)
    k += " n" + std::to_string(X) + "=" + std::to_string(static_cast<long long>(d->det[X].n));
  return k;
}

// The last cache line with this key (false: none, or the file is absent).
bool tune_cache_find(const char* path, const std::string& key, int32_t v[4], float* ms) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  const std::string kq = "\"key\": \"" + key + "\"";
  char line[4096];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    if (!std::strstr(line, kq.c_str())) continue;
    const char* t = std::strstr(line, "\"tune\": [");
    const char* m = std::strstr(line, "\"ms\": ");
    int32_t a[4];
    float x = 0.f;
    if (t && m && std::sscanf(t + 9, "%d , %d , %d , %d", &a[0], &a[1], &a[2], &a[3]) == 4 &&
        std::sscanf(m + 6, "%f", &x) == 1) {
      for (int i = 0; i < 4; ++i) v[i] = a[i];
      *ms = x;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void tune_cache_add(const char* path, const std::string& key, const fstat_plan_desc& d,
                    float ms) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"tune\": [%d, %d, %d, %d], \"ms\": %.6g}\n",
               key.c_str(), d.tune_col_log_len, d.tune_col_lines, d.tune_row_lines,
               d.tune_fft_radix, double(ms));
  std::fclose(f);
}

// Median device time of `repeats` searches (after one untimed) with the
// shape d; INFINITY with *err set when the shape does not run.
float time_search_shape(const fstat_plan_desc& d, const fstat_inputs* in,
                        const double* templates_host, const double* templates, int64_t ntmpl,
                        int32_t slots, int32_t repeats, float* twoF, hipStream_t st,
                        fstat_status* err) {
  *err = FSTAT_OK;
  fstat_plan* p = nullptr;
  if ((*err = fstat_plan_create(&d, &p)) != FSTAT_OK) return INFINITY;
  fstat_search* sr = nullptr;
  void* ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<float> t;
  fstat_status r = fstat_search_create(p, templates_host, ntmpl, slots, 0u, &sr);
  size_t wsb = 0;
  if (r == FSTAT_OK) r = fstat_search_info(sr, &wsb, nullptr, nullptr);
  if (r == FSTAT_OK) r = check_hip(hipMalloc(&ws, wsb), "autotune workspace");
  if (r == FSTAT_OK) r = check_hip(hipEventCreate(&e0), "event");
  if (r == FSTAT_OK) r = check_hip(hipEventCreate(&e1), "event");
  if (r == FSTAT_OK) r = fstat_search_run(sr, in, templates, twoF, nullptr, ws, wsb, st);
  for (int i = 0; r == FSTAT_OK && i < repeats; ++i) {
    float ms = 0.f;
    r = check_hip(hipEventRecord(e0, st), "event record");
    if (r == FSTAT_OK) r = fstat_search_run(sr, in, templates, twoF, nullptr, ws, wsb, st);
    if (r == FSTAT_OK) r = check_hip(hipEventRecord(e1, st), "event record");
    if (r == FSTAT_OK) r = check_hip(hipEventSynchronize(e1), "event synchronise");
    if (r == FSTAT_OK) r = check_hip(hipEventElapsedTime(&ms, e0, e1), "event time");
    if (r == FSTAT_OK) t.push_back(ms);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (ws) (void)hipFree(ws);
  fstat_search_destroy(sr);
  fstat_plan_destroy(p);
  *err = r;
  if (r != FSTAT_OK || t.empty()) return INFINITY;
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

}  // namespace

extern "C" {

fstat_status fstat_autotune_search(const fstat_plan_desc* desc, const fstat_inputs* in,
                                   const double* templates_host, const double* templates,
                                   int64_t ntmpl, int32_t slots, int32_t repeats, float* twoF,
                                   const char* cache_path, void* stream, fstat_plan_desc* best,
                                   float* best_ms, int32_t* from_cache) {
  if (!best || !best_ms) return fail(FSTAT_EINVAL, "best or best_ms is NULL");
  fstat_status s = validate_desc(desc);
  if (s != FSTAT_OK) return s;
  if (ntmpl < 1 || !templates_host || !templates || !twoF)
    return fail(FSTAT_EINVAL, "need ntmpl >= 1 sample templates (host and device) and twoF");
  if (slots < 1 || slots > kMaxSlots)
    return fail(FSTAT_EINVAL, "slots=%d outside [1, %d]", slots, kMaxSlots);
  if (repeats < 3) return fail(FSTAT_EINVAL, "repeats=%d: at least 3 timed runs", repeats);
  if (from_cache) *from_cache = 0;
  const char* cache = cache_path ? cache_path : std::getenv("FSTAT_AUTOTUNE_CACHE");
  if (cache && !*cache) cache = nullptr;
  const std::string key = tune_key(desc, slots);
  if (cache) {
    int32_t v[4];
    float ms = 0.f;
    if (tune_cache_find(cache, key, v, &ms)) {
      fstat_plan_desc d = *desc;
      d.tune_col_log_len = v[0];
      d.tune_col_lines = v[1];
      d.tune_row_lines = v[2];
      d.tune_fft_radix = v[3];
      fstat_plan* p = nullptr;
      if (fstat_plan_create(&d, &p) == FSTAT_OK) {
        fstat_plan_destroy(p);
        *best = d;
        *best_ms = ms;
        if (from_cache) *from_cache = 1;
        return ok();
      }
    }
  }
  if (!in) return fail(FSTAT_EINVAL, "inputs is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int log_n = ilog2(desc->n_fft);
  const int splits[2] = {log_n / 2, (log_n + 1) / 2};
  float best_t = INFINITY;
  fstat_plan_desc cand_best = *desc;
  fstat_status last = FSTAT_OK;
  std::string last_msg;
  for (int si = 0; si < 2; ++si) {
    if (si == 1 && splits[1] == splits[0]) break;
    const int lr = splits[si], lc = log_n - lr;
    if (lr < 6 || lr > 12 || lc < 6 || lc > 12) continue;
    for (int ch = 0; ch < 2; ++ch)
      for (int rh = 0; rh < 2; ++rh)
        for (int radix = 16; radix <= 32; radix *= 2) {
          fstat_plan_desc d = *desc;
          d.tune_col_log_len = lr;
          d.tune_col_lines = ch ? cols_lines_max(lr) / 2 : cols_lines_max(lr);
          d.tune_row_lines = rh ? rows_lines_max(lc) / 2 : rows_lines_max(lc);
          d.tune_fft_radix = radix;
          if (d.tune_col_lines < 1 || d.tune_row_lines < 1) continue;
          fstat_status r;
          const float ms = time_search_shape(d, in, templates_host, templates, ntmpl, slots,
                                             repeats, twoF, st, &r);
          if (r != FSTAT_OK) {
            last = r;
            last_msg = g_err;
            if (r == FSTAT_EHIP) break;
            continue;
          }
          if (ms < best_t) {
            best_t = ms;
            cand_best = d;
          }
        }
  }
  if (!(best_t < INFINITY))
    return fail(last != FSTAT_OK ? last : FSTAT_EINVAL, "autotune: no launch shape ran (%s)",
                last_msg.c_str());
  *best = cand_best;
  *best_ms = best_t;
  if (cache) tune_cache_add(cache, key, cand_best, best_t);
  return ok();
}

fstat_status fstat_resample(const fstat_plan* plan, const fstat_inputs* in,
                            const double* templates, int64_t ntmpl, void* y, void* workspace,
                            size_t ws_bytes, void* stream) {
  if (ntmpl > 0 && !y) return fail(FSTAT_EINVAL, "y is NULL");
  return run(plan, in, templates, ntmpl, nullptr, nullptr, y, workspace, ws_bytes, stream, 1);
}

fstat_status fstat_grad_workspace_size(const fstat_plan* plan, int64_t batch, size_t* bytes) {
  if (!plan || !bytes) return fail(FSTAT_EINVAL, "plan or bytes is NULL");
  if (batch < 1) return fail(FSTAT_EINVAL, "batch must be >= 1");
  *bytes = kHeaderBytes + size_t(batch) * grad_slot_bytes(plan);
  return ok();
}

fstat_status fstat_compute_2f_grad(const fstat_plan* plan, const fstat_inputs* in,
                                   const double* templates, int64_t ntmpl,
                                   const float* grad_twoF, double* grad, float* twoF,
                                   void* workspace, size_t ws_bytes, void* stream) {
  if (!plan) return fail(FSTAT_EINVAL, "plan is NULL");
  if (ntmpl < 0) return fail(FSTAT_EINVAL, "ntmpl < 0");
  if (ntmpl > 0 && (!templates || !grad_twoF || !grad))
    return fail(FSTAT_EINVAL, "templates, grad_twoF or grad is NULL");
  fstat_status s = validate_inputs(plan, in, true);
  if (s != FSTAT_OK) return s;
  if (!workspace) return fail(FSTAT_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(FSTAT_EINVAL, "workspace must be 256-byte aligned");
  const size_t sb = grad_slot_bytes(plan);
  if (ws_bytes < kHeaderBytes + sb)
    return fail(FSTAT_EWORKSPACE, "workspace %zu bytes < %zu needed for one template", ws_bytes,
                kHeaderBytes + sb);
  if (ntmpl == 0) return ok();
  const int64_t slots = std::min<int64_t>(int64_t((ws_bytes - kHeaderBytes) / sb), kMaxSlots);
  if ((s = set_lds_limits(plan)) != FSTAT_OK) return s;
  PlanConst P = make_const(plan, in);
  P.slot_stride = int64_t(sb);
  P.part_offset = int64_t(kParamBytes + size_t(4) * plan->desc.n_fft * sizeof(float2));
  P.knot_offset = P.part_offset + int64_t(grad_part_bytes(plan));
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_twiddles, dim3(kTwLen / 256), dim3(256), 0, st, workspace);
  for (int64_t t = 0; t < ntmpl; t += slots) {
    ChunkMap map;
    std::memset(&map, 0, sizeof map);
    map.n_tmpl = int(std::min<int64_t>(slots, ntmpl - t));
    for (int i = 0; i < map.n_tmpl; ++i) map.tmpl[i] = t + i;
    s = launch_grad_chunk(plan, P, templates, map, int(slots), grad_twoF, grad, twoF, workspace,
                          st);
    if (s != FSTAT_OK) return s;
  }
  return ok();
}

fstat_status fstat_grad_bin_workspace_size(const fstat_plan* plan, int64_t batch,
                                           size_t* bytes) {
  if (!plan || !bytes) return fail(FSTAT_EINVAL, "plan or bytes is NULL");
  if (batch < 1) return fail(FSTAT_EINVAL, "batch must be >= 1");
  *bytes = kHeaderBytes + size_t(batch) * grad_bin_slot_bytes(plan);
  return ok();
}

fstat_status fstat_compute_2f_grad_bin(const fstat_plan* plan, const fstat_inputs* in,
                                       const double* templates, int64_t ntmpl,
                                       const int64_t* bins, float* twoF, double* grad,
                                       void* workspace, size_t ws_bytes, void* stream) {
  if (!plan) return fail(FSTAT_EINVAL, "plan is NULL");
  if (ntmpl < 0) return fail(FSTAT_EINVAL, "ntmpl < 0");
  if (ntmpl > 0 && (!templates || !bins || !grad))
    return fail(FSTAT_EINVAL, "templates, bins or grad is NULL");
  fstat_status s = validate_inputs(plan, in, true);
  if (s != FSTAT_OK) return s;
  if (!workspace) return fail(FSTAT_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(FSTAT_EINVAL, "workspace must be 256-byte aligned");
  const size_t sb = grad_bin_slot_bytes(plan);
  if (ws_bytes < kHeaderBytes + sb)
    return fail(FSTAT_EWORKSPACE, "workspace %zu bytes < %zu needed for one template", ws_bytes,
                kHeaderBytes + sb);
  if (ntmpl == 0) return ok();
  const int64_t slots = std::min<int64_t>(int64_t((ws_bytes - kHeaderBytes) / sb), kMaxSlots);
  PlanConst P = make_const(plan, in);
  P.slot_stride = int64_t(sb);
  P.part_offset = int64_t(kParamBytes);
  P.knot_offset = 0;  // the single-bin tiles solve their own knots
  hipStream_t st = static_cast<hipStream_t>(stream);
  // (clears the flagged-template counter)
  hipLaunchKernelGGL(k_twiddles, dim3(kTwLen / 256), dim3(256), 0, st, workspace);
  for (int64_t t = 0; t < ntmpl; t += slots) {
    ChunkMap map;
    std::memset(&map, 0, sizeof map);
    map.n_tmpl = int(std::min<int64_t>(slots, ntmpl - t));
    for (int i = 0; i < map.n_tmpl; ++i) map.tmpl[i] = t + i;
    s = launch_grad_bin_chunk(plan, P, templates, map, int(slots), bins, twoF, grad, workspace,
                              st);
    if (s != FSTAT_OK) return s;
  }
  return ok();
}

fstat_status fstat_sinc_halfwidth_for(double band_fraction, double tol_2f, int32_t* D,
                                      double* err_2f) {
  if (!D) return fail(FSTAT_EINVAL, "D is NULL");
  if (!(band_fraction > 0.0 && band_fraction <= 1.0) || !(tol_2f > 0.0))
    return fail(FSTAT_EINVAL, "need 0 < band_fraction <= 1 and tol_2f > 0");
  // |zhat / z|^2 for a tone of nu cycles per sample interpolated at fractional
  // offset u with the 2D-tap Hann-windowed sinc (taps j = -D+1 .. D)
  auto power = [](int hw, double nu, double u) {
    double re = 0.0, im = 0.0;
    for (int j = -hw + 1; j <= hw; ++j) {
      const double s = u - j;
      const double h = s == 0.0 ? 1.0
                                : std::sin(M_PI * s) / (M_PI * s) * 0.5 *
                                      (1.0 + std::cos(M_PI * s / hw));
      const double ph = 2.0 * M_PI * nu * (j - u);
      re += h * std::cos(ph);
      im += h * std::sin(ph);
    }
    return re * re + im * im;
  };
  constexpr int kNu = 65, kU = 32, kRef = 32;
  const int choices[6] = {4, 6, 8, 10, 12, 16};
  double err = 0.0;
  for (int D_try : choices) {
    err = 0.0;
    for (int a = 0; a < kNu; ++a) {
      const double nu = 0.5 * band_fraction * a / (kNu - 1);
      for (int b = 0; b < kU; ++b) {
        const double u = double(b) / kU;
        err = std::max(err, std::fabs(power(D_try, nu, u) / power(kRef, nu, u) - 1.0));
      }
    }
    *D = D_try;
    if (err <= tol_2f) break;
  }
  if (err_2f) *err_2f = err;
  if (err > tol_2f)
    return fail(FSTAT_EUNSUPPORTED,
                "no half-width up to 16 keeps the 2F error below %.3g over %.3g of the band "
                "(16 gives %.3g)",
                tol_2f, band_fraction, err);
  return ok();
}

fstat_status fstat_sfts_to_series(const fstat_sft_desc* desc, const void* sfts,
                                  const uint8_t* present, void* x, uint8_t* valid,
                                  void* stream) {
  if (!desc || !sfts || !x) return fail(FSTAT_EINVAL, "desc, sfts or x is NULL");
  if (!finite_pos(desc->t_sft) || !std::isfinite(desc->t_start))
    return fail(FSTAT_EINVAL, "t_sft must be positive and finite, t_start finite");
  if (desc->n_sft < 1 || desc->k0 < 0 || desc->reserved != 0)
    return fail(FSTAT_EINVAL, "need n_sft >= 1, k0 >= 0, reserved = 0");
  const int K = desc->n_bins;
  if (K < 2 || K > kSftMaxBins || (K & 1))
    return fail(FSTAT_EUNSUPPORTED, "n_bins=%d: need an even count in [2, %d]", K, kSftMaxBins);
  SftPlan sp;
  std::memset(&sp, 0, sizeof sp);
  sp.K = K;
  int rest = K;
  for (int r : {4, 2, 3, 5}) {
    while (rest % r == 0 && sp.nstages < kSftMaxStages) {
      sp.radix[sp.nstages++] = r;
      rest /= r;
    }
  }
  if (rest != 1)
    return fail(FSTAT_EUNSUPPORTED, "n_bins=%d has a prime factor above 5", K);
  // f_h t_start in cycles, reduced exactly: f_h t_start = kc t_start / t_sft
  const double kc = double(desc->k0) + 0.5 * K;
  const double turns = desc->t_start / desc->t_sft;
  const double cyc = std::fmod(kc * (turns - std::floor(turns)), 1.0);
  sp.het = make_float2(float(std::cos(2.0 * M_PI * cyc)), float(-std::sin(2.0 * M_PI * cyc)));
  sp.scale = float(1.0 / desc->t_sft);
  const size_t lds = size_t(3) * K * sizeof(float2);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sft_series),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  fstat_status s = check_hip(e, "hipFuncSetAttribute(sft)");
  if (s != FSTAT_OK) return s;
  hipLaunchKernelGGL(k_sft_series, dim3(unsigned(desc->n_sft)), dim3(kSftThreads), lds,
                     static_cast<hipStream_t>(stream), sp, static_cast<const float2*>(sfts),
                     present, static_cast<float2*>(x), valid);
  s = check_hip(hipGetLastError(), "sft launch");
  return s == FSTAT_OK ? ok() : s;
}

fstat_status fstat_flagged_count(const void* workspace, size_t ws_bytes, void* stream,
                                 int64_t* count) {
  if (!workspace || !count) return fail(FSTAT_EINVAL, "workspace or count is NULL");
  if (ws_bytes < kHeaderBytes)
    return fail(FSTAT_EWORKSPACE, "workspace %zu bytes < %zu", ws_bytes, kHeaderBytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned long long v = 0;
  fstat_status s = check_hip(
      hipMemcpyAsync(&v, flag_counter(const_cast<void*>(workspace)), sizeof v,
                     hipMemcpyDeviceToHost, st),
      "flagged count copy");
  if (s == FSTAT_OK) s = check_hip(hipStreamSynchronize(st), "flagged count synchronise");
  if (s != FSTAT_OK) return s;
  *count = int64_t(v);
  return ok();
}

}  // extern "C"

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // device address of `scratch`, per device

// The current device's copy of the static scratch, looked up once per device.
fstat_status static_scratch(void** out) {
  int dev = 0;
  fstat_status s = check_hip(hipGetDevice(&dev), "get device");
  if (s != FSTAT_OK) return s;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr.size() <= size_t(dev)) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    s = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch symbol address");
    if (s != FSTAT_OK) return s;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FSTAT_OK;
}

}  // namespace

extern "C" {

fstat_status fstat_compute_2f_grad_bin_noalloc(const fstat_plan* plan, const fstat_inputs* in,
                                               const double* templates, int64_t ntmpl,
                                               const int64_t* bins, float* twoF, double* grad,
                                               void* stream) {
  if (!plan) return fail(FSTAT_EINVAL, "plan is NULL");
  size_t need = 0;
  fstat_status s = fstat_grad_bin_workspace_size(plan, 1, &need);
  if (s != FSTAT_OK) return s;
  if (need > kStaticScratchBytes)
    return fail(FSTAT_EWORKSPACE,
                "this plan needs %zu bytes of scratch for one template; the static scratch "
                "holds %zu",
                need, kStaticScratchBytes);
  void* ws = nullptr;
  if ((s = static_scratch(&ws)) != FSTAT_OK) return s;
  return fstat_compute_2f_grad_bin(plan, in, templates, ntmpl, bins, twoF, grad, ws,
                                   kStaticScratchBytes, stream);
}

fstat_status fstat_sync_check(void* stream) {
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(FSTAT_EHIP, "asynchronous HIP error: %s", hipGetErrorString(e));
  return ok();
}

}  // extern "C"
