/*
 * fstat.h - C ABI of the MI355X (gfx950) resampling F-statistic library.
 *
 * The library computes the F-statistic of arXiv:2201.00451 (Sec. 2, eq. Fstat)
 * by the resampling algorithm of Sec. 3, steps (iii)-(vii), for many templates
 * over the full frequency band of a heterodyned, downsampled complex series.
 *
 * Units: times in seconds on one time base, angles in radians, frequencies in
 * Hz, distances in light-seconds.  All device pointers are HIP device memory
 * owned by the caller; the library allocates no device memory, frees nothing
 * it did not allocate, and never synchronises the stream except where stated.
 * Every call is asynchronous on the stream given (a hipStream_t passed as
 * void*, NULL = the null stream).  Every function returns an fstat_status;
 * on failure no kernel has been launched and fstat_last_error() returns a
 * thread-local message.  Nothing is thrown across this boundary.
 */
#ifndef FSTAT_H
#define FSTAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define FSTAT_API __attribute__((visibility("default")))
#else
#define FSTAT_API
#endif

#define FSTAT_MAX_DET 4
#define FSTAT_TEMPLATE_STRIDE 8
/* Plan flag: Keplerian (eccentric) source orbits.  Template rows then hold
 * FSTAT_TEMPLATE_STRIDE_KEPLER doubles: the eight of a circular row and the
 * eccentricity (0 <= ecc < 1) and argument of periapsis argp (rad), with tp
 * the time of periapsis.  The orbit's Roemer delay is
 *   R(t') = asini [sin(argp) (cos E - ecc) + cos(argp) sqrt(1 - ecc^2) sin E],
 * E - ecc sin E = 2 pi (t' - tp) / porb (Kepler's equation); with ecc = 0 and
 * argp = 0 it is the circular asini sin(2 pi (t' - tp) / porb).  (The paper's
 * binary searches vary the orbital elements, Sec. 4.2 the period among them;
 * its own searches assume circular orbits.) */
#define FSTAT_PLAN_KEPLER 1u
#define FSTAT_TEMPLATE_STRIDE_KEPLER 10

typedef enum {
  FSTAT_OK = 0,
  FSTAT_EINVAL = -1,       /* an argument is invalid (null, out of range, inconsistent) */
  FSTAT_EUNSUPPORTED = -2, /* valid, but outside what this library implements */
  FSTAT_EWORKSPACE = -3,   /* workspace smaller than fstat_workspace_size() */
  FSTAT_EHIP = -4,         /* the HIP runtime reported an error */
  FSTAT_EINTERNAL = -5     /* an inconsistency inside the library (no kernel for a shape
                              the plan accepted); nothing was launched */
} fstat_status;

/* One detector: its site (for a(t), b(t) of Sec. 2 and the Roemer delay t_m)
 * and its input series x_h(t^k) of step (ii), sampled at t0 + j*dt. */
typedef struct {
  double lat;       /* geocentric latitude */
  double lon;       /* east longitude */
  double az_x;      /* azimuth of the x arm, counter-clockwise from local East */
  double az_y;      /* azimuth of the y arm; arms are orthogonal */
  double t0;        /* time of sample 0 */
  int64_t n;        /* number of samples, >= 1 */
  double noise_var; /* E|n|^2 of the complex noise; the weight is 1/noise_var (Sec. 2, S_h) */
} fstat_detector;

/* Search set-up shared by every template (host memory, copied at plan creation). */
typedef struct {
  int32_t ndet;                        /* 1..FSTAT_MAX_DET */
  int32_t sinc_halfwidth;              /* D: the step (v) interpolation uses 2D taps;
                                          one of 4, 6, 8, 10, 12, 16 */
  fstat_detector det[FSTAT_MAX_DET];
  double dt;                           /* sample step of the inputs and of the source-frame grid (step iv) */
  double f_het;                        /* heterodyne frequency f_h of step (ii) */
  double t_ref;                        /* reference time of the spin-down Taylor series Phi_s */
  double tau0;                         /* source-frame grid origin: tau_k = tau0 + k*dt (step iv) */
  double max_delay;                    /* bound on |t_src - t| over every template and sample */
  double sid_angle0;                   /* sidereal angle of the prime meridian at t = 0 */
  double sid_rate;                     /* sidereal rotation rate (rad/s) */
  int64_t n_fft;                       /* FFT length (step vi, zero-padded): power of two, 2^12..2^24 */
  int64_t bin_lo;                      /* first output bin of the ascending band, 0 <= bin_lo */
  int64_t n_bins;                      /* output bins; bin_lo + n_bins <= n_fft.  Bin i is at
                                          f_het + df + (i - n_fft/2)/(n_fft*dt) (Sec. 3: one pass
                                          gives the band centred on f_h) */
  /* Launch-shape tuning of the step (vi) FFT (0 = automatic).  They change
   * only how the work is laid out, never the result beyond FP32 rounding:
   *   tune_col_log_len: log2 of the column-pass FFT length, the row pass has
   *     log2(n_fft) - tune_col_log_len; both must lie in [6, 12];
   *   tune_col_lines: columns per workgroup of the column pass: the largest
   *     count that fits 128 KiB of LDS (512 threads, one workgroup per compute
   *     unit) or half of it (256 threads, two per unit: the automatic choice);
   *   tune_row_lines: rows per workgroup of the row pass (the a and b rows
   *     together): the largest count (512 threads: the automatic choice) or
   *     half of it (256 threads);
   *   tune_fft_radix: largest radix of a Stockham stage, 16 or 32 (automatic:
   *     32, so lines of 2^9 and 2^10 points take two stages). */
  int32_t tune_col_log_len;
  int32_t tune_col_lines;
  int32_t tune_row_lines;
  int32_t tune_fft_radix;
  uint32_t flags;                      /* 0 or FSTAT_PLAN_KEPLER */
} fstat_plan_desc;

/* A candidate of the search (device memory, written by
 * fstat_search_run_candidates): template index, bin in the band, 2F. */
typedef struct {
  int32_t tmpl;
  int32_t bin;
  float twoF;
  int32_t reserved;
} fstat_candidate;

/* Device-resident data, crossed to the device once (Sec. 3: the host-to-device
 * copy happens only between steps (ii) and (iii)). */
typedef struct {
  const void* x[FSTAT_MAX_DET];        /* float2 [det.n]: heterodyned series, zero in gaps */
  const uint8_t* valid[FSTAT_MAX_DET]; /* uint8 [det.n]: 1 = science sample; NULL = all valid */
  const double* ephem[FSTAT_MAX_DET];  /* double [n_eph][6]: detector position (light-s) and
                                          velocity (light-s/s) in the equatorial barycentric frame
                                          at eph_t0 + i*eph_dt, interpolated cubically */
  int64_t n_eph;
  double eph_t0;
  double eph_dt;
  const double* moments;               /* double [ndet][10] from fstat_antenna_moments(); read
                                          by fstat_compute_2f* for A, B, C of eq. Fstat */
} fstat_inputs;

typedef struct fstat_plan fstat_plan;  /* opaque, host memory owned by the library */

/* Short Fourier transforms of one detector's strain (the input of Sec. 3,
 * steps (i)-(ii)): n_sft contiguous slots of length t_sft starting at
 * t_start (slot s covers [t_start + s t_sft, t_start + (s+1) t_sft)); each
 * holds n_bins bins k0 .. k0 + n_bins - 1 (frequency k / t_sft) of its
 * segment's DFT normalised by the raw time step,
 *   X_s[k] = dt_raw sum_n r(t_s + n dt_raw) exp(-2 pi i k n / N_s). */
typedef struct {
  double t_start;
  double t_sft;
  int64_t n_sft;
  int64_t k0;
  int32_t n_bins;   /* K: even, 2..4096, prime factors 2, 3 and 5 only */
  int32_t reserved; /* must be 0 */
} fstat_sft_desc;

/* Steps (i)-(ii) of Sec. 3: the SFTs combined into one transform, low-passed
 * to their band, heterodyned at the band's centre f_h = (k0 + K/2) / t_sft
 * and transformed back, which gives the complex series x_h at
 * t_start + n dt, dt = t_sft / K, n < n_sft K:
 *   x_h(t_s + j dt) = (1/t_sft) sum_q X_s[k0 + q] exp(2 pi i (k0 + q) j / K)
 *                     exp(-2 pi i f_h (t_s + j dt)),
 * one K-point inverse DFT per SFT (the band of each SFT carries its segment
 * only; nothing of the raw series outside the band is needed).
 *   sfts:    device float2 [n_sft][K];
 *   present: device uint8 [n_sft], nullable (= all present); a missing SFT
 *            gives K zeros;
 *   x:       device float2 [n_sft K] (output, fstat_inputs.x of a plan with
 *            dt, f_het as above and detector t0 = t_start, n = n_sft K);
 *   valid:   device uint8 [n_sft K] (output, nullable): 1 where an SFT was present.
 * Fails with FSTAT_EINVAL for a null pointer, t_sft not positive and finite,
 * n_sft < 1, k0 < 0 or a non-zero reserved field, and FSTAT_EUNSUPPORTED for
 * K outside 2..4096, odd, or with a prime factor above 5. */
FSTAT_API fstat_status fstat_sfts_to_series(const fstat_sft_desc* desc, const void* sfts,
                                            const uint8_t* present, void* x, uint8_t* valid,
                                            void* stream);

/* Validate a set-up and build a plan.  Fails with FSTAT_EINVAL when: ndet out of
 * range; dt, noise_var or sid_rate not positive and finite; n_fft not a power of
 * two in [2^12, 2^24]; the band [bin_lo, bin_lo+n_bins) not inside [0, n_fft) or
 * empty; D not one of 4, 6, 8, 10, 12, 16; the source-frame grid [tau0, tau0 + n_fft*dt) does not
 * cover every sample's source time widened by max_delay; flags other than
 * FSTAT_PLAN_KEPLER.  Template rows of a plan are FSTAT_TEMPLATE_STRIDE
 * doubles, or FSTAT_TEMPLATE_STRIDE_KEPLER with FSTAT_PLAN_KEPLER (every
 * `templates` argument below and fstat_search_create's host rows). */
FSTAT_API fstat_status fstat_plan_create(const fstat_plan_desc* desc, fstat_plan** out);
FSTAT_API void fstat_plan_destroy(fstat_plan* plan);

/* What the plan derived from the set-up: k_pad, the number of source-frame
 * grid points that can be non-zero (data span plus delay bound plus the
 * interpolation half-width, rounded up to the resampling tile and to the FFT
 * row length) and the four-step FFT split n_fft = 2^log_col_len *
 * 2^log_row_len (column transforms of length 2^log_col_len first).  Any
 * output pointer may be NULL. */
FSTAT_API fstat_status fstat_plan_info(const fstat_plan* plan, int64_t* k_pad,
                                       int32_t* log_col_len, int32_t* log_row_len);

/* Bytes of device workspace for `batch` templates in flight (batch >= 1).
 * The plain path needs batch = 1; larger workspaces let the batched path keep
 * more templates in flight. */
FSTAT_API fstat_status fstat_workspace_size(const fstat_plan* plan, int64_t batch, size_t* bytes);

/* A, B, C of eq. Fstat (Sec. 2) are noise-weighted sums over the valid samples
 * of products of a(t), b(t).  With a, b trigonometric polynomials of degree 2 in
 * the local sidereal angle phi_X(t), every such sum follows from the five
 * per-detector moments M_n = sum_j valid_j exp(i n phi_X(t_j)), n = 0..4.  This
 * call computes them once per data set: moments[X][2n], moments[X][2n+1] =
 * Re, Im M_n.  Uses the workspace; deterministic (fixed reduction order). */
FSTAT_API fstat_status fstat_antenna_moments(const fstat_plan* plan, const fstat_inputs* in,
                                   double* moments, void* workspace, size_t ws_bytes,
                                   void* stream);

/* Plain path (Sec. 3, steps (iii)-(vii), one template after another): for each
 * template row p[8] = (alpha, delta, df, f1dot, f2dot, asini, porb, tp) of the
 * device array `templates` [ntmpl][8]:
 *   (iii) correct each input sample by exp(-2 pi i f_h (t_src - t)),
 *   (iv)  find the detector epochs T_k of the regular source-frame grid tau_k
 *         through the Roemer delay and the circular binary delay
 *         asini*sin(2 pi (t_src - tp)/porb) (asini = 0: isolated source),
 *   (v)   interpolate with a Hann-windowed sinc of half-width D,
 *   (vi)  weight by a(T_k), b(T_k) and 1/noise_var, sum detectors, remove the
 *         spin-down phase Phi_s(tau_k) (about t_ref) and the sub-bin offset df,
 *         and Fourier transform (length n_fft),
 *   (vii) form 2F = 2 (B|Fa|^2 + A|Fb|^2 - 2C Re(Fa Fb*)) / (AB - C^2).
 * Output twoF: float [ntmpl][n_bins] on the device, ascending frequency.
 * fafb (nullable): float2 [ntmpl][2][n_bins] receives Fa then Fb.
 * A template whose delays exceed max_delay, or whose parameters are not finite,
 * gets NaN in every bin.  Needs fstat_workspace_size(plan, 1). */
FSTAT_API fstat_status fstat_compute_2f(const fstat_plan* plan, const fstat_inputs* in,
                              const double* templates, int64_t ntmpl, float* twoF, void* fafb,
                              void* workspace, size_t ws_bytes, void* stream);

/* Batched path: the same result as fstat_compute_2f (bit-identical: same
 * kernels, same arithmetic), with as many templates in flight per launch as
 * the workspace holds (Sec. 6 names searching several templates at once as an
 * optimisation the CUDA code did not make). */
FSTAT_API fstat_status fstat_compute_2f_batched(const fstat_plan* plan, const fstat_inputs* in,
                                      const double* templates, int64_t ntmpl, float* twoF,
                                      void* fafb, void* workspace, size_t ws_bytes,
                                      void* stream);

/* fstat_compute_2f_batched with per-kernel timing: HIP events are recorded on
 * `stream` around every launch and, after synchronising the stream, the
 * summed device time of each kernel is returned in kernel_ms[4] (prologue,
 * resample, column FFT pass, row FFT pass with 2F) and the launch counts in
 * launches[4].  max_batch (>= 1) caps the templates in flight per launch
 * (1 = the plain per-template path).  Synchronises the stream. */
FSTAT_API fstat_status fstat_compute_2f_profiled(const fstat_plan* plan, const fstat_inputs* in,
                                       const double* templates, int64_t ntmpl, float* twoF,
                                       void* workspace, size_t ws_bytes, int64_t max_batch,
                                       void* stream, float* kernel_ms, int64_t* launches);

/* Grouped path for a template bank.  Sec. 4.1 measures that searching over
 * spin-down parameters at a fixed sky position can reuse the sky-dependent
 * barycentring; here every maximal run of consecutive templates with the
 * same sky position and orbit (alpha, delta, asini, porb, tp; porb and tp
 * ignored when asini = 0) is resampled once (steps (iii)-(v) and the antenna
 * weighting), and each template applies its own spin-down phase and sub-bin
 * offset as the FFT loads the shared series.  The result equals
 * fstat_compute_2f bit for bit.
 *
 * fstat_search_create plans the bank from a HOST copy of the templates (the
 * same rows the device array will hold at run time, in the same order),
 * with `slots` (1..32) templates in flight per launch sequence; flags may
 * combine FSTAT_SEARCH_GRAPH: the run functions capture their launch sequence
 * in a HIP graph on the first call and replay it while the arguments it was
 * captured with stay the same (needs a non-null stream): every device
 * pointer and scalar of the inputs that the plan's detectors use (x, valid,
 * ephem, n_eph, eph_t0, eph_dt, moments), the templates, outputs, threshold
 * and workspace; any other value captures again; and FSTAT_SEARCH_ACCUMULATE:
 * fstat_search_run adds 2F to twoF instead of storing it, so that runs over
 * several data segments with the same grid (dt, n_fft, f_het, t_ref, band)
 * sum 2F over the segments on the device (the semi-coherent sum the paper's
 * follow-up search uses; NaN stays NaN; the caller clears twoF before the
 * first segment; fstat_search_run_candidates ignores the flag).  The search
 * keeps a pointer to the plan, which
 * must outlive it.  fstat_search_info reports the workspace bytes, the
 * number of groups and of launch sequences.  fstat_search_run_profiled runs
 * without a graph and returns per-kernel device time like
 * fstat_compute_2f_profiled (synchronises the stream). */
#define FSTAT_SEARCH_GRAPH 1u
#define FSTAT_SEARCH_ACCUMULATE 2u
typedef struct fstat_search fstat_search;  /* opaque, host memory owned by the library */
FSTAT_API fstat_status fstat_search_create(const fstat_plan* plan, const double* templates_host,
                                           int64_t ntmpl, int32_t slots, uint32_t flags,
                                           fstat_search** out);
FSTAT_API void fstat_search_destroy(fstat_search* search);
FSTAT_API fstat_status fstat_search_info(const fstat_search* search, size_t* ws_bytes,
                                         int64_t* ngroups, int64_t* nchunks);
FSTAT_API fstat_status fstat_search_run(fstat_search* search, const fstat_inputs* in,
                                        const double* templates, float* twoF, void* fafb,
                                        void* workspace, size_t ws_bytes, void* stream);
/* Candidate retention on the device instead of the full band: every bin
 * whose 2F exceeds `threshold` is appended to cand (device fstat_candidate
 * [capacity]) in no particular order; *count (device int64) receives the
 * number of such bins, which may exceed capacity (then only capacity of them
 * are stored).  best (nullable, device uint64 [ntmpl]) receives per template
 * the largest 2F and its bin packed as (IEEE bits of 2F << 32) | bin (all
 * ones for a flagged template; equal maxima resolve to the highest bin).
 * Both are cleared by the call itself.  No 2F array is written.  Candidates
 * of one run are unique; their order is not. */
FSTAT_API fstat_status fstat_search_run_candidates(fstat_search* search, const fstat_inputs* in,
                                                   const double* templates, float threshold,
                                                   fstat_candidate* cand, int64_t capacity,
                                                   int64_t* count, uint64_t* best,
                                                   void* workspace, size_t ws_bytes,
                                                   void* stream);
FSTAT_API fstat_status fstat_search_run_profiled(fstat_search* search, const fstat_inputs* in,
                                                 const double* templates, float* twoF,
                                                 void* workspace, size_t ws_bytes, void* stream,
                                                 float* kernel_ms, int64_t* launches);

/* Several independent searches run as one unit (searches of uneven span,
 * band, FFT length and detector count, each with its own plan, data,
 * template bank, output and workspace).  fstat_batch_create takes `n` search
 * handles (host array; the searches and their plans must outlive the batch)
 * and spreads them over `lanes` (1..16) concurrent branches, the longest
 * first onto the least loaded branch (work ~ templates x n_fft).
 * fstat_batch_run takes host arrays of length n: inputs, device template
 * arrays, device 2F outputs [ntmpl][n_bins] (added to for searches created
 * with FSTAT_SEARCH_ACCUMULATE), workspaces of at least fstat_search_info's
 * size, and their sizes.  The first call captures every search's launch
 * sequence into one HIP graph (fork on `stream`, one branch per lane, join
 * back on `stream`) and later calls with the same arguments (every pointer
 * and scalar of every search's inputs, as for FSTAT_SEARCH_GRAPH, and the
 * templates, outputs and workspaces) replay it; any other value recaptures.  Each search's FSTAT_SEARCH_GRAPH flag is not used
 * here.  Needs a non-null stream; runs asynchronously on it.  Each output is
 * the one fstat_search_run gives for that search alone, bit for bit.
 * Searches of one batch must not share a workspace or an output. */
#define FSTAT_MAX_BATCH_LANES 16
typedef struct fstat_batch fstat_batch;  /* opaque, host memory owned by the library */
FSTAT_API fstat_status fstat_batch_create(fstat_search* const* searches, int32_t n,
                                          int32_t lanes, fstat_batch** out);
FSTAT_API void fstat_batch_destroy(fstat_batch* batch);
FSTAT_API fstat_status fstat_batch_run(fstat_batch* batch, const fstat_inputs* const* in,
                                       const double* const* templates, float* const* twoF,
                                       void* const* workspace, const size_t* ws_bytes,
                                       void* stream);

/* The interpolation half-width for an accuracy bound (the paper leaves the
 * step (v) kernel open; D sets its accuracy, so it is chosen by accuracy,
 * not time): the smallest D of 4, 6, 8, 10, 12, 16 for which a tone anywhere
 * in the central band_fraction of the band (|nu| <= band_fraction / 2 cycles
 * per sample), interpolated at any fractional offset, has its power (its 2F)
 * within tol_2f of what the same kernel with D = 32 gives (the worst case
 * over a grid of 65 frequencies and 32 offsets, evaluated on the host).  For
 * tol_2f = 1e-3: D = 10 for the central 30 % of the band, 12 for the
 * central half.  *err_2f (nullable) receives the worst error of the D
 * returned.  FSTAT_EUNSUPPORTED (with *D = 16) when even D = 16 misses the
 * bound. */
FSTAT_API fstat_status fstat_sinc_halfwidth_for(double band_fraction, double tol_2f, int32_t* D,
                                                double* err_2f);

/* Launch-shape autotuner: for the set-up *desc (its tune fields ignored),
 * times every FFT launch shape the plan accepts (both column/row splits of
 * n_fft around its square root, full or half line counts for each pass,
 * radix-16 or radix-32 stage plans) by running the batched path
 * on the given sample of templates (device [ntmpl][8], ntmpl >= 1; twoF a
 * device [ntmpl][n_bins] scratch output) with the given workspace, once
 * untimed and once timed with HIP events, and returns the fastest
 * description in *best (desc with the tune fields set) and its time in
 * *best_ms.  The interpolation half-width is not tuned (it sets the
 * accuracy).  Synchronises the stream.  Fails if no shape ran. */
FSTAT_API fstat_status fstat_autotune(const fstat_plan_desc* desc, const fstat_inputs* in,
                                      const double* templates, int64_t ntmpl, float* twoF,
                                      void* workspace, size_t ws_bytes, void* stream,
                                      fstat_plan_desc* best, float* best_ms);

/* The launch-shape autotuner on the search path (fstat_search_*, the path of
 * large banks): every FFT launch shape fstat_autotune tries runs a search of
 * the sample templates (templates_host: host copy of the rows, templates:
 * device copy, ntmpl >= 1, both of the plan's row width) with `slots`
 * template slots, once untimed and then `repeats` (>= 3) times timed with
 * HIP events on `stream`; the shape with the smallest median time is
 * returned in *best (desc with the tune fields set) and that median in
 * *best_ms.  in->moments must hold the data set's antenna moments.  twoF: a
 * device [ntmpl][n_bins] scratch output.  Each shape's workspace is
 * allocated and freed inside the call (hipMalloc), so this is a set-up call,
 * not one for a loop.  Synchronises the stream.
 * Cache: cache_path, or if it is NULL the environment variable
 * FSTAT_AUTOTUNE_CACHE (unset or empty: no cache), names a text file of one
 * JSON object per line,
 *   {"key": "n_fft=N ndet=K D=D flags=F slots=S n0=.. n1=..", "tune": [col_log_len,
 *    col_lines, row_lines, radix], "ms": median}
 * (n0.. the samples of each detector).  When a line with this set-up's key
 * holds a shape the plan accepts, that shape is returned without running
 * anything (*from_cache = 1; no input is read); otherwise the tuned result
 * is appended (*from_cache = 0).  from_cache may be NULL.  Fails if no shape
 * ran (with the last failure's status). */
FSTAT_API fstat_status fstat_autotune_search(const fstat_plan_desc* desc, const fstat_inputs* in,
                                             const double* templates_host,
                                             const double* templates, int64_t ntmpl,
                                             int32_t slots, int32_t repeats, float* twoF,
                                             const char* cache_path, void* stream,
                                             fstat_plan_desc* best, float* best_ms,
                                             int32_t* from_cache);

/* Diagnostic: steps (iii)-(v) and the weighting of (vi) only.  Writes the
 * weighted, resampled series before the transform, y: float2 [ntmpl][2][n_fft]
 * (y_a then y_b, zero beyond the data).  Needs fstat_workspace_size(plan, 1). */
FSTAT_API fstat_status fstat_resample(const fstat_plan* plan, const fstat_inputs* in,
                            const double* templates, int64_t ntmpl, void* y, void* workspace,
                            size_t ws_bytes, void* stream);

/* Gradient of a weighted sum of 2F with respect to the template parameters
 * (the derivative of the pipeline of Sec. 3, steps (iii)-(vii), and of
 * eq. Fstat; the paper itself computes no derivatives).  For each template m:
 *   grad[m][q] = d/d theta_q sum_b grad_twoF[m][b] * 2F_m[b],
 *   theta = (df, f1dot, alpha, delta, asini, porb, tp)
 * through the spin-down phase, the FFT, the sinc interpolation, the timing
 * model (both delay solves), the sample correction and the antenna weights
 * including the dependence of A, B, C on the sky position.  f2dot is held
 * fixed.  For an isolated source (asini = 0) the orbit derivatives are 0.
 * The forward path is run again inside this call (nothing is kept from an
 * earlier 2F call): the resampled series is recomputed, the adjoint
 * spectrum g conj(F) is transformed by the same FFT kernels, and one kernel
 * recomputes the series with its derivatives and reduces the gradient in
 * FP64 per template (fixed order: deterministic).
 *   templates: device double [ntmpl][8] as for fstat_compute_2f;
 *   grad_twoF: device float [ntmpl][n_bins], the weights g (e.g. the upstream
 *              gradient of a loss with respect to twoF);
 *   grad:      device double [ntmpl][7] (output);
 *   twoF:      nullable device float [ntmpl][n_bins], receives 2F as well.
 * A template flagged as in fstat_compute_2f gets NaN in all seven entries
 * (and in its 2F row).  The workspace must hold fstat_grad_workspace_size
 * (plan, 1) bytes at least; more lets more templates (up to 32) share each
 * launch. */
FSTAT_API fstat_status fstat_grad_workspace_size(const fstat_plan* plan, int64_t batch,
                                                 size_t* bytes);
FSTAT_API fstat_status fstat_compute_2f_grad(const fstat_plan* plan, const fstat_inputs* in,
                                             const double* templates, int64_t ntmpl,
                                             const float* grad_twoF, double* grad, float* twoF,
                                             void* workspace, size_t ws_bytes, void* stream);

/* Single-bin refinement form of fstat_compute_2f_grad: template m has one
 * bin bins[m] (device int64 [ntmpl], index into the band [0, n_bins)) and the
 * weights are one-hot there, L_m = 2F_m(bins[m]).  The transforms are needed
 * at that one bin only, so no FFT runs: the resampling kernel reduces the
 * direct sum Fa'(m), Fb'(m) over the grid (step (vi) for one output bin), and
 * the gradient kernel forms the adjoint series in closed form
 * X_k = conj(F'(m)) exp(-2 pi i m k / N).  Two passes over the input data per
 * template, and a workspace of about 1 KiB plus 64 bytes per 512 grid points
 * per template in flight (fstat_grad_bin_workspace_size; up to 32 per
 * launch).  Outputs: twoF (nullable) device float [ntmpl] = 2F at the bin;
 * grad device double [ntmpl][7] as in fstat_compute_2f_grad.  A flagged
 * template or a bin outside the band gives NaN. */
FSTAT_API fstat_status fstat_grad_bin_workspace_size(const fstat_plan* plan, int64_t batch,
                                                     size_t* bytes);
FSTAT_API fstat_status fstat_compute_2f_grad_bin(const fstat_plan* plan, const fstat_inputs* in,
                                                 const double* templates, int64_t ntmpl,
                                                 const int64_t* bins, float* twoF, double* grad,
                                                 void* workspace, size_t ws_bytes, void* stream);

/* Templates whose outputs the last call on `workspace` set to NaN (any
 * status bit: parameters not finite or out of range, delays beyond
 * max_delay, a tile's input window beyond the staging capacity, a bin
 * outside the band).  Every compute call clears the count in its first
 * kernel and counts each such template once: fstat_compute_2f, _batched,
 * _profiled, fstat_search_run, _run_candidates, _run_profiled, each
 * search's own workspace after fstat_batch_run, fstat_compute_2f_grad and
 * fstat_compute_2f_grad_bin.  (The paper's problem statement has one 2F per
 * template and bin; a NaN row is this library's report of a template it
 * cannot evaluate.)  Waits for the stream, then writes the count to the host
 * int64 *count. */
FSTAT_API fstat_status fstat_flagged_count(const void* workspace, size_t ws_bytes, void* stream,
                                           int64_t* count);

/* fstat_compute_2f_grad_bin for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation, with the workspace taken from a static
 * device array of the library (32 MiB per GPU, held until the process ends)
 * instead of an argument.  Calls nothing that allocates.  Fails with
 * FSTAT_EWORKSPACE when fstat_grad_bin_workspace_size(plan, 1) exceeds the
 * array (a 2^24-point grid needs about 2.2 MB per template); as many
 * templates as fit, up to 32, share each launch.  Every call on one GPU
 * uses that GPU's one array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller. */
FSTAT_API fstat_status fstat_compute_2f_grad_bin_noalloc(const fstat_plan* plan,
                                                         const fstat_inputs* in,
                                                         const double* templates, int64_t ntmpl,
                                                         const int64_t* bins, float* twoF,
                                                         double* grad, void* stream);

/* Wait for the stream and report any asynchronous HIP error as FSTAT_EHIP. */
FSTAT_API fstat_status fstat_sync_check(void* stream);

/* Thread-local description of the last failure in this thread ("" if none). */
FSTAT_API const char* fstat_last_error(void);

/* Library version string. */
FSTAT_API const char* fstat_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FSTAT_H */
