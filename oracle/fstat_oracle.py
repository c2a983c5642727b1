"""FP64 CPU oracle for the resampling F-statistic.  TEST INFRASTRUCTURE ONLY.

This module exists to check the GPU path.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it; the product library
never calls it and shares no code with it.

It is a plain, slow, step-by-step implementation in float64 of the resampling
algorithm of Sec. 3 (steps (iii)-(vii)) applied to a heterodyned, downsampled
complex series, plus the discretised detector-frame definition of Fa, Fb
(eqs. Fa_DET, Fb_DET of Sec. 2) evaluated as a direct sum, which the resampling
algorithm approximates.  Each function cites the passage it follows.  Where the
paper does not print a formula (antenna patterns, the normalised A, B, C, the
interpolation kernel, the binary and ephemeris models) the reading taken is
stated in the docstring.

Conventions (all times in s, angles in rad, frequencies in Hz, distances in
light-seconds):

* Roemer delay (Sec. 2, t_b = t + t_m): t_b = t + r_X(t) . n, with r_X the
  detector position and n the unit vector towards the source.
* Binary (reading: Roemer term only): t_b = t_src + R(t_src), circular
  R(t') = asini sin(2 pi (t' - tp) / porb), or Keplerian with eccentricity
  and argument of periapsis (binary_delay).
* Spin-down phase (Sec. 2, Phi_s is a Taylor series in f^(k), k >= 1):
  Phi_s(tau) = 2 pi [f1dot (tau - t_ref)^2 / 2 + f2dot (tau - t_ref)^3 / 6].
* Output bin i in [0, n_fft) has frequency f_het + df + (i - n_fft/2)/(n_fft dt).

Parity unpinned: agreement with any third-party implementation of the
paper's CPU or CUDA code (its interpolation kernel, normalisation and timing
routines are not printed).  Everything below is pinned by the tests in
tests/test_oracle_*.py against closed forms, brute force and statistics.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------
# Steps (i)-(ii) of Sec. 3: SFTs to the heterodyned, downsampled series
# ----------------------------------------------------------------------------

def sfts_to_series(sfts, present, k0, t_sft, t_start):
    """x_h(t) on t = t_start + n dt from short Fourier transforms (reading of
    steps (i)-(ii), which the paper leaves to existing code).

    SFT s covers [t_s, t_s + t_sft), t_s = t_start + s t_sft, and holds the K
    bins k = k0 .. k0 + K - 1 (frequency k / t_sft) of the segment's DFT with
    the time-step normalisation X_s[k] = dt_raw sum_n r(t_s + n dt_raw)
    exp(-2 pi i k n / N_sft).  Combining the SFTs into one transform of the
    whole span and keeping the band [k0, k0 + K) / t_sft is the low-pass of
    step (ii); with f_h = (k0 + K/2) / t_sft at the band's centre and
    dt = t_sft / K, the inverse transform over the band, heterodyned by
    exp(-2 pi i f_h t), is, sample by sample,

      x_h(t_s + j dt) = (1 / t_sft) sum_q X_s[k0 + q]
                        exp(2 pi i (k0 + q) j / K) exp(-2 pi i f_h (t_s + j dt)),

    which this function evaluates literally (a K x K sum per SFT, phases
    reduced exactly: (k0 + q) j mod K and f_h t mod 1 in float64).  Missing
    SFTs (present = 0) give zeros and valid = 0.  Returns (x complex128
    [n_sft K], valid uint8, f_h, dt)."""
    sfts = np.asarray(sfts, dtype=np.complex128)
    n_sft, K = sfts.shape
    f_h = (k0 + K / 2) / t_sft
    dt = t_sft / K
    j = np.arange(K)
    q = np.arange(K)
    E = np.exp(2j * np.pi * (((k0 + q)[None, :] * j[:, None]) % K) / K)
    x = np.zeros(n_sft * K, dtype=np.complex128)
    valid = np.zeros(n_sft * K, dtype=np.uint8)
    for s in range(n_sft):
        if not present[s]:
            continue
        t = t_start + s * t_sft + j * dt
        het = np.exp(-2j * np.pi * np.mod(f_h * t, 1.0))
        x[s * K:(s + 1) * K] = (E @ sfts[s]) * het / t_sft
        valid[s * K:(s + 1) * K] = 1
    return x, valid, f_h, dt


# ----------------------------------------------------------------------------
# O1-O2: sky vector, detector position and Roemer delay (Sec. 2, t_m; step iv)
# ----------------------------------------------------------------------------

def sky_vector(alpha, delta):
    """Unit vector towards the source in equatorial coordinates."""
    return np.array([math.cos(delta) * math.cos(alpha),
                     math.cos(delta) * math.sin(alpha),
                     math.sin(delta)])


def detector_position(model, det, t):
    """Detector position (light-s), shape (3, n), for the analytic ephemeris:
    circular Earth orbit inclined by the obliquity plus a rotating site on a
    spherical Earth (reading of the unprinted ephemeris, Sec. 2 t_m)."""
    t = np.asarray(t, dtype=np.float64)
    th = model["orbit_phase0_rad"] + TWO_PI * t / model["period_orbit_s"]
    eps = model["obliquity_rad"]
    r_o = model["r_orbit_s"]
    phi = sidereal_angle(model, det, t)
    r_e = model["r_earth_s"]
    x = r_o * np.cos(th) + r_e * math.cos(det.lat) * np.cos(phi)
    y = r_o * np.sin(th) * math.cos(eps) + r_e * math.cos(det.lat) * np.sin(phi)
    z = r_o * np.sin(th) * math.sin(eps) + r_e * math.sin(det.lat) + 0.0 * t
    return np.stack([x, y, z])


def sidereal_angle(model, det, t):
    """Local sidereal angle of the detector meridian."""
    return det.lon + model["sidereal_angle0_rad"] + model["sidereal_rate_rad_s"] * np.asarray(t)


def roemer_delay(model, det, nhat, t):
    """t_b - t for detector time t: projection of the detector position on n."""
    return nhat @ detector_position(model, det, t)


# ----------------------------------------------------------------------------
# O3: circular binary Roemer delay (reading of the orbit model varied in Sec. 4.2)
# ----------------------------------------------------------------------------

def eccentric_anomaly(mean_anomaly, ecc):
    """E solving Kepler's equation E - e sin E = M: M is reduced to
    [-pi, pi] by whole turns, then Newton's iteration from E = M + e sin M
    runs until the update is at the rounding level."""
    M = np.asarray(mean_anomaly, dtype=np.float64)
    turns = np.round(M / TWO_PI)
    Mr = M - TWO_PI * turns
    E = Mr + ecc * np.sin(Mr)
    for _ in range(100):
        step = (E - ecc * np.sin(E) - Mr) / (1.0 - ecc * np.cos(E))
        E = E - step
        if np.max(np.abs(step), initial=0.0) < 1e-15:
            return E + TWO_PI * turns
    raise RuntimeError("Kepler's equation did not converge")


def binary_delay(tm, t_src):
    """R(t') of the source's orbit (Roemer term only).  Circular orbit
    (ecc = argp = 0): asini sin(2 pi (t' - tp) / porb), tp the time of the
    ascending node.  Eccentric orbit (reading of the orbital elements the
    paper's binary searches vary, the period among them, Sec. 4.2): mean
    anomaly M = 2 pi (t' - tp) / porb with tp the time of periapsis, E from
    Kepler's equation, and
    R = asini [sin(argp) (cos E - ecc) + cos(argp) sqrt(1 - ecc^2) sin E],
    which for ecc = argp = 0 is the circular form."""
    asini, porb, tp = tm["asini"], tm["porb"], tm["tp"]
    if asini == 0.0:
        return np.zeros_like(np.asarray(t_src, dtype=np.float64))
    ecc, argp = tm.get("ecc", 0.0), tm.get("argp", 0.0)
    M = TWO_PI * (np.asarray(t_src, dtype=np.float64) - tp) / porb
    if ecc == 0.0 and argp == 0.0:
        return asini * np.sin(M)
    E = eccentric_anomaly(M, ecc)
    return asini * (math.sin(argp) * (np.cos(E) - ecc) +
                    math.cos(argp) * math.sqrt(1.0 - ecc * ecc) * np.sin(E))


def emission_time_delay(tm, t_b):
    """Return R(t_src) where t_src solves t_src + R(t_src) = t_b.

    Plain fixed-point iteration t_src <- t_b - R(t_src); the map contracts with
    factor max|R'| (asini * 2 pi / porb for a circular orbit) < 1e-2 for every
    orbit considered."""
    t_b = np.asarray(t_b, dtype=np.float64)
    r = np.zeros_like(t_b)
    if tm["asini"] == 0.0:
        return r
    for _ in range(200):
        r_new = binary_delay(tm, t_b - r)
        if np.max(np.abs(r_new - r)) < 1e-13:
            return r_new
        r = r_new
    raise RuntimeError("binary inversion did not converge")


# ----------------------------------------------------------------------------
# O5: detector epochs for a regular source-frame grid (step iv)
# ----------------------------------------------------------------------------

def detector_epochs(model, det, nhat, tm, tau):
    """For source-frame times tau return (T, delay) with T the detector time
    whose emission time is tau; delay = T - tau.

    t_b = tau + R(tau); T solves T + roemer(T) = t_b by fixed-point iteration
    started at T = t_b (contraction |d roemer/dt| < 1e-4)."""
    tau = np.asarray(tau, dtype=np.float64)
    rb = binary_delay(tm, tau)
    t_b = tau + rb
    dr = roemer_delay(model, det, nhat, t_b)
    for _ in range(100):
        dr_new = roemer_delay(model, det, nhat, t_b - dr)
        if np.max(np.abs(dr_new - dr)) < 1e-12:
            dr = dr_new
            break
        dr = dr_new
    else:
        raise RuntimeError("Roemer inversion did not converge")
    delay = rb - dr          # T - tau, a small number
    return tau + delay, delay


# ----------------------------------------------------------------------------
# O6: heterodyne correction at the detector samples (step iii)
# ----------------------------------------------------------------------------

def corrected_series(model, det, nhat, tm, x, dt, f_het):
    """z_j = x_j exp(-2 pi i f_het (t_src,j - t_j)).

    Step (iii) moves the heterodyne from the detector frame to the source
    frame.  The sign is fixed by the heterodyne convention x ~ exp(+i(Phi -
    2 pi f_het t)): after the correction z ~ exp(+2 pi i (f - f_het) t_src).
    The delay t_src - t_j = roemer(t_j) - R(t_src,j) is formed from small
    numbers before multiplying by f_het."""
    t = det.t0 + dt * np.arange(det.n)
    roem = roemer_delay(model, det, nhat, t)
    t_b = t + roem
    rbin = emission_time_delay(tm, t_b)
    delay = roem - rbin
    cyc = np.mod(f_het * delay, 1.0)
    return np.asarray(x, dtype=np.complex128) * np.exp(-1j * TWO_PI * cyc)


# ----------------------------------------------------------------------------
# O7: interpolation onto the detector epochs (step v)
# ----------------------------------------------------------------------------

def sinc_kernel(s, D):
    """Hann-windowed sinc of half-width D (reading: the paper does not name
    the interpolation kernel).  h(s) = sinc(s) (1 + cos(pi s / D)) / 2 for
    |s| < D, else 0; sinc(0) = 1."""
    s = np.asarray(s, dtype=np.float64)
    h = np.sinc(s) * 0.5 * (1.0 + np.cos(np.pi * s / D))
    return np.where(np.abs(s) < D, h, 0.0)


def interpolate(z, u, D):
    """zhat(u) = sum_{j = floor(u)-D+1}^{floor(u)+D} z_j h(u - j); z_j = 0
    for j outside [0, len(z))."""
    u = np.asarray(u, dtype=np.float64)
    j0 = np.floor(u).astype(np.int64)
    out = np.zeros(u.shape, dtype=np.complex128)
    n = len(z)
    for i in range(2 * D):
        j = j0 - D + 1 + i
        ok = (j >= 0) & (j < n)
        w = sinc_kernel(u - j, D)
        out += np.where(ok, w * z[np.clip(j, 0, n - 1)], 0.0)
    return out


# ----------------------------------------------------------------------------
# O8: antenna patterns a(t), b(t)
# ----------------------------------------------------------------------------

def antenna_ab(model, det, alpha, delta, t):
    """a(t), b(t) of a 90-degree interferometer (closed form of Jaranowski,
    Krolak & Schutz 1998, eqs. 12-13, which Sec. 2 cites but does not print).

    gamma is the azimuth of the arm bisector measured counter-clockwise from
    local East, lambda the latitude, x = alpha - (local sidereal angle)."""
    lam = det.lat
    gam = 0.5 * (det.az_x + det.az_y)
    x = alpha - sidereal_angle(model, det, t)
    s2g, c2g = math.sin(2 * gam), math.cos(2 * gam)
    sl, cl = math.sin(lam), math.cos(lam)
    s2l, c2l = math.sin(2 * lam), math.cos(2 * lam)
    sd, cd = math.sin(delta), math.cos(delta)
    s2d, c2d = math.sin(2 * delta), math.cos(2 * delta)
    a = (s2g * (3 - c2l) * (3 - c2d) * np.cos(2 * x) / 16.0
         - c2g * sl * (3 - c2d) * np.sin(2 * x) / 4.0
         + s2g * s2l * s2d * np.cos(x) / 4.0
         - c2g * cl * s2d * np.sin(x) / 2.0
         + 0.75 * s2g * cl * cl * cd * cd)
    b = (c2g * sl * sd * np.cos(2 * x)
         + s2g * (3 - c2l) * sd * np.sin(2 * x) / 4.0
         + c2g * cl * cd * np.cos(x)
         + s2g * s2l * cd * np.sin(x) / 2.0)
    return a, b


# ----------------------------------------------------------------------------
# O9: spin-down phase (Sec. 2, Phi_s) and sub-bin offset
# ----------------------------------------------------------------------------

def spindown_cycles(tm, tau, t_ref):
    """Phi_s(tau) / (2 pi), reduced modulo one cycle."""
    dtau = np.asarray(tau, dtype=np.float64) - t_ref
    return np.mod(tm["f1dot"] * dtau ** 2 / 2.0 + tm["f2dot"] * dtau ** 3 / 6.0, 1.0)


# ----------------------------------------------------------------------------
# O12-O13: antenna-pattern matrix and 2F (Sec. 2 eq. Fstat)
# ----------------------------------------------------------------------------

def antenna_matrix(model, dets, valid, alpha, delta, dt):
    """A, B, C: noise-weighted sums of a^2, b^2, ab over the valid detector
    samples (reading of the normalised A, B, C: the discrete counterpart of the
    integrals in eq. Fstat, weights w_X = 1/sigma_X^2)."""
    A = B = C = 0.0
    for det, v in zip(dets, valid):
        t = det.t0 + dt * np.arange(det.n)
        a, b = antenna_ab(model, det, alpha, delta, t)
        w = 1.0 / det.noise_var
        m = np.asarray(v, dtype=np.float64)
        A += w * np.sum(m * a * a)
        B += w * np.sum(m * b * b)
        C += w * np.sum(m * a * b)
    return A, B, C


def two_f(Fa, Fb, A, B, C):
    """2F = 2 (B|Fa|^2 + A|Fb|^2 - 2 C Re(Fa Fb*)) / D, D = AB - C^2."""
    D = A * B - C * C
    return 2.0 * (B * np.abs(Fa) ** 2 + A * np.abs(Fb) ** 2
                  - 2.0 * C * np.real(Fa * np.conj(Fb))) / D


# ----------------------------------------------------------------------------
# The resampling algorithm, steps (iii)-(vii) of Sec. 3
# ----------------------------------------------------------------------------

def template_dict(row):
    """Template row: (alpha, delta, df, f1dot, f2dot, asini, porb, tp) and, in
    rows of ten, the eccentricity and the argument of periapsis."""
    tm = dict(alpha=float(row[0]), delta=float(row[1]), df=float(row[2]), f1dot=float(row[3]),
              f2dot=float(row[4]), asini=float(row[5]), porb=float(row[6]), tp=float(row[7]),
              ecc=0.0, argp=0.0)
    if len(row) >= 10:
        tm["ecc"], tm["argp"] = float(row[8]), float(row[9])
    return tm


def resampled_series(ds, tm):
    """y_a, y_b on the source-frame grid tau_k = tau0 + k dt, k < n_fft.

    For each detector: (iii) correct the heterodyne at the input samples,
    (iv) find the detector epochs of the regular grid, (v) interpolate, then
    weight by w_X a(T_k), w_X b(T_k) and sum over detectors (linearity: the
    multi-detector sum of Sec. 3 taken before the transform); finally remove
    the spin-down phase and the sub-bin frequency offset."""
    model = ds.ephem_model
    nhat = sky_vector(tm["alpha"], tm["delta"])
    k = np.arange(ds.n_fft)
    tau = ds.tau0 + ds.dt * k
    ya = np.zeros(ds.n_fft, dtype=np.complex128)
    yb = np.zeros(ds.n_fft, dtype=np.complex128)
    for det, x in zip(ds.detectors, ds.x):
        z = corrected_series(model, det, nhat, tm, x, ds.dt, ds.f_het)
        T, delay = detector_epochs(model, det, nhat, tm, tau)
        # u = (T - t0)/dt assembled from small terms
        u = k + (ds.tau0 - det.t0) / ds.dt + delay / ds.dt
        zh = interpolate(z, u, ds.sinc_halfwidth)
        a, b = antenna_ab(model, det, tm["alpha"], tm["delta"], T)
        w = 1.0 / det.noise_var
        ya += w * a * zh
        yb += w * b * zh
    cyc = spindown_cycles(tm, tau, ds.t_ref) + np.mod(tm["df"] * (tau - ds.tau0), 1.0)
    rot = np.exp(-1j * TWO_PI * cyc)
    return ya * rot, yb * rot


def fa_fb(ds, tm):
    """Step (vi): forward DFT (negative exponent, no 1/N) of y_a and y_b,
    returned on the output bins in ascending frequency."""
    ya, yb = resampled_series(ds, tm)
    Fa = np.fft.fftshift(np.fft.fft(ya))
    Fb = np.fft.fftshift(np.fft.fft(yb))
    sl = slice(ds.bin_lo, ds.bin_lo + ds.n_bins)
    return Fa[sl], Fb[sl]


def oracle_twoF(ds, templates=None, return_fafb=False):
    """2F over the output band for each template: steps (iii)-(vii)."""
    templates = ds.templates if templates is None else np.atleast_2d(templates)
    out = np.empty((templates.shape[0], ds.n_bins), dtype=np.float64)
    fafb = []
    for i, row in enumerate(templates):
        tm = template_dict(row)
        Fa, Fb = fa_fb(ds, tm)
        A, B, C = antenna_matrix(ds.ephem_model, ds.detectors, ds.valid, tm["alpha"], tm["delta"],
                                 ds.dt)
        out[i] = two_f(Fa, Fb, A, B, C)
        if return_fafb:
            fafb.append((Fa, Fb, (A, B, C)))
    return (out, fafb) if return_fafb else out


def twoF_at_bin(ds, row, i):
    """2F of one template at band bin i only: steps (iii)-(v) as in
    resampled_series, then step (vi) restricted to that one output bin, the
    DFT sum F[m] = sum_k y_k exp(-2 pi i m k / n_fft) at the natural index m
    of band bin i (no FFT), then eq. Fstat.  Cost O(n_fft) after the
    resampling, for checks at sizes where a full transform per evaluation is
    not wanted."""
    tm = template_dict(row)
    ya, yb = resampled_series(ds, tm)
    m = (ds.bin_lo + int(i) + ds.n_fft // 2) % ds.n_fft
    k = np.arange(ds.n_fft)
    e = np.exp(-1j * TWO_PI * ((m * k) % ds.n_fft) / ds.n_fft)
    Fa, Fb = np.sum(ya * e), np.sum(yb * e)
    A, B, C = antenna_matrix(ds.ephem_model, ds.detectors, ds.valid, tm["alpha"], tm["delta"],
                             ds.dt)
    return float(two_f(Fa, Fb, A, B, C))


# ----------------------------------------------------------------------------
# Direct sum: eqs. Fa_DET, Fb_DET of Sec. 2 discretised over the samples
# ----------------------------------------------------------------------------

def direct_fa_fb(ds, tm, freqs):
    """Fa(f), Fb(f) = sum_X w_X sum_j v_j {a,b}(t_j) x_j exp(-i Psi_j(f)) with
    Psi_j(f) = 2 pi (f - f_het)(t_src,j - tau0) + 2 pi f_het (t_src,j - t_j)
    + Phi_s(t_src,j) + 2 pi df ... (df is part of f here).

    This is the detector-frame definition: no change of variables, no
    interpolation.  Cost O(n_samples * n_freqs); use on small inputs."""
    model = ds.ephem_model
    nhat = sky_vector(tm["alpha"], tm["delta"])
    freqs = np.atleast_1d(np.asarray(freqs, dtype=np.float64))
    Fa = np.zeros(freqs.shape, dtype=np.complex128)
    Fb = np.zeros(freqs.shape, dtype=np.complex128)
    for det, x, v in zip(ds.detectors, ds.x, ds.valid):
        t = det.t0 + ds.dt * np.arange(det.n)
        roem = roemer_delay(model, det, nhat, t)
        rbin = emission_time_delay(tm, t + roem)
        delay = roem - rbin                      # t_src - t
        t_src_rel = (t - ds.tau0) + delay        # t_src - tau0
        a, b = antenna_ab(model, det, tm["alpha"], tm["delta"], t)
        w = 1.0 / det.noise_var
        base = np.mod(ds.f_het * delay, 1.0) + spindown_cycles(tm, t + delay, ds.t_ref)
        xv = np.asarray(x, dtype=np.complex128) * np.asarray(v, dtype=np.float64)
        for s0 in range(0, len(freqs), 256):
            fr = freqs[s0:s0 + 256] - ds.f_het
            cyc = np.mod(np.outer(fr, t_src_rel), 1.0) + base[None, :]
            e = np.exp(-1j * TWO_PI * cyc)
            Fa[s0:s0 + 256] += w * (e @ (a * xv))
            Fb[s0:s0 + 256] += w * (e @ (b * xv))
    return Fa, Fb


def direct_twoF(ds, tm, freqs):
    Fa, Fb = direct_fa_fb(ds, tm, freqs)
    A, B, C = antenna_matrix(ds.ephem_model, ds.detectors, ds.valid, tm["alpha"], tm["delta"], ds.dt)
    return two_f(Fa, Fb, A, B, C)


# ----------------------------------------------------------------------------
# Comparison metrics of Sec. 4.2
# ----------------------------------------------------------------------------

def _f64(v):
    v = np.ravel(v)
    return v.astype(np.complex128) if np.iscomplexobj(v) else v.astype(np.float64)


def rel_err(x, y, p):
    """r_p(x, y) = 2 |x - y|_p / (|x|_p + |y|_p), evaluated in float64."""
    x, y = _f64(x), _f64(y)
    n = lambda v: np.linalg.norm(v, ord=p)
    return 2.0 * n(x - y) / (n(x) + n(y))


def angle(x, y):
    """theta = arccos[Re(x* . y) / (|x|_2 |y|_2)]: the angle between x and y
    as real vectors, evaluated in float64 as 2 atan2(|u - v|, |u + v|) on the
    unit vectors u, v (the same angle, without arccos's loss near 0)."""
    x, y = _f64(x), _f64(y)
    u = x / np.linalg.norm(x)
    v = y / np.linalg.norm(y)
    return float(2.0 * np.arctan2(np.linalg.norm(u - v), np.linalg.norm(u + v)))
