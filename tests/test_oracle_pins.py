"""Pins of the FP64 oracle against closed forms, brute force and statistics.

Each test fixes one part of the oracle by something other than the oracle
itself, so that a dropped term, a wrong sign or index, or a transposed operand
anywhere in it fails at least one test.
"""
import math
import os

import numpy as np
import pytest

from oracle import fstat_oracle as O
from paper_2201_00451_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def on_bin(ds, f):
    """df and bin index that put frequency f exactly on an output bin."""
    m = round((f - ds.f_het) * ds.n_fft * ds.dt)
    return f - ds.f_het - m / (ds.n_fft * ds.dt), m + ds.n_fft // 2


# --------------------------------------------------------------------------
# Interpolation kernel (step v)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("D", [4, 8, 12])
def test_sinc_exact_at_integer_offsets(D):
    rng = np.random.default_rng(0)
    z = rng.standard_normal(200) + 1j * rng.standard_normal(200)
    u = np.arange(0, 200).astype(np.float64)
    np.testing.assert_allclose(O.interpolate(z, u, D), z, rtol=0, atol=1e-15)
    s = np.arange(-D - 2, D + 3).astype(float)
    h = O.sinc_kernel(s, D)
    assert h[s == 0][0] == 1.0
    assert np.all(np.abs(h[s != 0]) < 1e-15)


@pytest.mark.parametrize("D", [3, 8])
def test_interpolation_equals_full_convolution(D):
    """Brute force: sum over every sample j of z_j h(u - j) equals the 2D-tap
    window used by the interpolation, including samples near both data ends."""
    rng = np.random.default_rng(4)
    z = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    u = rng.uniform(-D, 40 + D, 300)
    j = np.arange(40)
    brute = np.array([np.sum(z * O.sinc_kernel(ui - j, D)) for ui in u])
    np.testing.assert_allclose(O.interpolate(z, u, D), brute, rtol=0, atol=1e-13)


def test_sinc_tone_response_bound():
    """A tone at |nu| <= 0.4 cycles/sample is reproduced within the Hann-sinc
    D = 8 passband ripple (7.8e-3), and worse near Nyquist: fixes the window
    shape and half-width."""
    rng = np.random.default_rng(1)
    j = np.arange(400)
    u = 150 + rng.uniform(0, 100, 500)
    worst_in = 0.0
    for nu in np.linspace(-0.4, 0.4, 17):
        z = np.exp(2j * np.pi * nu * j)
        err = np.abs(O.interpolate(z, u, 8) - np.exp(2j * np.pi * nu * u))
        worst_in = max(worst_in, err.max())
    assert 1e-4 < worst_in < 7.8e-3
    z = np.exp(2j * np.pi * 0.49 * j)
    err = np.abs(O.interpolate(z, u, 8) - np.exp(2j * np.pi * 0.49 * u)).max()
    assert err > 0.1


# --------------------------------------------------------------------------
# Antenna patterns (JKS closed form) vs the tensor route of the generator
# --------------------------------------------------------------------------

@pytest.mark.parametrize("site", ["H", "L"])
def test_jks_is_linear_map_of_tensor_route(site):
    m = synth.EPHEM_MODEL
    det = synth.make_detector(site, 0, 10, 1.0)
    rng = np.random.default_rng(2)
    t = np.linspace(0, 2 * 86400, 3000)
    for _ in range(5):
        al, de, psi = rng.uniform(0, 2 * np.pi), rng.uniform(-1.5, 1.5), rng.uniform(-1, 1)
        a, b = O.antenna_ab(m, det, al, de, t)
        fp, fx = synth.tensor_response(m, det, al, de, psi, t)
        X = np.stack([a, b], 1)
        L, *_ = np.linalg.lstsq(X, np.stack([fp, fx], 1), rcond=None)
        assert np.abs(X @ L - np.stack([fp, fx], 1)).max() < 1e-12
        # the map is a rotation by 2 psi combined with a reflection
        np.testing.assert_allclose(L @ L.T, np.eye(2), atol=1e-12)


def test_jks_gamma_sign_is_detected():
    """Negative control: mirroring the arm orientation breaks the linear map."""
    m = synth.EPHEM_MODEL
    det = synth.make_detector("H", 0, 10, 1.0)
    bad = synth.Detector("bad", det.lat, det.lon, -det.az_x, -det.az_y, 0, 10, 1.0)
    t = np.linspace(0, 86400, 2000)
    a, b = O.antenna_ab(m, bad, 1.0, -0.5, t)
    fp, fx = synth.tensor_response(m, det, 1.0, -0.5, 0.0, t)
    X = np.stack([a, b], 1)
    L, *_ = np.linalg.lstsq(X, np.stack([fp, fx], 1), rcond=None)
    assert np.abs(X @ L - np.stack([fp, fx], 1)).max() > 0.05


def test_polar_detector_polar_source():
    m = synth.EPHEM_MODEL
    det = synth.Detector("pole", math.pi / 2, 0.3, 0.4, 0.4 + math.pi / 2, 0, 10, 1.0)
    t = np.linspace(0, 86400, 500)
    a, b = O.antenna_ab(m, det, 0.7, math.pi / 2, t)
    np.testing.assert_allclose(a * a + b * b, 1.0, atol=1e-14)


# --------------------------------------------------------------------------
# Timing (steps iii, iv)
# --------------------------------------------------------------------------

def test_roemer_bounds_and_ecliptic_pole():
    m = synth.EPHEM_MODEL
    det = synth.make_detector("L", 0, 10, 1.0)
    t = np.linspace(0, 365.25 * 86400, 20000)
    rng = np.random.default_rng(3)
    for _ in range(4):
        n = O.sky_vector(rng.uniform(0, 6.3), rng.uniform(-1.5, 1.5))
        d = O.roemer_delay(m, det, n, t)
        assert np.abs(d).max() <= m["r_orbit_s"] + m["r_earth_s"] + 1e-9
    eps = m["obliquity_rad"]
    pole = np.array([0.0, -math.sin(eps), math.cos(eps)])
    d = O.roemer_delay(m, det, pole, t)
    # only the rotating site remains: bounded by the Earth radius
    assert np.abs(d).max() <= m["r_earth_s"] + 1e-12
    assert np.ptp(d) > 0.5 * m["r_earth_s"] * math.cos(det.lat)


@pytest.mark.parametrize("binary", [False, True])
def test_detector_epoch_residual(binary):
    m = synth.EPHEM_MODEL
    det = synth.make_detector("H", 0, 10, 1.0)
    tm = dict(alpha=2.0, delta=0.3, df=0, f1dot=0, f2dot=0, asini=0.8 if binary else 0.0,
              porb=0.25 * 86400, tp=1234.5)
    tau = np.linspace(-600, 20 * 86400, 5001)
    n = O.sky_vector(tm["alpha"], tm["delta"])
    T, delay = O.detector_epochs(m, det, n, tm, tau)
    t_b = tau + O.binary_delay(tm, tau)
    res = T + O.roemer_delay(m, det, n, T) - t_b
    assert np.abs(res).max() < 1e-9
    # the binary inversion used at the input samples is the inverse map
    rb = O.emission_time_delay(tm, t_b)
    np.testing.assert_allclose(tau + 0 * rb, t_b - rb, atol=1e-8)


def test_binary_zero_amplitude_is_isolated():
    ds = synth.small_case(seed=21, n=3000, n_fft=1 << 13, noise=True)
    row = ds.templates[0].copy()
    iso = O.oracle_twoF(ds, row[None])[0]
    row[5], row[6], row[7] = 0.0, 4321.0, 99.0
    np.testing.assert_array_equal(O.oracle_twoF(ds, row[None])[0], iso)


# --------------------------------------------------------------------------
# Whole method against the detector-frame definition (direct sum)
# --------------------------------------------------------------------------

def test_zero_ephemeris_reduces_to_dft():
    """No detector motion, no binary, no spin-down and a grid aligned with the
    samples: resampling is the identity and Fa is the plain DFT of w a x."""
    model = dict(synth.EPHEM_MODEL, r_orbit_s=0.0, r_earth_s=0.0)
    ds = synth.small_case(seed=22, n=1500, n_fft=1 << 12, ndet=2, noise=True, model=model,
                          f1dot=0.0, noise_vars=[0.7, 1.3])
    tm = O.template_dict(ds.templates[1])
    Fa, Fb = O.fa_fb(ds, tm)
    N, off = ds.n_fft, int(round((0.0 - ds.tau0) / ds.dt))
    m = np.arange(N) - N // 2
    k = np.arange(1500) + off
    E = np.exp(-2j * np.pi * np.outer(m, k) / N)
    ra = np.zeros(N, complex)
    rb = np.zeros(N, complex)
    for det, x in zip(ds.detectors, ds.x):
        a, b = O.antenna_ab(model, det, tm["alpha"], tm["delta"], det.t0 + ds.dt * np.arange(det.n))
        ra += E @ (a * x / det.noise_var)
        rb += E @ (b * x / det.noise_var)
    assert O.rel_err(Fa, ra, 2) < 1e-12
    assert O.rel_err(Fb, rb, 2) < 1e-12
    # and the direct sum evaluated on the bin frequencies agrees too
    dFa, dFb = O.direct_fa_fb(ds, tm, ds.bin_frequencies(tm["df"]))
    assert O.rel_err(Fa, dFa, 2) < 1e-11


@pytest.mark.parametrize("binary,ndet,gaps", [(False, 1, False), (False, 2, True), (True, 2, True)])
def test_noiseless_direct_sum_equals_rho2(binary, ndet, gaps):
    """At the injected parameters, 2F of the direct sum is the optimal SNR^2."""
    ds = synth.small_case(seed=23, n=5000, n_fft=1 << 14, ndet=ndet, noise=False, binary=binary,
                          gaps=gaps, keep_f64=True, noise_vars=[0.9, 1.2][:ndet])
    inj = ds.injections[0]
    tm = O.template_dict(ds.templates[0])
    v = O.direct_twoF(ds, tm, [inj["f"]])[0]
    assert abs(v / inj["rho2"] - 1) < 1e-11


@pytest.mark.parametrize("binary", [False, True])
def test_resampled_matches_direct_sum(binary):
    """Resampling approximates the direct sum (interpolation and dt/dt_b ~ 1):
    Fa, Fb near the peak agree to the ~1e-3 level; the peak recovers rho^2."""
    ds = synth.small_case(seed=24, n=6000, n_fft=1 << 14, ndet=2, noise=False, binary=binary,
                          gaps=True, f_inj=0.05)
    inj = ds.injections[0]
    tm = O.template_dict(ds.templates[0])
    tm["df"], ipk = on_bin(ds, inj["f"])
    Fa, Fb = O.fa_fb(ds, tm)
    A, B, C = O.antenna_matrix(ds.ephem_model, ds.detectors, ds.valid, tm["alpha"], tm["delta"], ds.dt)
    tf = O.two_f(Fa, Fb, A, B, C)
    assert int(np.argmax(tf)) == ipk
    assert abs(tf[ipk] / inj["rho2"] - 1.0) < 5e-3
    idx = np.arange(ipk - 30, ipk + 31)
    dFa, dFb = O.direct_fa_fb(ds, tm, ds.bin_frequencies(tm["df"])[idx])
    assert O.rel_err(Fa[idx], dFa, 2) < 3e-3
    assert O.rel_err(Fb[idx], dFb, 2) < 3e-3
    assert O.angle(Fa[idx], dFa) < 3e-3


def test_resampled_noise_band_matches_direct_sum():
    """Pure noise over the inner 80% of the band: 2F of both routes agree."""
    ds = synth.small_case(seed=25, n=3000, n_fft=1 << 13, noise=True, rho=0.0)
    tm = O.template_dict(ds.templates[0])
    tf = O.oracle_twoF(ds, ds.templates[:1])[0]
    N = ds.n_fft
    idx = np.arange(N // 2 - int(0.4 * N), N // 2 + int(0.4 * N), 7)
    d = O.direct_twoF(ds, tm, ds.bin_frequencies()[idx])
    assert O.rel_err(tf[idx], d, 2) < 1e-2


# --------------------------------------------------------------------------
# Invariances and closed-form shifts
# --------------------------------------------------------------------------

def test_grid_origin_shift_invariance():
    ds = synth.small_case(seed=26, n=3000, n_fft=1 << 13, noise=True, binary=True)
    ref = O.oracle_twoF(ds, ds.templates[:1])[0]
    ds.tau0 -= 37 * ds.dt
    np.testing.assert_allclose(O.oracle_twoF(ds, ds.templates[:1])[0], ref, rtol=1e-9, atol=1e-9)


def test_spindown_reference_time_shift():
    """Phi_s(tau; t_ref + s) = Phi_s(tau; t_ref) - 2 pi f1dot s (tau - t_ref) + const,
    so moving t_ref by s moves the 2F spectrum up by f1dot * s in frequency."""
    ds = synth.small_case(seed=27, n=3000, n_fft=1 << 13, noise=True, f1dot=0.0)
    row = ds.templates[0].copy()
    row[3] = 2.5e-9
    shift_bins = 5
    s = shift_bins / (ds.n_fft * ds.dt * row[3])
    ref = O.oracle_twoF(ds, row[None])[0]
    ds.t_ref += s
    moved = O.oracle_twoF(ds, row[None])[0]
    np.testing.assert_allclose(moved[shift_bins:], ref[:-shift_bins], rtol=1e-8, atol=1e-8)


def test_second_spindown_term_noiseless_rho2():
    """Phi_s carries the second frequency derivative as f2dot (tau - t_ref)^3 / 6
    (Sec. 2: Phi_s is the Taylor series in the f^(k)).  The generator injects
    a source whose cubic term moves its phase by about 1.7 cycles over the
    data; at the injected parameters the noiseless direct sum recovers the
    optimal rho^2 exactly, which a wrong Taylor factor (or a dropped cubic)
    does not."""
    ds = synth.small_case(seed=61, n=5000, n_fft=1 << 14, ndet=2, noise=False, keep_f64=True,
                          f2dot=1e-11, gaps=True)
    inj = ds.injections[0]
    tm = O.template_dict(ds.templates[0])
    assert tm["f2dot"] == 1e-11
    v = O.direct_twoF(ds, tm, [inj["f"]])[0]
    assert abs(v / inj["rho2"] - 1) < 1e-11
    # the resampled series recovers it too (interpolation loss only)
    tm["df"], ipk = on_bin(ds, inj["f"])
    Fa, Fb = O.fa_fb(ds, tm)
    A, B, C = O.antenna_matrix(ds.ephem_model, ds.detectors, ds.valid, tm["alpha"], tm["delta"],
                               ds.dt)
    tf = O.two_f(Fa, Fb, A, B, C)
    assert int(np.argmax(tf)) == ipk
    assert abs(tf[ipk] / inj["rho2"] - 1.0) < 5e-3
    # without the cubic term the template loses most of the signal
    tm0 = dict(tm, f2dot=0.0)
    assert O.direct_twoF(ds, tm0, [inj["f"]])[0] < 0.5 * inj["rho2"]


def test_spindown_reference_time_shift_with_f2dot():
    """Re-expanding the Taylor series about t_ref + s: with x = tau - t_ref - s,
    f1dot (x + s)^2 / 2 + f2dot (x + s)^3 / 6 = f2dot x^3 / 6
    + (f1dot + f2dot s) x^2 / 2 + (f1dot s + f2dot s^2 / 2) x + const, so the
    template (f1dot + f2dot s, f2dot) about t_ref + s sees the spectrum of
    (f1dot, f2dot) about t_ref moved up by f1dot s + f2dot s^2 / 2 in
    frequency (closed form; s is chosen to make that a whole number of bins)."""
    ds = synth.small_case(seed=62, n=3000, n_fft=1 << 13, noise=True, f1dot=0.0)
    f1, f2 = 2.0e-10, 1.2e-11
    m = 7
    width = 1.0 / (ds.n_fft * ds.dt)
    # f1 s + f2 s^2 / 2 = m width
    s = (-f1 + math.sqrt(f1 * f1 + 2.0 * f2 * m * width)) / f2
    assert f2 * s * (ds.detectors[0].n * ds.dt) ** 2 > 1.0   # the cubic matters
    row = ds.templates[0].copy()
    row[3], row[4] = f1, f2
    ref = O.oracle_twoF(ds, row[None])[0]
    row2 = row.copy()
    row2[3] = f1 + f2 * s
    ds.t_ref += s
    moved = O.oracle_twoF(ds, row2[None])[0]
    np.testing.assert_allclose(moved[m:], ref[:-m], rtol=1e-8, atol=1e-8)


def test_detector_permutation_and_duplication():
    ds = synth.small_case(seed=28, n=3000, n_fft=1 << 13, ndet=2, noise=True, noise_vars=[0.8, 1.1])
    ref = O.oracle_twoF(ds, ds.templates[:1])[0]
    ds.detectors, ds.x, ds.valid = ds.detectors[::-1], ds.x[::-1], ds.valid[::-1]
    np.testing.assert_allclose(O.oracle_twoF(ds, ds.templates[:1])[0], ref, rtol=1e-10, atol=1e-10)
    one = synth.small_case(seed=28, n=3000, n_fft=1 << 13, ndet=1, noise=True)
    r1 = O.oracle_twoF(one, one.templates[:1])[0]
    one.detectors, one.x, one.valid = one.detectors * 2, one.x * 2, one.valid * 2
    np.testing.assert_allclose(O.oracle_twoF(one, one.templates[:1])[0], 2 * r1, rtol=1e-10)


# --------------------------------------------------------------------------
# Statistics: chi-square with 4 degrees of freedom in Gaussian noise
# --------------------------------------------------------------------------

def _noise_2f(nseed, n=2000, n_fft=1 << 12, ndet=1, gaps=False):
    vals = []
    for s in range(nseed):
        ds = synth.small_case(seed=1000 + s, n=n, n_fft=n_fft, ndet=ndet, rho=0.0, gaps=gaps,
                              noise_vars=[0.8, 1.2][:ndet])
        tf = O.oracle_twoF(ds, ds.templates[:1])[0]
        N = ds.n_fft
        # inner 80% of the band, bins spaced by the padding factor
        step = int(math.ceil(N / n))
        vals.append(tf[N // 2 - int(0.4 * N): N // 2 + int(0.4 * N): step])
    return np.concatenate(vals)


def test_chi2_4dof_in_noise():
    from scipy import stats
    v = _noise_2f(40, ndet=2, gaps=True)
    se = math.sqrt(8.0 / v.size)
    assert abs(v.mean() - 4.0) < 4 * se + 0.03  # interpolation gain <= 1 in the passband
    assert abs(v.var() / 8.0 - 1.0) < 0.05
    assert stats.kstest(v, stats.chi2(4).cdf).pvalue > 1e-4


def test_chi2_survival_reproduces_pilot_false_alarm():
    """The chi2_4 survival at 2F = 70 over the pilot's 9.36e12 values gives the
    printed false-alarm probability; and the oracle's noise tail is chi2_4."""
    from scipy import stats
    g = {}
    for line in open(os.path.join(GOLDEN, "chi2_fap_pilot.txt")):
        if line.strip() and not line.startswith("#"):
            k, val = line.split()
            g[k] = float(val)
    surv = math.exp(-g["threshold"] / 2) * (1 + g["threshold"] / 2)
    assert surv == pytest.approx(stats.chi2(4).sf(g["threshold"]), rel=1e-12)
    fap = -math.expm1(g["n_values"] * math.log1p(-surv))
    assert abs(fap - g["fap"]) < g["fap_tol"]
    v = _noise_2f(20)
    for thr in (8.0, 12.0):
        p_emp = np.mean(v > thr)
        p_th = stats.chi2(4).sf(thr)
        assert abs(p_emp - p_th) < 5 * math.sqrt(p_th / v.size) + 0.004


def test_signal_mean_is_4_plus_rho2():
    """E[2F] at the injection is 4 + rho^2 for the direct sum (non-central chi2_4)."""
    vals = []
    for s in range(60):
        ds = synth.small_case(seed=2000 + s, n=1500, n_fft=1 << 12, rho=6.0, f1dot=0.0)
        inj = ds.injections[0]
        vals.append(O.direct_twoF(ds, O.template_dict(ds.templates[0]), [inj["f"]])[0])
    vals = np.array(vals)
    assert abs(vals.mean() - (4 + 36.0)) < 4 * math.sqrt((8 + 4 * 36.0) / vals.size)


def test_accuracy_metrics_closed_forms():
    """r_1, r_2 and theta of Sec. 4.2 on vectors with known answers."""
    x = np.array([1.0 + 0j, 0.0])
    th = 1e-6
    y = np.array([np.cos(th) + 0j, np.sin(th) + 0j])
    assert abs(O.angle(x, y) - th) < 1e-15
    assert abs(O.angle(x.astype(np.complex64), (1j * x).astype(np.complex64)) - np.pi / 2) < 1e-12
    assert O.rel_err([1.0, 2.0], [1.0, 2.0], 2) == 0.0
    assert abs(O.rel_err([3.0, 0.0], [0.0, 4.0], 1) - 2 * 7.0 / 7.0) < 1e-15
    assert abs(O.rel_err([3.0, 0.0], [0.0, 4.0], 2) - 2 * 5.0 / 7.0) < 1e-15


def test_single_bin_2f_equals_full_transform():
    """2F at one bin from the DFT sum at that bin equals the FFT band's bin
    (two different evaluations of step (vi)), also in a sub-band."""
    ds = synth.small_case(seed=17, n=2000, n_fft=1 << 12, ndet=2, binary=True, gaps=True,
                          ntmpl=1, bin_lo=700, n_bins=1500)
    row = ds.templates[0]
    full = O.oracle_twoF(ds, row[None])[0]
    for i in (0, 3, int(np.argmax(full)), ds.n_bins - 1):
        assert abs(O.twoF_at_bin(ds, row, i) - full[i]) <= 1e-9 * max(1.0, full[i])


# --------------------------------------------------------------------------
# Keplerian (eccentric) orbits
# --------------------------------------------------------------------------

def test_kepler_solution_and_orbit_closed_forms():
    """E solves Kepler's equation; at periapsis (M = 0) and apoapsis (M = pi)
    the delay takes its closed forms asini sin(argp) (1 -+ e); ecc = 0 with an
    argument of periapsis is the circular orbit with tp moved by argp P / 2pi."""
    M = np.linspace(-20.0, 20.0, 4001)
    for e in (0.0, 0.1, 0.5, 0.9):
        E = O.eccentric_anomaly(M, e)
        assert np.abs(E - e * np.sin(E) - M).max() < 1e-13
    P, a, tp, w, e = 0.7 * 86400.0, 0.6, 1234.0, 0.8, 0.35
    tm = dict(asini=a, porb=P, tp=tp, ecc=e, argp=w)
    r = O.binary_delay(tm, np.array([tp, tp + 0.5 * P, tp + 3 * P]))
    np.testing.assert_allclose(r, a * math.sin(w) * np.array([1 - e, -1 - e, 1 - e]),
                               rtol=0, atol=1e-14)
    t = np.linspace(0, 5 * 86400, 1001)
    circ = O.binary_delay(dict(asini=a, porb=P, tp=tp - w * P / (2 * math.pi), ecc=0.0,
                               argp=0.0), t)
    np.testing.assert_allclose(O.binary_delay(dict(tm, ecc=0.0), t), circ, rtol=0, atol=1e-12)
    # ecc = 0 and argp = 0 is the circular form itself
    np.testing.assert_array_equal(O.binary_delay(dict(tm, ecc=0.0, argp=0.0), t),
                                  a * np.sin(2 * math.pi * (t - tp) / P))


@pytest.mark.parametrize("ecc,argp", [(0.3, 1.1), (0.6, -2.0)])
def test_eccentric_noiseless_direct_sum_equals_rho2(ecc, argp):
    """The generator's independent Keplerian timing and the oracle's agree:
    at the injected orbit the direct-sum 2F is rho^2; a wrong element does not."""
    ds = synth.small_case(seed=27, n=5000, n_fft=1 << 14, ndet=2, noise=False, binary=True,
                          keep_f64=True, ecc=ecc, argp=argp)
    inj = ds.injections[0]
    tm = O.template_dict(ds.templates[0])
    assert tm["ecc"] == ecc and tm["argp"] == argp
    v = O.direct_twoF(ds, tm, [inj["f"]])[0]
    assert abs(v / inj["rho2"] - 1) < 1e-10
    off = O.direct_twoF(ds, dict(tm, argp=argp + 0.3), [inj["f"]])[0]
    assert off < 0.9 * inj["rho2"]


def test_eccentric_resampled_matches_direct_sum():
    ds = synth.small_case(seed=28, n=6000, n_fft=1 << 14, ndet=2, noise=False, binary=True,
                          gaps=True, f_inj=0.05, ecc=0.4, argp=0.7)
    inj = ds.injections[0]
    tm = O.template_dict(ds.templates[0])
    tm["df"], ipk = on_bin(ds, inj["f"])
    Fa, Fb = O.fa_fb(ds, tm)
    A, B, C = O.antenna_matrix(ds.ephem_model, ds.detectors, ds.valid, tm["alpha"], tm["delta"],
                               ds.dt)
    tf = O.two_f(Fa, Fb, A, B, C)
    assert int(np.argmax(tf)) == ipk
    assert abs(tf[ipk] / inj["rho2"] - 1.0) < 5e-3
    idx = np.arange(ipk - 30, ipk + 31)
    dFa, dFb = O.direct_fa_fb(ds, tm, ds.bin_frequencies(tm["df"])[idx])
    assert O.rel_err(Fa[idx], dFa, 2) < 3e-3


def test_eccentric_detector_epoch_residual():
    m = synth.EPHEM_MODEL
    det = synth.make_detector("H", 0, 10, 1.0)
    tm = dict(alpha=2.0, delta=0.3, df=0, f1dot=0, f2dot=0, asini=0.8, porb=0.25 * 86400,
              tp=1234.5, ecc=0.5, argp=2.5)
    tau = np.linspace(-600, 20 * 86400, 5001)
    n = O.sky_vector(tm["alpha"], tm["delta"])
    T, _ = O.detector_epochs(m, det, n, tm, tau)
    t_b = tau + O.binary_delay(tm, tau)
    assert np.abs(T + O.roemer_delay(m, det, n, T) - t_b).max() < 1e-9
    rb = O.emission_time_delay(tm, t_b)
    np.testing.assert_allclose(t_b - rb, tau, atol=1e-8)


# --------------------------------------------------------------------------
# Steps (i)-(ii): SFTs to the heterodyned series
# --------------------------------------------------------------------------

def _tone_sfts(freqs, amps, t_sft, n_sft, f_raw, k0, K, t_start):
    """SFTs (time-step normalised DFT bins k0..k0+K-1) of the real strain
    r = 2 Re sum_m A_m exp(2 pi i f_m t), written out here."""
    n = int(t_sft * f_raw)
    out = np.zeros((n_sft, K), dtype=np.complex128)
    for s in range(n_sft):
        t = t_start + s * t_sft + np.arange(n) / f_raw
        r = np.zeros(n)
        for f, a in zip(freqs, amps):
            r += 2.0 * np.real(a * np.exp(2j * np.pi * f * t))
        out[s] = np.fft.rfft(r)[k0:k0 + K] / f_raw
    return out


def test_sft_series_exact_for_on_grid_tones():
    """Tones on the SFT frequency grid inside the band come out as the exact
    heterodyned tones A exp(2 pi i (f - f_h) t); a missing SFT gives zeros."""
    t_sft, K, f_raw, n_sft, t0 = 60.0, 30, 64.0, 5, 1234.0
    kc = 607                      # f_h = 10.1167 Hz: f_h dt is not a whole number
    k0 = kc - K // 2
    freqs = [(k0 + 3) / t_sft, (k0 + 17) / t_sft, (k0 + 29) / t_sft]
    amps = [0.7 - 0.2j, 1.3j, -0.4]
    sfts = _tone_sfts(freqs, amps, t_sft, n_sft, f_raw, k0, K, t0)
    present = np.array([1, 1, 0, 1, 1], dtype=np.uint8)
    x, v, f_h, dt = O.sfts_to_series(sfts, present, k0, t_sft, t0)
    assert f_h == kc / t_sft and dt == 2.0
    t = t0 + dt * np.arange(n_sft * K)
    want = sum(a * np.exp(2j * np.pi * (f - f_h) * t) for f, a in zip(freqs, amps))
    want = want * np.repeat(present, K)
    np.testing.assert_allclose(x, want, rtol=0, atol=1e-10)
    np.testing.assert_array_equal(v, np.repeat(present, K))


def test_sft_series_parseval_and_cw_signal():
    """Per SFT, sum |x_h|^2 = K / t_sft^2 sum |X|^2 (unitary up to the
    normalisation); for a Doppler-modulated CW signal the series matches the
    generator's heterodyned signal away from SFT edges (per-SFT band
    limiting rings only near the edges)."""
    ds, sfts = synth.sft_case(seed=82, noise=False, drop_p=0.0, ndet=1)
    sf = ds.sft
    S, pres = sfts[0]
    x, v, f_h, dt = O.sfts_to_series(S, pres, sf["k0"], sf["t_sft"], sf["t_start"])
    K = sf["K"]
    for s in range(3):
        lhs = np.sum(np.abs(x[s * K:(s + 1) * K]) ** 2)
        rhs = K / sf["t_sft"] ** 2 * np.sum(np.abs(S[s].astype(np.complex128)) ** 2)
        assert abs(lhs / rhs - 1) < 1e-12
    det = ds.detectors[0]
    t = det.t0 + ds.dt * np.arange(det.n)
    inj = ds.injections[0]
    ref = synth.signal_series(ds.ephem_model, det, t, inj, ds.f_het, 0.0) * inj["h0"]
    j = np.arange(det.n) % K
    mid = (j > K // 3) & (j < 2 * K // 3)
    assert np.abs(x - ref)[mid].max() < 1e-2 * np.abs(ref).max()
    assert np.abs(x - ref).max() > 3e-2 * np.abs(ref).max()   # the edges ring


def test_sft_pipeline_recovers_rho2_and_chi2_noise():
    """Steps (i)-(vii) from SFTs: noiseless, 2F at the injection is rho^2
    within the per-SFT edge loss; in noise alone the mean of 2F is 4 (the
    series' noise normalisation E|n|^2 = 1)."""
    ds, sfts = synth.sft_case(seed=83, noise=False, drop_p=0.1, ndet=2, rho=20.0)
    sf = ds.sft
    xs, vs = [], []
    for S, pres in sfts:
        x, v, _, _ = O.sfts_to_series(S, pres, sf["k0"], sf["t_sft"], sf["t_start"])
        xs.append(x)
        vs.append(v)
    ds.x, ds.valid = xs, vs
    inj = ds.injections[0]
    tm = O.template_dict(ds.templates[0])
    tm["df"], ipk = on_bin(ds, inj["f"])
    Fa, Fb = O.fa_fb(ds, tm)
    A, B, C = O.antenna_matrix(ds.ephem_model, ds.detectors, ds.valid, tm["alpha"], tm["delta"],
                               ds.dt)
    tf = O.two_f(Fa, Fb, A, B, C)
    # rho^2 was set with every SFT present; the dropped ones remove their share
    kept = np.mean([v.mean() for v in vs])
    assert int(np.argmax(tf)) == ipk
    assert 0.9 * kept * inj["rho2"] < tf[ipk] < 1.02 * inj["rho2"]
    dn, sn = synth.sft_case(seed=84, noise=True, drop_p=0.1, ndet=1, rho=0.0)
    S, pres = sn[0]
    x, v, _, _ = O.sfts_to_series(S, pres, dn.sft["k0"], dn.sft["t_sft"], dn.sft["t_start"])
    dn.x, dn.valid = [x], [v]
    var = np.mean(np.abs(x[v == 1]) ** 2)
    assert abs(var - 1.0) < 0.05
    tf = O.oracle_twoF(dn, dn.templates[:1])[0]
    inner = tf[dn.n_fft // 10: -dn.n_fft // 10]
    assert abs(inner.mean() - 4.0) < 0.15
