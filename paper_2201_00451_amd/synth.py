"""Seeded synthetic inputs for the resampling F-statistic.

This module builds the *inputs* of the method and nothing else: a synthetic
solar-system ephemeris (circular Earth orbit plus sidereal rotation), detector
sites, heterodyned and downsampled complex strain series with Gaussian noise,
SFT-like gaps and injected continuous-wave signals, template banks, and the
tabulated detector trajectory that the GPU path reads.  It holds none of the
F-statistic arithmetic (no resampling, no antenna-pattern closed form, no FFT,
no 2F); both the GPU path and the FP64 oracle consume what it produces.

The signal model follows the phase model of Sec. 2 (eq. for Phi(t)): the phase
at the source is phi0 + 2 pi f (t_src - t_ref) + Phi_s(t_src), with Phi_s a
Taylor series in the frequency derivatives; the arrival time at the detector
includes the Roemer delay of the detector position projected on the sky
direction and, for binaries, the circular-orbit Roemer delay of the source.
The detector response is computed by the tensor route (detector tensor
contracted with the plus/cross polarisation tensors), which is independent of
the closed-form a(t), b(t) used by the method.

Every random draw comes from ``numpy.random.default_rng(SeedSequence(seed))``
spawned per purpose, so the same seed reproduces the same dataset.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299792458.0
DAY = 86400.0

# Synthetic ephemeris: a circular 1 AU Earth orbit with a 365.25 d period in
# the ecliptic (obliquity 23.44 deg) plus rotation of a spherical Earth at the
# sidereal rate.  Orbital phase and Greenwich sidereal angle are zero at t = 0.
EPHEM_MODEL = {
    "r_orbit_s": 499.004784,          # 1 AU in light-seconds
    "period_orbit_s": 365.25 * DAY,
    "obliquity_rad": math.radians(23.44),
    "orbit_phase0_rad": 0.0,
    "r_earth_s": 6.371e6 / C_LIGHT,   # Earth radius in light-seconds
    "sidereal_rate_rad_s": 2.0 * math.pi / 86164.0905,
    "sidereal_angle0_rad": 0.0,
}

# Detector sites: geocentric latitude, east longitude and arm azimuths measured
# counter-clockwise from local East, all in degrees; 90 deg opening angle.
SITES = {
    "H": dict(lat=46.45, lon=-119.41, az_x=125.9, az_y=215.9),
    "L": dict(lat=30.56, lon=-90.77, az_x=197.7, az_y=287.7),
}

# Template parameter order used everywhere: one row of 8 float64 per template.
TEMPLATE_FIELDS = ("alpha", "delta", "df", "f1dot", "f2dot", "asini", "porb", "tp")


@dataclass
class Detector:
    name: str
    lat: float        # rad
    lon: float        # rad
    az_x: float       # rad, CCW from East
    az_y: float       # rad, CCW from East
    t0: float         # s, time of sample 0
    n: int            # number of samples
    noise_var: float  # E|n|^2 of the complex noise


@dataclass
class Dataset:
    """Everything one search needs.  Arrays are host numpy arrays."""
    name: str
    dt: float
    f_het: float
    t_ref: float
    tau0: float
    n_fft: int
    sinc_halfwidth: int
    bin_lo: int
    n_bins: int
    detectors: list
    x: list                      # complex64 [n] per detector (zero in gaps)
    valid: list                  # uint8 [n] per detector
    templates: np.ndarray        # float64 [ntmpl, 8]
    ephem_model: dict = field(default_factory=lambda: dict(EPHEM_MODEL))
    eph_tables: list = None      # float64 [n_eph, 6] per detector: pos (ls), vel (ls/s)
    eph_t0: float = 0.0
    eph_dt: float = 60.0
    injections: list = field(default_factory=list)
    max_delay: float = 0.0       # bound on |t_src - t| over all templates (s)

    @property
    def ndet(self):
        return len(self.detectors)

    @property
    def ntmpl(self):
        return int(self.templates.shape[0])

    def bin_frequencies(self, df=0.0):
        i = np.arange(self.bin_lo, self.bin_lo + self.n_bins)
        return self.f_het + df + (i - self.n_fft // 2) / (self.n_fft * self.dt)


def make_detector(site, t0, n, noise_var, name=None):
    s = SITES[site] if isinstance(site, str) else site
    return Detector(name or (site if isinstance(site, str) else "X"),
                    math.radians(s["lat"]), math.radians(s["lon"]),
                    math.radians(s["az_x"]), math.radians(s["az_y"]),
                    float(t0), int(n), float(noise_var))


# ----------------------------------------------------------------------------
# Ephemeris: detector position and velocity in the equatorial SSB frame.
# ----------------------------------------------------------------------------

def detector_pos_vel(model, det, t):
    """Position (light-s) and velocity (light-s per s) of a detector, shape (3, n)."""
    t = np.asarray(t, dtype=np.float64)
    w_orb = 2.0 * math.pi / model["period_orbit_s"]
    th = model["orbit_phase0_rad"] + w_orb * t
    eps = model["obliquity_rad"]
    ro = model["r_orbit_s"]
    pos = np.empty((3,) + t.shape)
    vel = np.empty((3,) + t.shape)
    c_th, s_th = np.cos(th), np.sin(th)
    pos[0] = ro * c_th
    pos[1] = ro * s_th * math.cos(eps)
    pos[2] = ro * s_th * math.sin(eps)
    vel[0] = -ro * w_orb * s_th
    vel[1] = ro * w_orb * c_th * math.cos(eps)
    vel[2] = ro * w_orb * c_th * math.sin(eps)
    w_sid = model["sidereal_rate_rad_s"]
    phi = det.lon + model["sidereal_angle0_rad"] + w_sid * t
    re = model["r_earth_s"]
    c_l, s_l = math.cos(det.lat), math.sin(det.lat)
    c_p, s_p = np.cos(phi), np.sin(phi)
    pos[0] += re * c_l * c_p
    pos[1] += re * c_l * s_p
    pos[2] += re * s_l
    vel[0] += -re * c_l * w_sid * s_p
    vel[1] += re * c_l * w_sid * c_p
    return pos, vel


def ephemeris_table(model, det, t_start, t_end, spacing=60.0):
    """Tabulate position and velocity at uniform spacing covering [t_start, t_end]."""
    t0 = math.floor(t_start / spacing) * spacing
    n = int(math.ceil((t_end - t0) / spacing)) + 2
    t = t0 + spacing * np.arange(n)
    pos, vel = detector_pos_vel(model, det, t)
    tab = np.ascontiguousarray(np.concatenate([pos, vel], axis=0).T)
    return tab, float(t0), float(spacing)


# ----------------------------------------------------------------------------
# Signal synthesis (tensor-route response, forward timing model).
# ----------------------------------------------------------------------------

def sky_unit(alpha, delta):
    return np.array([math.cos(delta) * math.cos(alpha),
                     math.cos(delta) * math.sin(alpha),
                     math.sin(delta)])


def tensor_response(model, det, alpha, delta, psi, t):
    """F+ and Fx from the detector tensor and the polarisation tensors."""
    t = np.asarray(t, dtype=np.float64)
    nhat = sky_unit(alpha, delta)
    p0 = np.array([math.sin(alpha), -math.cos(alpha), 0.0])
    q0 = np.cross(nhat, p0)
    p = p0 * math.cos(psi) + q0 * math.sin(psi)
    q = -p0 * math.sin(psi) + q0 * math.cos(psi)
    eplus = np.outer(p, p) - np.outer(q, q)
    ecross = np.outer(p, q) + np.outer(q, p)
    phi = det.lon + model["sidereal_angle0_rad"] + model["sidereal_rate_rad_s"] * t
    c_p, s_p = np.cos(phi), np.sin(phi)
    c_l, s_l = math.cos(det.lat), math.sin(det.lat)
    east = np.stack([-s_p, c_p, np.zeros_like(t)])
    north = np.stack([-s_l * c_p, -s_l * s_p, np.full_like(t, c_l)])

    def arm(az):
        return math.cos(az) * east + math.sin(az) * north

    u, v = arm(det.az_x), arm(det.az_y)
    fp = 0.5 * (np.einsum("in,ij,jn->n", u, eplus, u) - np.einsum("in,ij,jn->n", v, eplus, v))
    fx = 0.5 * (np.einsum("in,ij,jn->n", u, ecross, u) - np.einsum("in,ij,jn->n", v, ecross, v))
    return fp, fx


def orbit_delay(t_src, asini, porb, tp, ecc=0.0, argp=0.0):
    """Roemer delay of the source in its orbit and its time derivative.
    Keplerian elements: tp is the time of periapsis (of the ascending node
    for a circular orbit, argp = 0).  The eccentric anomaly comes from a
    Halley iteration on E - ecc sin E = mean anomaly (then the delay is
    asini (sin argp (cos E - ecc) + cos argp sqrt(1 - ecc^2) sin E))."""
    om = 2.0 * math.pi / porb
    M = om * (np.asarray(t_src, dtype=np.float64) - tp)
    if ecc == 0.0:
        s_, c_ = np.sin(M + argp), np.cos(M + argp)
        return asini * s_, asini * om * c_
    E = M.copy()
    for _ in range(12):
        f0 = E - ecc * np.sin(E) - M
        f1 = 1.0 - ecc * np.cos(E)
        f2 = ecc * np.sin(E)
        E = E - 2.0 * f0 * f1 / (2.0 * f1 * f1 - f0 * f2)
    sq = math.sqrt(1.0 - ecc * ecc)
    r = asini * (math.sin(argp) * (np.cos(E) - ecc) + math.cos(argp) * sq * np.sin(E))
    dr_dE = asini * (-math.sin(argp) * np.sin(E) + math.cos(argp) * sq * np.cos(E))
    return r, dr_dE * om / (1.0 - ecc * np.cos(E))


def source_emission_time(t_b, asini, porb, tp, ecc=0.0, argp=0.0):
    """Solve t_src + R(t_src) = t_b by Newton steps."""
    t_b = np.asarray(t_b, dtype=np.float64)
    if asini == 0.0:
        return t_b.copy()
    ts = t_b - orbit_delay(t_b, asini, porb, tp, ecc, argp)[0]
    for _ in range(8):
        r, dr = orbit_delay(ts, asini, porb, tp, ecc, argp)
        ts = ts - (ts + r - t_b) / (1.0 + dr)
    return ts


def signal_series(model, det, t, inj, f_het, t_ref):
    """Complex heterodyned signal at detector sample times t (no noise)."""
    nhat = sky_unit(inj["alpha"], inj["delta"])
    pos, _ = detector_pos_vel(model, det, t)
    roemer = nhat @ pos
    t_b = t + roemer
    orbit = (inj.get("asini", 0.0), inj.get("porb", 1.0), inj.get("tp", 0.0),
             inj.get("ecc", 0.0), inj.get("argp", 0.0))
    t_src = source_emission_time(t_b, *orbit)
    # delay t_src - t formed from small numbers
    if orbit[0] != 0.0:
        delay = roemer - orbit_delay(t_src, *orbit)[0]
    else:
        delay = roemer
    tau = t_src - t_ref
    cyc_spin = inj.get("f1dot", 0.0) * tau ** 2 / 2.0 + inj.get("f2dot", 0.0) * tau ** 3 / 6.0
    cyc = ((inj["f"] - f_het) * tau) % 1.0 + (f_het * delay) % 1.0 + cyc_spin % 1.0 \
        - (f_het * t_ref) % 1.0
    phase = inj["phi0"] + 2.0 * math.pi * (cyc % 1.0)
    fp, fx = tensor_response(model, det, inj["alpha"], inj["delta"], inj["psi"], t)
    cosi = inj["cosi"]
    ap = 0.5 * (1.0 + cosi * cosi)
    ax = cosi
    return (fp * ap - 1j * fx * ax) * np.exp(1j * phase)


def make_data(detectors, dt, f_het, t_ref, injections, rng_seed, model=None, gaps=None,
              noise=True, keep_f64=False):
    """Noise + injected signals.  Each injection's h0 is set for its target rho.

    rho^2 = 2 sum_X sum_j v_j |s_j|^2 / sigma_X^2 is the optimal signal-to-noise
    of the noiseless signal; h0 scales s linearly, so one evaluation fixes it.
    """
    model = model or EPHEM_MODEL
    ss = np.random.SeedSequence(rng_seed)
    noise_seeds = ss.spawn(len(detectors))
    xs, valids = [], []
    sigs = [[None] * len(injections) for _ in detectors]
    for xi, det in enumerate(detectors):
        t = det.t0 + dt * np.arange(det.n)
        v = np.ones(det.n, dtype=np.uint8) if gaps is None else gaps[xi]
        valids.append(v)
        for ii, inj in enumerate(injections):
            sigs[xi][ii] = signal_series(model, det, t, inj, f_het, t_ref)
    for ii, inj in enumerate(injections):
        rho2 = 0.0
        for xi, det in enumerate(detectors):
            rho2 += 2.0 * np.sum(valids[xi] * np.abs(sigs[xi][ii]) ** 2) / det.noise_var
        scale = inj["rho"] / math.sqrt(rho2)
        inj["h0"] = scale
        inj["rho2"] = inj["rho"] ** 2
        for xi in range(len(detectors)):
            sigs[xi][ii] = sigs[xi][ii] * scale
    for xi, det in enumerate(detectors):
        s = np.zeros(det.n, dtype=np.complex128)
        for ii in range(len(injections)):
            s += sigs[xi][ii]
        if noise:
            rng = np.random.default_rng(noise_seeds[xi])
            sd = math.sqrt(det.noise_var / 2.0)
            s = s + sd * (rng.standard_normal(det.n) + 1j * rng.standard_normal(det.n))
        xs.append((s * valids[xi]).astype(np.complex128 if keep_f64 else np.complex64))
    return xs, valids


def random_gaps(rng, n, dt, ngaps, gap_s):
    """n-sample validity mask with ngaps non-overlapping gaps of gap_s seconds."""
    v = np.ones(n, dtype=np.uint8)
    glen = int(round(gap_s / dt))
    placed = []
    while len(placed) < ngaps:
        s = int(rng.integers(0, n - glen))
        if all(s + glen <= p or s >= p + glen for p in placed):
            placed.append(s)
            v[s:s + glen] = 0
    return v


def duty_gaps(rng, n, dt, block_s, drop_p):
    """Drop each block_s-second block independently with probability drop_p."""
    v = np.ones(n, dtype=np.uint8)
    blen = int(round(block_s / dt))
    for s in range(0, n, blen):
        if rng.random() < drop_p:
            v[s:s + blen] = 0
    return v


def finish(ds, model=None, spacing=60.0):
    """Attach ephemeris tables and the delay bound."""
    model = model or ds.ephem_model
    # cover every sample and the whole source-frame grid, widened by the delays
    t_lo = min(min(d.t0 for d in ds.detectors), ds.tau0) - 2000.0
    t_hi = max(max(d.t0 + d.n * ds.dt for d in ds.detectors),
               ds.tau0 + ds.n_fft * ds.dt) + 2000.0
    tabs = []
    for d in ds.detectors:
        tab, t0, sp = ephemeris_table(model, d, t_lo, t_hi, spacing)
        tabs.append(tab)
    ds.eph_tables, ds.eph_t0, ds.eph_dt = tabs, t0, sp
    amax = float(np.max(ds.templates[:, 5])) if ds.ntmpl else 0.0
    ds.max_delay = model["r_orbit_s"] + model["r_earth_s"] + amax + 1.0
    return ds


def grid_origin(t0, dt, max_delay):
    """Source-frame grid start: t0 minus a whole number of samples covering the delay."""
    return t0 - math.ceil(max_delay / dt) * dt


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def config_tiny(seed=1, n=43200, dt=2.0, n_fft=1 << 17, rho=20.0, D=8, noise=True):
    """One detector, 1 day at 2 s, f_het 100 Hz; 11 spin-down templates."""
    det = make_detector("H", 0.0, n, 1.0)
    inj = dict(alpha=1.0, delta=-0.5, f=100.2, f1dot=-1e-10, cosi=0.3, psi=0.4, phi0=1.0,
               rho=rho)
    xs, vs = make_data([det], dt, 100.0, 0.0, [inj], seed, noise=noise)
    tm = np.zeros((11, 8))
    tm[:, 0], tm[:, 1] = 1.0, -0.5
    tm[:, 3] = -5e-10 + 1e-10 * np.arange(11)
    tm[:, 6] = 1.0
    tau0 = -512.0 if dt == 2.0 else grid_origin(0.0, dt, 512.0)
    ds = Dataset("tiny", dt, 100.0, 0.0, tau0, n_fft, D, 0, n_fft, [det], xs, vs, tm,
                 injections=[inj])
    return finish(ds)


def config_sky_spindown(seed=2, ndays=10.0, dt=1.0, n_fft=1 << 21, nsky=10, nf1=10,
                        f_het=150.0, D=8, ninj=3, noise=True):
    """Two detectors, 10 d at 1 s around 150 Hz, ten 1800 s gaps each,
    noise variance U(0.8, 1.2); 3 injections; 10x10 sky patch x 10 spin-downs."""
    ss = np.random.SeedSequence(seed)
    s_det, s_inj, s_gap = ss.spawn(3)
    rng_det = np.random.default_rng(s_det)
    n = int(round(ndays * DAY / dt))
    dets = [make_detector("H", 0.0, n, rng_det.uniform(0.8, 1.2)),
            make_detector("L", 0.0, n, rng_det.uniform(0.8, 1.2))]
    rng_gap = np.random.default_rng(s_gap)
    gaps = [random_gaps(rng_gap, n, dt, 10, 1800.0) for _ in dets]
    sky_a = 1.0 + 0.01 * (np.arange(nsky) - (nsky - 1) / 2.0)
    sky_d = -0.5 + 0.01 * (np.arange(nsky) - (nsky - 1) / 2.0)
    f1 = 1e-10 * (np.arange(nf1) - (nf1 - 1) / 2.0)
    rng = np.random.default_rng(s_inj)
    injs = []
    for _ in range(ninj):
        injs.append(dict(alpha=float(rng.choice(sky_a)), delta=float(rng.choice(sky_d)),
                         f=float(rng.uniform(f_het - 0.4, f_het + 0.4)),
                         f1dot=float(rng.choice(f1)), cosi=float(rng.uniform(-1, 1)),
                         psi=float(rng.uniform(-math.pi / 4, math.pi / 4)),
                         phi0=float(rng.uniform(0, 2 * math.pi)), rho=float(rng.uniform(8, 30))))
    xs, vs = make_data(dets, dt, f_het, 0.0, injs, seed, gaps=gaps, noise=noise)
    A, Dd, F = np.meshgrid(sky_a, sky_d, f1, indexing="ij")
    tm = np.zeros((A.size, 8))
    tm[:, 0], tm[:, 1], tm[:, 3] = A.ravel(), Dd.ravel(), F.ravel()
    tm[:, 6] = 1.0
    ds = Dataset("sky_spindown", dt, f_het, 0.0, grid_origin(0.0, dt, 512.0), n_fft, D, 0,
                 n_fft, dets, xs, vs, tm, injections=injs)
    return finish(ds)


def binary_lattice(f, asini, porb, tp, tspan, shape=(22, 22, 21), mu=0.1 / 3.0, limit=None):
    """Lattice in (asini, porb, tp) from the diagonal circular-orbit phase metric."""
    om = 2.0 * math.pi / porb
    d_a = math.sqrt(2 * mu) / (2 * math.pi * f)
    d_tp = math.sqrt(2 * mu) / (2 * math.pi * f * asini * om)
    d_om = math.sqrt(24 * mu) / (2 * math.pi * f * asini * tspan)
    ia = np.arange(shape[0]) - (shape[0] - 1) / 2.0
    io = np.arange(shape[1]) - (shape[1] - 1) / 2.0
    it = np.arange(shape[2]) - (shape[2] - 1) / 2.0
    A, O, T = np.meshgrid(asini + d_a * ia, om + d_om * io, tp + d_tp * it, indexing="ij")
    out = np.stack([A.ravel(), 2 * math.pi / O.ravel(), T.ravel()], axis=1)
    return out if limit is None else out[:limit]


def config_binary(seed=3, ndays=120.0, dt=2.0, n_fft=1 << 23, ntmpl=10000, D=8, noise=True,
                  shape=(22, 22, 21)):
    """Two detectors, 120 d at 2 s, 70% duty in 1800 s blocks, band centre
    U(200, 600) Hz, one circular binary injection at rho 20, lattice templates."""
    ss = np.random.SeedSequence(seed)
    s_par, s_gap = ss.spawn(2)
    rng = np.random.default_rng(s_par)
    n = int(round(ndays * DAY / dt))
    f_het = float(rng.uniform(200.0, 600.0))
    dets = [make_detector("H", 0.0, n, 1.0), make_detector("L", 0.0, n, 1.0)]
    rng_gap = np.random.default_rng(s_gap)
    gaps = [duty_gaps(rng_gap, n, dt, 1800.0, 0.3) for _ in dets]
    alpha, delta = 3.52004, -0.828935
    asini = float(rng.uniform(0.01, 1.0))
    porb = float(rng.uniform(0.1, 2.0)) * DAY
    tp = float(rng.uniform(0.0, porb))
    f = f_het + float(rng.uniform(-0.15, 0.15))
    inj = dict(alpha=alpha, delta=delta, f=f, f1dot=0.0, cosi=float(rng.uniform(-1, 1)),
               psi=float(rng.uniform(-math.pi / 4, math.pi / 4)),
               phi0=float(rng.uniform(0, 2 * math.pi)), rho=20.0, asini=asini, porb=porb, tp=tp)
    xs, vs = make_data(dets, dt, f_het, 0.0, [inj], seed, gaps=gaps, noise=noise)
    lat = binary_lattice(f, asini, porb, tp, n * dt, shape=shape, limit=ntmpl)
    tm = np.zeros((lat.shape[0], 8))
    tm[:, 0], tm[:, 1] = alpha, delta
    tm[:, 5:8] = lat
    max_a = float(np.max(lat[:, 0]))
    ds = Dataset("binary", dt, f_het, 0.0, grid_origin(0.0, dt, 512.0 + max_a), n_fft, D, 0,
                 n_fft, dets, xs, vs, tm, injections=[inj])
    return finish(ds)


def config_refine(seed=5, ndays=30.0, dt=1.0, n_fft=1 << 22, f_het=400.0, band=0.2, ninj=8,
                  per_inj=8, D=8, noise=True, mu=0.1 / 3.0):
    """Candidate refinement: two detectors, 30 d at 1 s around 400 Hz, output
    band 0.2 Hz; ninj circular-binary injections (rho U(10, 40), asini
    U(0.005, 0.05) ls, porb U(0.5, 2) d) at frequencies 0.025 Hz apart, and
    per injection per_inj candidates displaced 0.3-1 metric spacing (mismatch
    mu per axis) in a random direction of (f, asini, porb, tp).  The dataset's
    templates are the candidates; ds.cand_bins holds each candidate's bin in
    the band and ds.cand_inj its injection."""
    ss = np.random.SeedSequence(seed)
    s_par, s_cand = ss.spawn(2)
    rng = np.random.default_rng(s_par)
    n = int(round(ndays * DAY / dt))
    dets = [make_detector("H", 0.0, n, 1.0), make_detector("L", 0.0, n, 1.0)]
    alpha, delta = 3.52004, -0.828935
    injs = []
    for i in range(ninj):
        porb = float(rng.uniform(0.5, 2.0)) * DAY
        injs.append(dict(alpha=alpha, delta=delta,
                         f=f_het + 0.025 * (i - (ninj - 1) / 2.0) + float(rng.uniform(-2e-3, 2e-3)),
                         f1dot=0.0, cosi=float(rng.uniform(-1, 1)),
                         psi=float(rng.uniform(-math.pi / 4, math.pi / 4)),
                         phi0=float(rng.uniform(0, 2 * math.pi)), rho=float(rng.uniform(10, 40)),
                         asini=float(rng.uniform(0.005, 0.05)), porb=porb,
                         tp=float(rng.uniform(0.0, porb))))
    xs, vs = make_data(dets, dt, f_het, 0.0, injs, seed, noise=noise)
    tspan = n * dt
    n_bins = int(round(band * n_fft * dt))
    bin_lo = n_fft // 2 - n_bins // 2
    rc = np.random.default_rng(s_cand)
    rows, bins, which = [], [], []
    for i, inj in enumerate(injs):
        om = 2.0 * math.pi / inj["porb"]
        d_f = math.sqrt(3.0 * mu) / (math.pi * tspan)
        d_a = math.sqrt(2 * mu) / (2 * math.pi * inj["f"])
        d_tp = math.sqrt(2 * mu) / (2 * math.pi * inj["f"] * inj["asini"] * om)
        d_om = math.sqrt(24 * mu) / (2 * math.pi * inj["f"] * inj["asini"] * tspan)
        for _ in range(per_inj):
            u = rc.normal(size=4)
            u *= rc.uniform(0.3, 1.0) / np.linalg.norm(u)
            fc = inj["f"] + u[0] * d_f
            m = int(round((fc - f_het) * n_fft * dt)) + n_fft // 2
            r = np.zeros(8)
            r[0], r[1] = alpha, delta
            r[2] = (fc - f_het) - (m - n_fft // 2) / (n_fft * dt)
            r[5] = inj["asini"] + u[1] * d_a
            r[6] = 2.0 * math.pi / (om + u[2] * d_om)
            r[7] = inj["tp"] + u[3] * d_tp
            rows.append(r)
            bins.append(m - bin_lo)
            which.append(i)
    tm = np.array(rows)
    max_a = float(np.max(tm[:, 5]))
    ds = Dataset("refine", dt, f_het, 0.0, grid_origin(0.0, dt, 512.0 + max_a), n_fft, D, bin_lo,
                 n_bins, dets, xs, vs, tm, injections=injs)
    ds.cand_bins = np.array(bins, dtype=np.int64)
    ds.cand_inj = np.array(which, dtype=np.int64)
    return finish(ds)


def small_case(seed=11, n=6000, dt=2.0, n_fft=1 << 14, ndet=1, f_het=100.0, ntmpl=4, D=8,
               rho=15.0, noise=True, binary=False, gaps=False, noise_vars=None, f_inj=None,
               bin_lo=0, n_bins=None, keep_f64=False, model=None, sites=None, f1dot=None,
               t0=0.0, noise_seed=None, f2dot=0.0, ecc=None, argp=None, eph_spacing=60.0):
    """Small search (a few hours of data) for oracle pins and quick parity.

    t0 shifts the data (and the computed grid) in time with the reference time
    kept at 0, so that cases with the same seed and different t0 are segments
    of one source; noise_seed (default: seed) draws their noise independently.
    f2dot is the injection's second frequency derivative (the templates carry
    it too).  ecc and argp (binary only) make the orbit Keplerian; the
    templates then have ten columns (eccentricity and argument of periapsis
    last).  eph_spacing is the tabulated trajectory's time step (coarse grids
    need a coarser table: a resampling tile stages a bounded number of its
    nodes)."""
    ss = np.random.SeedSequence(seed)
    s_par, s_gap = ss.spawn(2)
    rng = np.random.default_rng(s_par)
    sites = sites or ["H", "L", "H", "L"][:ndet]
    nv = noise_vars or [1.0] * ndet
    dets = [make_detector(s, t0, n, v, name=f"{s}{i}") for i, (s, v) in enumerate(zip(sites, nv))]
    band = 0.5 / dt
    inj = dict(alpha=float(rng.uniform(0, 2 * math.pi)), delta=float(rng.uniform(-1.2, 1.2)),
               f=f_het + (f_inj if f_inj is not None else float(rng.uniform(-0.6, 0.6) * band)),
               f1dot=float(rng.uniform(-2e-9, 2e-9)) if f1dot is None else f1dot,
               cosi=float(rng.uniform(-1, 1)),
               psi=float(rng.uniform(-0.7, 0.7)), phi0=float(rng.uniform(0, 6.28)), rho=rho,
               f2dot=float(f2dot))
    if binary:
        inj.update(asini=float(rng.uniform(0.05, 0.5)), porb=float(rng.uniform(0.2, 1.0)) * DAY,
                   tp=float(rng.uniform(0, 1e4)))
    kepler = binary and (ecc is not None or argp is not None)
    if kepler:
        inj.update(ecc=float(ecc or 0.0), argp=float(argp or 0.0))
    g = None
    if gaps:
        rg = np.random.default_rng(s_gap)
        g = [random_gaps(rg, n, dt, 2, 600.0) for _ in dets]
    model = dict(model or EPHEM_MODEL)
    xs, vs = make_data(dets, dt, f_het, 0.0, [inj], seed if noise_seed is None else noise_seed,
                       gaps=g, noise=noise, keep_f64=keep_f64, model=model)
    tm = np.zeros((ntmpl, 10 if kepler else 8))
    tm[:, 0] = inj["alpha"] + 0.02 * np.arange(ntmpl)
    tm[:, 1] = inj["delta"]
    tm[:, 3] = inj["f1dot"]
    tm[:, 4] = inj["f2dot"]
    tm[:, 6] = 1.0
    if binary:
        tm[:, 5], tm[:, 6], tm[:, 7] = inj["asini"], inj["porb"], inj["tp"]
    if kepler:
        tm[:, 8], tm[:, 9] = inj["ecc"], inj["argp"]
    margin = 512.0 + (inj.get("asini", 0.0) if binary else 0.0)
    nb = n_fft if n_bins is None else n_bins
    ds = Dataset("small", dt, f_het, 0.0, grid_origin(t0, dt, margin), n_fft, D, bin_lo, nb,
                 dets, xs, vs, tm, ephem_model=model, injections=[inj])
    return finish(ds, spacing=eph_spacing)


def config_uneven(seed=4, n_search=256, days=(1.0, 30.0), dts=(0.5, 1.0, 2.0, 5.0),
                  max_log_n=22, ntmpl=(8, 64), f_het=(50.0, 1000.0), D=8, noise=True,
                  pick=None):
    """Independent searches of uneven shape for batched serving: per search a
    span log-uniform in `days`, dt from `dts`, one or two detectors, a
    heterodyne frequency uniform in `f_het`, n_fft the power of two >= twice
    the samples (span and dt redrawn while n_fft > 2^max_log_n), full band,
    one injection (rho U(10, 30)) and a template count uniform in `ntmpl`:
    even searches a spin-down grid at the injection's sky position, odd ones
    a circular-binary lattice around the injection's orbit.  Returns a list of
    Datasets; with ``pick`` (indices) only those searches are built, the same
    as in the full list (every search's parameters are still drawn in order
    and its data has a seed of its own)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    out = []
    for k in range(n_search):
        while True:
            span = math.exp(rng.uniform(math.log(days[0]), math.log(days[1]))) * DAY
            dt = float(rng.choice(dts))
            n = int(round(span / dt))
            n_fft = 1 << max(12, int(math.ceil(math.log2(2 * n))))
            if n_fft <= (1 << max_log_n):
                break
        ndet = int(rng.integers(1, 3))
        fh = float(rng.uniform(*f_het))
        nt = int(rng.integers(ntmpl[0], ntmpl[1] + 1))
        binary = k % 2 == 1
        dets = [make_detector(site, 0.0, n, float(rng.uniform(0.8, 1.2)))
                for site in ("H", "L")[:ndet]]
        inj = dict(alpha=float(rng.uniform(0, 2 * math.pi)), delta=float(rng.uniform(-1.2, 1.2)),
                   f=fh + float(rng.uniform(-0.3, 0.3)) * 0.5 / dt, f1dot=0.0,
                   cosi=float(rng.uniform(-1, 1)), psi=float(rng.uniform(-0.7, 0.7)),
                   phi0=float(rng.uniform(0, 2 * math.pi)), rho=float(rng.uniform(10, 30)))
        tm = np.zeros((nt, 8))
        tm[:, 0], tm[:, 1] = inj["alpha"], inj["delta"]
        max_a = 0.0
        if binary:
            inj.update(asini=float(rng.uniform(0.01, 0.2)),
                       porb=float(rng.uniform(0.5, 2.0)) * DAY, tp=float(rng.uniform(0, 1e4)))
            side = int(math.ceil(nt ** (1.0 / 3.0)))
            lat = binary_lattice(inj["f"], inj["asini"], inj["porb"], inj["tp"], n * dt,
                                 shape=(side, side, side), limit=nt)
            tm[:, 5:8] = lat
            max_a = float(np.max(lat[:, 0]))
        else:
            inj["f1dot"] = float(rng.uniform(-1e-10, 1e-10))
            tm[:, 3] = inj["f1dot"] + 2e-11 * (np.arange(nt) - (nt - 1) / 2.0)
            tm[:, 6] = 1.0
        if pick is not None and k not in pick:
            continue
        xs, vs = make_data(dets, dt, fh, 0.0, [inj], seed * 1000 + k, noise=noise)
        ds = Dataset(f"uneven{k}", dt, fh, 0.0, grid_origin(0.0, dt, 512.0 + max_a), n_fft, D, 0,
                     n_fft, dets, xs, vs, tm, injections=[inj])
        out.append(finish(ds))
    return out


def make_sfts(det, t_start, t_sft, n_sft, f_raw, k0, K, injections, f_het, t_ref, seed,
              drop_p=0.0, noise_var=1.0, model=None, noise=True):
    """Short Fourier transforms of a real detector strain, the input of steps
    (i)-(ii): the strain r(t) = 2 Re[s(t) exp(2 pi i f_het t)] + real white
    noise sampled at f_raw over n_sft contiguous t_sft-second segments, where
    s is the complex heterodyned signal of the injections (their h0 already
    set); each segment's DFT with the time-step normalisation
    X[k] = (1/f_raw) sum_n r_n exp(-2 pi i k n / N) keeps bins k0 .. k0+K-1.
    Segments are dropped independently with probability drop_p.  The noise
    variance is set so that the heterodyned series has E|n|^2 = noise_var.
    Returns (sfts complex64 [n_sft, K], present uint8 [n_sft])."""
    model = model or EPHEM_MODEL
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    s_noise, s_drop = ss.spawn(2)
    rng_n = np.random.default_rng(s_noise)
    present = (np.random.default_rng(s_drop).random(n_sft) >= drop_p).astype(np.uint8)
    n_seg = int(round(t_sft * f_raw))
    sd = math.sqrt(noise_var * f_raw * t_sft / K)
    out = np.zeros((n_sft, K), dtype=np.complex64)
    for s_ in range(n_sft):
        t = t_start + s_ * t_sft + np.arange(n_seg) / f_raw
        r = np.zeros(n_seg)
        for inj in injections:
            sig = signal_series(model, det, t, inj, f_het, t_ref) * inj["h0"]
            r += 2.0 * np.real(sig * np.exp(2j * np.pi * np.mod(f_het * t, 1.0)))
        if noise:
            r += sd * rng_n.standard_normal(n_seg)
        if present[s_]:
            out[s_] = (np.fft.rfft(r)[k0:k0 + K] / f_raw).astype(np.complex64)
    return out, present


def sft_case(seed=81, t_sft=300.0, n_sft=40, f_raw=256.0, dt=2.0, f_het=30007.0 / 300.0, ndet=2,
             rho=20.0, drop_p=0.15, ntmpl=3, binary=False, noise=True):
    """A search whose input comes as SFTs: per detector make_sfts output, and a
    Dataset with everything but the series (x and valid are None: steps
    (i)-(ii) fill them).  Band of K = t_sft / dt bins centred on f_het (f_het
    t_sft an integer; the default puts f_het dt off whole and half cycles);
    one injection at rho over the SFT span."""
    K = int(round(t_sft / dt))
    kc = int(round(f_het * t_sft))
    assert abs(kc - f_het * t_sft) < 1e-6 and K % 2 == 0
    f_het = kc / t_sft
    k0 = kc - K // 2
    ss = np.random.SeedSequence(seed)
    s_par, s_sft = ss.spawn(2)
    rng = np.random.default_rng(s_par)
    n = n_sft * K
    dets = [make_detector(site, 0.0, n, 1.0, name=f"{site}{i}")
            for i, site in enumerate(["H", "L", "H", "L"][:ndet])]
    inj = dict(alpha=float(rng.uniform(0, 2 * math.pi)), delta=float(rng.uniform(-1.2, 1.2)),
               f=f_het + float(rng.uniform(-0.15, 0.15)) / dt,
               f1dot=float(rng.uniform(-1e-9, 1e-9)), cosi=float(rng.uniform(-1, 1)),
               psi=float(rng.uniform(-0.7, 0.7)), phi0=float(rng.uniform(0, 6.28)), rho=rho)
    if binary:
        inj.update(asini=float(rng.uniform(0.05, 0.3)), porb=float(rng.uniform(0.2, 1.0)) * DAY,
                   tp=float(rng.uniform(0, 1e4)))
    # h0 for the target rho, from the heterodyned signal on the output grid
    # (all SFTs present)
    rho2 = 0.0
    for det in dets:
        t = det.t0 + dt * np.arange(n)
        rho2 += 2.0 * np.sum(np.abs(signal_series(EPHEM_MODEL, det, t, inj, f_het, 0.0)) ** 2)
    inj["h0"] = rho / math.sqrt(rho2)
    inj["rho2"] = rho * rho
    seeds = s_sft.spawn(ndet)
    sfts = [make_sfts(det, 0.0, t_sft, n_sft, f_raw, k0, K, [inj], f_het, 0.0, seeds[i],
                      drop_p=drop_p, noise=noise) for i, det in enumerate(dets)]
    tm = np.zeros((ntmpl, 8))
    tm[:, 0] = inj["alpha"] + 0.01 * np.arange(ntmpl)
    tm[:, 1] = inj["delta"]
    tm[:, 3] = inj["f1dot"]
    tm[:, 6] = 1.0
    if binary:
        tm[:, 5], tm[:, 6], tm[:, 7] = inj["asini"], inj["porb"], inj["tp"]
    n_fft = 1 << int(math.ceil(math.log2(n + 1024)))
    ds = Dataset("sft", dt, f_het, 0.0, grid_origin(0.0, dt, 512.0 + inj.get("asini", 0.0)),
                 n_fft, 8, 0, n_fft, dets, None, None, tm, injections=[inj])
    ds = finish(ds)
    ds.sft = dict(t_start=0.0, t_sft=t_sft, k0=k0, K=K, f_raw=f_raw)
    return ds, sfts


CONFIGS = {
    "tiny": config_tiny,
    "sky_spindown": config_sky_spindown,
    "binary": config_binary,
    "refine": config_refine,
}
